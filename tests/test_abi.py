"""C-ABI checks that need no GPU: the library loads, exports every symbol the
public header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2504_05808_amd import lt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lt.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lt_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = lt.load()
    names = _declared_functions()
    assert "lt_edt" in names and "lt_thickness" in names and "lt_object_measures" in names
    for name in names:
        assert hasattr(lib, name), f"{name} declared in lt.h but not exported"


def test_status_strings_and_version():
    lib = lt.load()
    assert lib.lt_status_str(0) == b"ok"
    assert lib.lt_status_str(6) == b"label out of range"
    assert lib.lt_status_str(99) == b"unknown status"
    assert b"gfx950" in lib.lt_version()


def test_null_context_rejected():
    lib = lt.load()
    shape = (ctypes.c_int64 * 3)(4, 4, 4)
    assert lib.lt_edt(None, ctypes.c_void_p(8), lt.LT_U16, 3, shape, ctypes.c_void_p(8), None) == 1
    assert lib.lt_thickness(None, None, lt.LT_U16, 3, shape, None, 5, None, None) == 1
    assert lib.lt_sync_status(None, None) == 1
    assert lib.lt_pipeline(None, ctypes.c_void_p(8), lt.LT_U16, 3, shape, 5, None, None, None, None) == 1
    assert b"ctx" in lib.lt_last_error()


def test_argument_errors_before_device_use():
    """dtype and shape are validated before the context is dereferenced."""
    lib = lt.load()
    fake = ctypes.create_string_buffer(64)      # never dereferenced on these paths
    ctx = ctypes.cast(fake, ctypes.c_void_p)
    ok3 = (ctypes.c_int64 * 3)(4, 4, 4)
    assert lib.lt_edt(ctx, ctypes.c_void_p(8), 9, 3, ok3, ctypes.c_void_p(8), None) == 2
    bad_nd = (ctypes.c_int64 * 4)(2, 2, 2, 2)
    assert lib.lt_edt(ctx, ctypes.c_void_p(8), lt.LT_U16, 4, bad_nd, ctypes.c_void_p(8), None) == 3
    neg = (ctypes.c_int64 * 3)(4, -1, 4)
    assert lib.lt_edt(ctx, ctypes.c_void_p(8), lt.LT_U16, 3, neg, ctypes.c_void_p(8), None) == 3
    big3 = (ctypes.c_int64 * 3)(1025, 8, 8)
    assert lib.lt_edt(ctx, ctypes.c_void_p(8), lt.LT_I32, 3, big3, ctypes.c_void_p(8), None) == 3
    big2 = (ctypes.c_int64 * 2)(8, 2049)
    assert lib.lt_edt(ctx, ctypes.c_void_p(8), lt.LT_I32, 2, big2, ctypes.c_void_p(8), None) == 3
    assert b"2048" in lib.lt_last_error()
    assert lib.lt_edt(ctx, ctypes.c_void_p(8), lt.LT_U32, 3, None, ctypes.c_void_p(8), None) == 1
    assert lib.lt_closed_forms(None, None, None, None, None, 4, 5, None, None, None, None, None) == 3
    assert lib.lt_closed_forms(None, None, None, None, None, 0, 3, None, None, None, None, None) == 0
    assert lib.lt_closed_forms(None, None, None, None, None, 4, 3, None, None, None, None, None) == 1


def test_binding_rejects_host_and_bad_dtype_tensors():
    torch = pytest.importorskip("torch")
    with pytest.raises(TypeError):
        lt._labels(torch.zeros((4, 4), dtype=torch.float32))
    with pytest.raises(ValueError):
        lt._labels(torch.zeros((4, 4), dtype=torch.int32))


def test_learned_correction_argument_errors():
    """The network and GEMM entry points check arguments before any device call."""
    lib = lt._mlp_lib()
    out = ctypes.c_void_p()
    assert lib.lt_mlp_create(None, 0, ctypes.byref(out)) == 1
    assert lib.lt_mlp_destroy(None) == 0
    assert lib.lt_mlp_train_step(None, None, None, 16, 0.0, 0.0, None, None) == 1
    assert lib.lt_mlp_infer(None, None, 4, None, None) == 1
    assert lib.lt_mlp_read(None, 0, None, 0) == 1
    assert lib.lt_mlp_features(None, None, None, None, 0, None, None) == 1
    assert lib.lt_bf16_gemm(15, 16, 16, None, 16, 0, None, 16, 0, None, 16, None) == 3
    assert lib.lt_bf16_gemm(16, 16, 8, None, 16, 0, None, 16, 0, None, 16, None) == 3
    assert lib.lt_bf16_gemm(0, 16, 16, None, 16, 0, None, 16, 0, None, 16, None) == 0
    assert lib.lt_bf16_gemm(16, 16, 16, None, 16, 0, None, 16, 0, None, 16, None) == 1
    assert lib.lt_mlp_state_size() == (3 * 12496 + 4 * 34 + 3 + 2) * 4


def test_static_pipeline_size_checks_without_device():
    """lt_pipeline_static refuses problems beyond its fixed scratch from the sizes
    alone, before the context is used."""
    lib = lt.load()
    fake = ctypes.create_string_buffer(64)      # never dereferenced on these paths
    ctx = ctypes.cast(fake, ctypes.c_void_p)
    assert lt.pipeline_static_bytes((128, 128, 128), 300) <= lt.STATIC_SCRATCH_BYTES
    assert lt.pipeline_static_bytes((512, 512, 512), 2000) > lt.STATIC_SCRATCH_BYTES
    assert lt.pipeline_static_bytes((1025, 4, 4), 3) == 0
    big = (ctypes.c_int64 * 3)(512, 512, 512)
    assert lib.lt_pipeline_static(ctx, ctypes.c_void_p(8), lt.LT_U16, 3, big, 2000, None, None, None, None) == 8
    assert b"fixed scratch" in lib.lt_last_error()
    assert lib.lt_pipeline_static(None, ctypes.c_void_p(8), lt.LT_U16, 3, big, 2000, None, None, None, None) == 1


def test_mesh_tables_match_the_oracle_per_cell():
    """The library's host-built cell tables (lt_mesh_table) against the mesh oracle
    evaluated on one unit cube / square per inside pattern (no padding, so only that
    cell counts).  Q.32 rounding of the table entries is below 2^-32."""
    from oracle import mesh_area as M
    lib = lt.load()
    lib.lt_mesh_table.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    cube = (ctypes.c_double * 256)()
    assert lib.lt_mesh_table(3, cube) == 0
    for m in range(256):
        mask = np.zeros((2, 2, 2), dtype=bool)
        for k in range(8):
            mask[k >> 2, (k >> 1) & 1, k & 1] = (m >> k) & 1
        assert cube[m] == pytest.approx(M.iso_area(mask, pad=False), abs=2 ** -31), m
    sq = (ctypes.c_double * 16)()
    assert lib.lt_mesh_table(2, sq) == 0
    for m in range(16):
        mask = np.zeros((2, 2), dtype=bool)
        for k in range(4):
            mask[k >> 1, k & 1] = (m >> k) & 1
        assert sq[m] == pytest.approx(M.contour_length(mask, pad=False), abs=2 ** -31), m
    assert lib.lt_mesh_table(4, cube) == 3


def test_filtered_roundness_and_remap_argument_errors():
    """Half-width range, NULL outputs and r_min are checked before any device use."""
    lib = lt.load()
    fake = ctypes.create_string_buffer(64)
    ctx = ctypes.cast(fake, ctypes.c_void_p)
    shape = (ctypes.c_int64 * 3)(4, 4, 4)
    p = ctypes.c_void_p(8)
    f = lib.lt_filtered_roundness
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    assert f(ctx, p, lt.LT_U16, 3, shape, p, p, 5, 17, p, None) == 1
    assert b"half_width" in lib.lt_last_error()
    assert f(ctx, p, lt.LT_U16, 3, shape, p, p, 5, -1, p, None) == 1
    assert f(ctx, p, lt.LT_U16, 3, shape, p, p, 5, 2, None, None) == 1
    assert f(None, p, lt.LT_U16, 3, shape, p, p, 5, 2, p, None) == 1
    r = lib.lt_remap_roundness
    r.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32, ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p]
    assert r(None, p, 4, float("nan"), p, None) == 1
    assert r(ctx, p, 0, float("nan"), p, None) == 0              # nothing to do
    assert r(ctx, None, 4, float("nan"), p, None) == 1
    assert r(ctx, p, 4, float("inf"), p, None) == 1


def test_injected_allocation_failure_on_context_create(monkeypatch):
    """LT_FAULT_INJECT=alloc: a context needs device memory, so lt_ctx_create fails
    with LT_E_ALLOC before touching the device, and leaves *out NULL; without the
    variable the call goes on (LT_OK on a GPU machine, a HIP error without one)."""
    lib = lt.load()
    h = ctypes.c_void_p(123)
    monkeypatch.setenv("LT_FAULT_INJECT", "alloc")
    assert lib.lt_ctx_create(ctypes.byref(h), 0) == 4
    assert h.value is None
    assert b"injected" in lib.lt_last_error()
    monkeypatch.delenv("LT_FAULT_INJECT")
    st = lib.lt_ctx_create(ctypes.byref(h), 0)
    assert st in (0, 5)
    if st == 0:
        lib.lt_ctx_destroy(h)
