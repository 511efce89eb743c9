"""Python binding of liblt (include/lt.h): argument marshalling only.

Every step of the pipeline runs in the HIP library; this module only passes device
pointers, shapes and the current torch stream across the C ABI.  PyTorch is used
for device memory and streams.  If the built library is missing the binding raises
at load time -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_liblt.so")

LT_U16, LT_I32, LT_U32 = 1, 2, 3
_DTYPES = {torch.uint16: LT_U16, torch.int32: LT_I32, torch.uint32: LT_U32}

_lib = None


class LTError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"liblt status {status}: {message}")
        self.status = status


class _KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("total_ms", ctypes.c_double),
                ("launches", ctypes.c_uint64)]


class _Measures(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in (
        "volume", "shell_count", "max_lt_sq", "mean_lt", "shell_mean_lt", "sphericity",
        "roundness", "hist32")]


class _Volume(ctypes.Structure):
    _fields_ = [("labels", ctypes.c_void_p), ("ndim", ctypes.c_int), ("shape", ctypes.c_int64 * 3),
                ("max_label", ctypes.c_uint32), ("dist_sq", ctypes.c_void_p), ("lt_sq", ctypes.c_void_p),
                ("measures", _Measures)]


class _Tuning(ctypes.Structure):
    _fields_ = [("paint_tile_rows", ctypes.c_int), ("paint_blocks_per_cu", ctypes.c_int),
                ("front_chunk", ctypes.c_int), ("batch_lanes", ctypes.c_int)]


def load():
    """Load the built HIP library (fails loudly if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"liblt is not built ({LIB_PATH} missing); run "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, U32, V = ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.lt_ctx_create.argtypes = [ctypes.POINTER(P), I]
    lib.lt_ctx_destroy.argtypes = [P]
    lib.lt_edt.argtypes = [P, P, I, I, i64p, P, V]
    lib.lt_thickness.argtypes = [P, P, I, I, i64p, P, U32, P, V]
    lib.lt_object_measures.argtypes = [P, P, I, I, i64p, P, U32, ctypes.POINTER(_Measures), V]
    lib.lt_pipeline.argtypes = [P, P, I, I, i64p, U32, P, P, ctypes.POINTER(_Measures), V]
    lib.lt_pipeline_static.argtypes = [P, P, I, I, i64p, U32, P, P, ctypes.POINTER(_Measures), V]
    lib.lt_pipeline_static_bytes.argtypes = [I, i64p, U32]
    lib.lt_pipeline_static_bytes.restype = ctypes.c_size_t
    lib.lt_closed_forms.argtypes = [P, P, P, P, P, U32, I, P, P, P, P, V]
    lib.lt_mesh_measures.argtypes = [P, P, I, I, i64p, U32, P, P, P, V]
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.lt_edt_aniso.argtypes = [P, P, I, I, i64p, i32p, P, V]
    lib.lt_thickness_aniso.argtypes = [P, P, I, I, i64p, i32p, P, U32, P, V]
    lib.lt_object_measures_aniso.argtypes = [P, P, I, I, i64p, i32p, P, U32, ctypes.POINTER(_Measures), V]
    lib.lt_pipeline_aniso.argtypes = [P, P, I, I, i64p, i32p, U32, P, P, ctypes.POINTER(_Measures), V]
    lib.lt_filtered_roundness.argtypes = [P, P, I, I, i64p, P, P, U32, I, P, V]
    lib.lt_remap_roundness.argtypes = [P, P, U32, ctypes.c_float, P, V]
    lib.lt_sync_status.argtypes = [P, V]
    lib.lt_ctx_info.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(I)]
    lib.lt_profile_enable.argtypes = [P, I]
    lib.lt_batch_create.argtypes = [P, ctypes.POINTER(_Volume), I, I, ctypes.POINTER(P)]
    lib.lt_batch_run.argtypes = [P, V]
    lib.lt_batch_destroy.argtypes = [P]
    lib.lt_batch_status.argtypes = [P, V, ctypes.POINTER(ctypes.c_int32)]
    lib.lt_get_tuning.argtypes = [P, ctypes.POINTER(_Tuning)]
    lib.lt_set_tuning.argtypes = [P, ctypes.POINTER(_Tuning)]
    lib.lt_autotune.argtypes = [P, P, I, I, i64p, U32, ctypes.c_char_p, I, ctypes.POINTER(_Tuning)]
    lib.lt_autotune_batch.argtypes = [P, ctypes.POINTER(_Volume), I, I, ctypes.c_char_p, I,
                                      ctypes.POINTER(_Tuning)]
    lib.lt_profile_read.argtypes = [P, ctypes.POINTER(_KernelTime), I, ctypes.POINTER(I)]
    lib.lt_profile_reset.argtypes = [P]
    lib.lt_status_str.argtypes = [I]
    lib.lt_status_str.restype = ctypes.c_char_p
    lib.lt_last_error.restype = ctypes.c_char_p
    lib.lt_version.restype = ctypes.c_char_p
    for f in ("lt_ctx_create", "lt_ctx_destroy", "lt_edt", "lt_thickness", "lt_object_measures", "lt_pipeline",
              "lt_pipeline_static", "lt_mesh_measures", "lt_edt_aniso", "lt_thickness_aniso",
              "lt_object_measures_aniso", "lt_pipeline_aniso", "lt_filtered_roundness", "lt_remap_roundness",
              "lt_closed_forms", "lt_sync_status", "lt_profile_enable", "lt_profile_read",
              "lt_profile_reset", "lt_ctx_info", "lt_batch_create", "lt_batch_run", "lt_batch_status",
              "lt_batch_destroy", "lt_get_tuning", "lt_set_tuning", "lt_autotune",
              "lt_autotune_batch"):
        getattr(lib, f).restype = I
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        lib = load()
        raise LTError(status, f"{lib.lt_status_str(status).decode()}: {lib.lt_last_error().decode()}")


def _shape(t: torch.Tensor):
    arr = (ctypes.c_int64 * t.dim())(*t.shape)
    return arr


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _labels(labels: torch.Tensor):
    if labels.dtype not in _DTYPES:
        raise TypeError(f"labels must be uint16, int32 or uint32 (got {labels.dtype})")
    if labels.dim() not in (2, 3):
        raise ValueError("labels must be 2D or 3D")
    if not labels.is_cuda:
        raise ValueError("labels must be a device tensor")
    return labels.contiguous(), _DTYPES[labels.dtype]


class Context:
    """Owns a liblt context (scratch memory, tables, error word) on one device."""

    def __init__(self, device: int | None = None):
        self._lib = load()
        self.device = torch.cuda.current_device() if device is None else int(device)
        h = ctypes.c_void_p()
        _check(self._lib.lt_ctx_create(ctypes.byref(h), self.device))
        self._h = h

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lt_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync_status(self, stream=None):
        _check(self._lib.lt_sync_status(self._h, _stream(stream)))

    def info(self) -> dict:
        cu, tr = ctypes.c_int(0), ctypes.c_int(0)
        lds = ctypes.c_uint64(0)
        _check(self._lib.lt_ctx_info(self._h, ctypes.byref(cu), ctypes.byref(lds), ctypes.byref(tr)))
        return {"n_cu": cu.value, "lds_per_block": lds.value, "paint_tile_rows": tr.value}

    def get_tuning(self) -> dict:
        t = _Tuning()
        _check(self._lib.lt_get_tuning(self._h, ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in _Tuning._fields_}

    def set_tuning(self, **kw):
        cur = self.get_tuning()
        cur.update(kw)
        t = _Tuning(**cur)
        _check(self._lib.lt_set_tuning(self._h, ctypes.byref(t)))

    def autotune(self, labels: torch.Tensor, max_label: int, cache_path: str | None = None,
                 repeats: int = 3) -> dict:
        lab, dt = _labels(labels)
        t = _Tuning()
        _check(self._lib.lt_autotune(self._h, _ptr(lab), dt, lab.dim(), _shape(lab), int(max_label),
                                     cache_path.encode() if cache_path else None, repeats,
                                     ctypes.byref(t)))
        return {k: getattr(t, k) for k, _ in _Tuning._fields_}

    def profile(self, on: bool = True):
        _check(self._lib.lt_profile_enable(self._h, 1 if on else 0))

    def profile_reset(self):
        _check(self._lib.lt_profile_reset(self._h))

    def profile_read(self) -> dict:
        """{kernel name: (total ms, launches)} accumulated since the last reset."""
        cap = 64
        arr = (_KernelTime * cap)()
        n = ctypes.c_int(0)
        _check(self._lib.lt_profile_read(self._h, arr, cap, ctypes.byref(n)))
        return {arr[i].name.decode(): (arr[i].total_ms, int(arr[i].launches))
                for i in range(min(n.value, cap))}


_default_ctx: dict[int, Context] = {}


def default_context() -> Context:
    dev = torch.cuda.current_device()
    if dev not in _default_ctx:
        _default_ctx[dev] = Context(dev)
    return _default_ctx[dev]


def edt(labels: torch.Tensor, out: torch.Tensor | None = None, ctx: Context | None = None,
        stream=None) -> torch.Tensor:
    """Per-label squared EDT (int32), see lt_edt."""
    lab, dt = _labels(labels)
    ctx = ctx or default_context()
    out = out if out is not None else torch.empty(lab.shape, dtype=torch.int32, device=lab.device)
    _check(ctx._lib.lt_edt(ctx.handle, _ptr(lab), dt, lab.dim(), _shape(lab), _ptr(out), _stream(stream)))
    return out


def thickness(labels: torch.Tensor, dist_sq: torch.Tensor, max_label: int,
              out: torch.Tensor | None = None, ctx: Context | None = None, stream=None) -> torch.Tensor:
    """Squared local thickness (int32), see lt_thickness."""
    lab, dt = _labels(labels)
    ctx = ctx or default_context()
    out = out if out is not None else torch.empty(lab.shape, dtype=torch.int32, device=lab.device)
    _check(ctx._lib.lt_thickness(ctx.handle, _ptr(lab), dt, lab.dim(), _shape(lab),
                                 _ptr(dist_sq.contiguous()), int(max_label), _ptr(out), _stream(stream)))
    return out


@dataclass
class Measures:
    volume: torch.Tensor
    shell_count: torch.Tensor
    max_lt_sq: torch.Tensor
    mean_lt: torch.Tensor
    shell_mean_lt: torch.Tensor
    sphericity: torch.Tensor
    roundness: torch.Tensor
    hist32: torch.Tensor | None = None


def alloc_measures(n: int, device, hist: bool = False) -> Measures:
    f = dict(device=device)
    return Measures(
        volume=torch.empty(n, dtype=torch.uint64, **f),
        shell_count=torch.empty(n, dtype=torch.uint64, **f),
        max_lt_sq=torch.empty(n, dtype=torch.int32, **f),
        mean_lt=torch.empty(n, dtype=torch.float32, **f),
        shell_mean_lt=torch.empty(n, dtype=torch.float32, **f),
        sphericity=torch.empty(n, dtype=torch.float32, **f),
        roundness=torch.empty(n, dtype=torch.float32, **f),
        hist32=torch.empty((n, 32), dtype=torch.float32, **f) if hist else None)


def object_measures(labels: torch.Tensor, lt_sq: torch.Tensor, max_label: int, hist: bool = False,
                    out: Measures | None = None, ctx: Context | None = None, stream=None) -> Measures:
    """Per-object measures (arrays indexed by label 0..max_label), see lt_object_measures."""
    lab, dt = _labels(labels)
    ctx = ctx or default_context()
    out = out or alloc_measures(int(max_label) + 1, lab.device, hist)
    m = _Measures(*[_ptr(getattr(out, k)).value for k in (
        "volume", "shell_count", "max_lt_sq", "mean_lt", "shell_mean_lt", "sphericity", "roundness",
        "hist32")])
    _check(ctx._lib.lt_object_measures(ctx.handle, _ptr(lab), dt, lab.dim(), _shape(lab),
                                       _ptr(lt_sq.contiguous()), int(max_label), ctypes.byref(m),
                                       _stream(stream)))
    return out


def closed_forms(volume, sum_lt_q23, max_lt_sq, shell_count, shell_sum_q23, ndim: int,
                 stream=None):
    """Closed forms from per-object sums (device tensors), see lt_closed_forms."""
    lib = load()
    n = volume.numel()
    dev = volume.device
    outs = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(4)]
    _check(lib.lt_closed_forms(_ptr(volume), _ptr(sum_lt_q23), _ptr(max_lt_sq), _ptr(shell_count),
                               _ptr(shell_sum_q23), n, ndim, *[_ptr(o) for o in outs], _stream(stream)))
    return dict(zip(("mean_lt", "shell_mean_lt", "sphericity", "roundness"), outs))


def pipeline(labels: torch.Tensor, max_label: int, hist: bool = False, out=None, ctx: Context | None = None,
             stream=None):
    """Whole path in one call (lt_pipeline): (dist_sq, lt_sq, Measures).  `out` may
    hold preallocated (dist_sq, lt_sq, Measures)."""
    lab, dt = _labels(labels)
    ctx = ctx or default_context()
    if out is None:
        d = torch.empty(lab.shape, dtype=torch.int32, device=lab.device)
        t = torch.empty(lab.shape, dtype=torch.int32, device=lab.device)
        m = alloc_measures(int(max_label) + 1, lab.device, hist)
    else:
        d, t, m = out
    ms = _measures_struct(m)
    _check(ctx._lib.lt_pipeline(ctx.handle, _ptr(lab), dt, lab.dim(), _shape(lab), int(max_label), _ptr(d),
                                _ptr(t), ctypes.byref(ms), _stream(stream)))
    return d, t, m


STATIC_SCRATCH_BYTES = 64 * 1024 * 1024


def pipeline_static_bytes(shape, max_label: int) -> int:
    """Scratch bytes lt_pipeline_static needs (0 for an invalid shape)."""
    arr = (ctypes.c_int64 * len(shape))(*shape)
    return int(load().lt_pipeline_static_bytes(len(shape), arr, int(max_label)))


def pipeline_static(labels: torch.Tensor, max_label: int, out, ctx: Context | None = None, stream=None):
    """lt_pipeline_static: the whole path with the library's fixed scratch (no device
    allocation inside the call).  `out` = preallocated (dist_sq, lt_sq, Measures)."""
    lab, dt = _labels(labels)
    ctx = ctx or default_context()
    d, t, m = out
    ms = _measures_struct(m)
    _check(ctx._lib.lt_pipeline_static(ctx.handle, _ptr(lab), dt, lab.dim(), _shape(lab), int(max_label),
                                       _ptr(d), _ptr(t), ctypes.byref(ms), _stream(stream)))
    return d, t, m


def measure(labels: torch.Tensor, max_label: int, hist: bool = False, ctx: Context | None = None,
            stream=None):
    """Whole pipeline as three calls: (dist_sq, lt_sq, Measures)."""
    ctx = ctx or default_context()
    d = edt(labels, ctx=ctx, stream=stream)
    t = thickness(labels, d, max_label, ctx=ctx, stream=stream)
    m = object_measures(labels, t, max_label, hist=hist, ctx=ctx, stream=stream)
    return d, t, m


def mesh_measures(labels: torch.Tensor, max_label: int, ctx: Context | None = None, stream=None) -> dict:
    """Per-object voxel count, mesh area (3D marching tetrahedra) or contour length
    (2D marching squares) and mesh sphericity, see lt_mesh_measures."""
    lab, dt = _labels(labels)
    ctx = ctx or default_context()
    n = int(max_label) + 1
    out = dict(volume=torch.empty(n, dtype=torch.uint64, device=lab.device),
               area=torch.empty(n, dtype=torch.float32, device=lab.device),
               sphericity=torch.empty(n, dtype=torch.float32, device=lab.device))
    _check(ctx._lib.lt_mesh_measures(ctx.handle, _ptr(lab), dt, lab.dim(), _shape(lab), int(max_label),
                                     _ptr(out["volume"]), _ptr(out["area"]), _ptr(out["sphericity"]),
                                     _stream(stream)))
    return out


def filtered_roundness(labels: torch.Tensor, dist_sq: torch.Tensor, lt_sq: torch.Tensor, max_label: int,
                       half_width: int, out: torch.Tensor | None = None, ctx: Context | None = None,
                       stream=None) -> torch.Tensor:
    """Per-object roundness from the filtered shell local thickness (float32,
    indexed by label), see lt_filtered_roundness."""
    lab, dt = _labels(labels)
    ctx = ctx or default_context()
    out = out if out is not None else torch.empty(int(max_label) + 1, dtype=torch.float32, device=lab.device)
    _check(ctx._lib.lt_filtered_roundness(ctx.handle, _ptr(lab), dt, lab.dim(), _shape(lab),
                                          _ptr(dist_sq.contiguous()), _ptr(lt_sq.contiguous()), int(max_label),
                                          int(half_width), _ptr(out), _stream(stream)))
    return out


def remap_roundness(roundness: torch.Tensor, r_min: float | None = None, out: torch.Tensor | None = None,
                    ctx: Context | None = None, stream=None) -> torch.Tensor:
    """(R - m) / (1 - m) with m = r_min or the smallest finite R, see lt_remap_roundness."""
    ctx = ctx or default_context()
    r = roundness.contiguous()
    if r.dtype != torch.float32 or not r.is_cuda:
        raise TypeError("roundness must be a float32 device tensor")
    out = out if out is not None else torch.empty_like(r)
    m = float("nan") if r_min is None else float(r_min)
    _check(ctx._lib.lt_remap_roundness(ctx.handle, _ptr(r), r.numel(), ctypes.c_float(m), _ptr(out),
                                       _stream(stream)))
    return out


def _spacing(sq_spacing, ndim: int):
    w = [int(v) for v in sq_spacing]
    if len(w) != ndim:
        raise ValueError(f"sq_spacing needs {ndim} entries (got {len(w)})")
    return (ctypes.c_int32 * ndim)(*w)


def measure_aniso(labels: torch.Tensor, max_label: int, sq_spacing, ctx: Context | None = None, stream=None):
    """Anisotropic spacing, three calls (lt_edt_aniso, lt_thickness_aniso,
    lt_object_measures_aniso): (dist_sq, lt_sq, Measures)."""
    lab, dt = _labels(labels)
    ctx = ctx or default_context()
    w = _spacing(sq_spacing, lab.dim())
    d = torch.empty(lab.shape, dtype=torch.int32, device=lab.device)
    t = torch.empty(lab.shape, dtype=torch.int32, device=lab.device)
    m = alloc_measures(int(max_label) + 1, lab.device)
    _check(ctx._lib.lt_edt_aniso(ctx.handle, _ptr(lab), dt, lab.dim(), _shape(lab), w, _ptr(d), _stream(stream)))
    _check(ctx._lib.lt_thickness_aniso(ctx.handle, _ptr(lab), dt, lab.dim(), _shape(lab), w, _ptr(d),
                                       int(max_label), _ptr(t), _stream(stream)))
    ms = _measures_struct(m)
    _check(ctx._lib.lt_object_measures_aniso(ctx.handle, _ptr(lab), dt, lab.dim(), _shape(lab), w, _ptr(t),
                                             int(max_label), ctypes.byref(ms), _stream(stream)))
    return d, t, m


def pipeline_aniso(labels: torch.Tensor, max_label: int, sq_spacing, out=None, ctx: Context | None = None,
                   stream=None):
    """Anisotropic spacing in one call (lt_pipeline_aniso): (dist_sq, lt_sq, Measures)."""
    lab, dt = _labels(labels)
    ctx = ctx or default_context()
    w = _spacing(sq_spacing, lab.dim())
    if out is None:
        d = torch.empty(lab.shape, dtype=torch.int32, device=lab.device)
        t = torch.empty(lab.shape, dtype=torch.int32, device=lab.device)
        m = alloc_measures(int(max_label) + 1, lab.device)
    else:
        d, t, m = out
    ms = _measures_struct(m)
    _check(ctx._lib.lt_pipeline_aniso(ctx.handle, _ptr(lab), dt, lab.dim(), _shape(lab), w, int(max_label),
                                      _ptr(d), _ptr(t), ctypes.byref(ms), _stream(stream)))
    return d, t, m


def version() -> str:
    return load().lt_version().decode()


def _measures_struct(m: Measures) -> _Measures:
    return _Measures(*[_ptr(getattr(m, k)).value for k in (
        "volume", "shell_count", "max_lt_sq", "mean_lt", "shell_mean_lt", "sphericity", "roundness",
        "hist32")])


class Batch:
    """Many volumes (one label dtype) captured into one graph; see lt_batch_create.

    ``volumes`` is a list of (labels, max_label).  Outputs are allocated here and
    exposed as ``outputs[i] = (dist_sq, lt_sq, Measures)``; they keep their
    addresses for the life of the batch, so every run() rewrites them in place."""

    def __init__(self, volumes, ctx: Context | None = None, autotune_cache: str | None = None,
                 autotune_repeats: int = 0):
        self.ctx = ctx or default_context()
        self._lib = load()
        self.labels = []
        self.outputs = []
        arr = (_Volume * len(volumes))()
        dts = set()
        for k, (labels, max_label) in enumerate(volumes):
            lab, dt = _labels(labels)
            dts.add(dt)
            d = torch.empty(lab.shape, dtype=torch.int32, device=lab.device)
            t = torch.empty(lab.shape, dtype=torch.int32, device=lab.device)
            m = alloc_measures(int(max_label) + 1, lab.device)
            self.labels.append(lab)
            self.outputs.append((d, t, m))
            shape = list(lab.shape) + [0] * (3 - lab.dim())
            arr[k] = _Volume(_ptr(lab).value, lab.dim(), (ctypes.c_int64 * 3)(*shape), int(max_label),
                             _ptr(d).value, _ptr(t).value, _measures_struct(m))
        if len(dts) > 1:
            raise TypeError("all volumes of a batch must share one label dtype")
        self.dtype = dts.pop() if dts else LT_U16
        self._vols = arr
        if autotune_repeats > 0:
            tt = _Tuning()
            _check(self._lib.lt_autotune_batch(self.ctx.handle, arr, len(volumes), self.dtype,
                                               autotune_cache.encode() if autotune_cache else None,
                                               autotune_repeats, ctypes.byref(tt)))
        h = ctypes.c_void_p()
        _check(self._lib.lt_batch_create(self.ctx.handle, arr, len(volumes), self.dtype, ctypes.byref(h)))
        self._h = h

    def run(self, stream=None):
        _check(self._lib.lt_batch_run(self._h, _stream(stream)))

    def status(self, stream=None) -> list[int]:
        """Per-volume statuses of the replays so far (0 = ok, 6 = label out of range,
        7 = overflow), read and cleared; see lt_batch_status."""
        arr = (ctypes.c_int32 * len(self.outputs))()
        self._lib.lt_batch_status(self._h, _stream(stream), arr)
        return list(arr)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- learned correction

N_FEATURES = 34


def _mlp_lib():
    lib = load()
    if not getattr(lib, "_mlp_bound", False):
        P, I, V = ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p
        f = ctypes.c_float
        lib.lt_mlp_create.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(P)]
        lib.lt_mlp_destroy.argtypes = [P]
        lib.lt_mlp_set_normalization.argtypes = [P, P, P, f, f]
        lib.lt_mlp_set_guard.argtypes = [P, P, P, f]
        lib.lt_mlp_train_step.argtypes = [P, P, P, I, f, f, P, V]
        lib.lt_mlp_infer.argtypes = [P, P, I, P, V]
        lib.lt_mlp_features.argtypes = [P, P, P, P, ctypes.c_uint32, P, V]
        lib.lt_mlp_correct.argtypes = [P, P, P, I, P, P, P, V]
        lib.lt_mlp_state_size.restype = ctypes.c_size_t
        lib.lt_mlp_get_state.argtypes = [P, P, ctypes.c_size_t]
        lib.lt_mlp_set_state.argtypes = [P, P, ctypes.c_size_t]
        lib.lt_mlp_buffers.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(I)]
        lib.lt_bf16_gemm.argtypes = [I, I, I, P, I, I, P, I, I, P, I, V]
        lib.lt_mlp_read.argtypes = [P, I, P, ctypes.c_size_t]
        for name in ("lt_mlp_create", "lt_mlp_destroy", "lt_mlp_set_normalization", "lt_mlp_set_guard",
                     "lt_mlp_train_step", "lt_mlp_infer", "lt_mlp_features", "lt_mlp_correct",
                     "lt_mlp_get_state", "lt_mlp_set_state", "lt_mlp_buffers", "lt_bf16_gemm", "lt_mlp_read"):
            getattr(lib, name).restype = I
        lib._mlp_bound = True
    return lib


def _host_f32(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def bf16_gemm(A: torch.Tensor, B: torch.Tensor, trans_a: bool = False, trans_b: bool = False,
              stream=None) -> torch.Tensor:
    """C = op(A) op(B) for bfloat16 device matrices with the library's MFMA kernel."""
    lib = _mlp_lib()
    assert A.dtype == torch.bfloat16 and B.dtype == torch.bfloat16
    A, B = A.contiguous(), B.contiguous()
    M, K = (A.shape[1], A.shape[0]) if trans_a else A.shape
    K2, N = (B.shape[1], B.shape[0]) if trans_b else B.shape
    assert K == K2
    C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    _check(lib.lt_bf16_gemm(M, N, K, _ptr(A), A.shape[1], int(trans_a), _ptr(B), B.shape[1], int(trans_b),
                            _ptr(C), N, _stream(stream)))
    return C


class MLP:
    """Sphericity-correction network (see the lt_mlp_* declarations in lt.h)."""

    def __init__(self, seed: int = 0, ctx: Context | None = None):
        self.ctx = ctx or default_context()
        self._lib = _mlp_lib()
        h = ctypes.c_void_p()
        _check(self._lib.lt_mlp_create(self.ctx.handle, int(seed), ctypes.byref(h)))
        self._h = h
        self._loss = torch.zeros(1, dtype=torch.float32, device=f"cuda:{self.ctx.device}")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lt_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_normalization(self, mean, std, target_shift: float, target_scale: float):
        m, mp = _host_f32(mean)
        s, sp = _host_f32(std)
        _check(self._lib.lt_mlp_set_normalization(self._h, mp, sp, float(target_shift), float(target_scale)))

    def set_guard(self, fmin, fmax, max_abs_delta: float):
        a, ap = _host_f32(fmin)
        b, bp = _host_f32(fmax)
        _check(self._lib.lt_mlp_set_guard(self._h, ap, bp, float(max_abs_delta)))

    def train_step(self, x: torch.Tensor, y: torch.Tensor, lr: float, weight_decay: float = 0.0,
                   stream=None) -> torch.Tensor:
        """One AdamW step; returns the (device) sum of squared errors."""
        x, y = x.contiguous(), y.contiguous()
        _check(self._lib.lt_mlp_train_step(self._h, _ptr(x), _ptr(y), x.shape[0], float(lr),
                                           float(weight_decay), _ptr(self._loss), _stream(stream)))
        return self._loss

    def infer(self, x: torch.Tensor, stream=None) -> torch.Tensor:
        x = x.contiguous()
        out = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        _check(self._lib.lt_mlp_infer(self._h, _ptr(x), x.shape[0], _ptr(out), _stream(stream)))
        return out

    def correct(self, x: torch.Tensor, s_lt: torch.Tensor, stream=None):
        """(s_corr, n_fallback) with the guard applied."""
        x, s_lt = x.contiguous(), s_lt.contiguous()
        n = x.shape[0]
        delta = torch.empty(n, dtype=torch.float32, device=x.device)
        out = torch.empty(n, dtype=torch.float32, device=x.device)
        nf = torch.zeros(1, dtype=torch.int32, device=x.device)
        _check(self._lib.lt_mlp_correct(self._h, _ptr(x), _ptr(s_lt), n, _ptr(delta), _ptr(out), _ptr(nf),
                                        _stream(stream)))
        return out, nf

    def buffers(self):
        w, g, n = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_int(0)
        _check(self._lib.lt_mlp_buffers(self._h, ctypes.byref(w), ctypes.byref(g), ctypes.byref(n)))
        return w.value, g.value, n.value

    def _read(self, which: int):
        import numpy as np
        _, _, n = self.buffers()
        out = np.empty(n, dtype=np.float32)
        _check(self._lib.lt_mlp_read(self._h, which, out.ctypes.data_as(ctypes.c_void_p), n))
        return out

    def params(self):
        """FP32 master weights (packed layout), host copy."""
        return self._read(0)

    def grads(self):
        """Gradients of the last step (packed layout), host copy."""
        return self._read(1)

    def moments(self):
        """AdamW first and second moments, host copies."""
        return self._read(2), self._read(3)

    def get_state(self) -> bytes:
        size = self._lib.lt_mlp_state_size()
        buf = ctypes.create_string_buffer(size)
        _check(self._lib.lt_mlp_get_state(self._h, buf, size))
        return buf.raw

    def set_state(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(self._lib.lt_mlp_set_state(self._h, buf, len(blob)))


def mlp_features(m: Measures, ctx: Context | None = None, stream=None) -> torch.Tensor:
    """Per-object network features (max_label + 1 rows x 34) from measures with hist32."""
    assert m.hist32 is not None, "object_measures(..., hist=True) is needed for the features"
    ctx = ctx or default_context()
    n = m.volume.numel()
    x = torch.empty((n, N_FEATURES), dtype=torch.float32, device=m.volume.device)
    _check(_mlp_lib().lt_mlp_features(ctx.handle, _ptr(m.hist32), _ptr(m.volume), _ptr(m.mean_lt), n,
                                      _ptr(x), _stream(stream)))
    return x
