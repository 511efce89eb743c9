"""GPU parity of the mesh-based surface measures (lt_mesh_measures) against the
mesh oracle: per label the voxel count (exact), the marching-tetrahedra surface
area (3D) or marching-squares contour length (2D), and the mesh sphericity.

Tolerance: the device sums Q.32 table entries (each rounded by at most 2^-33) and
returns FP32, so area and sphericity are held to 1e-6 relative of the FP64 oracle;
the FP32 output rounding (2^-24) dominates."""
import math
import sys

import numpy as np
import pytest

from oracle import mesh_area as M
from paper_2504_05808_amd import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-6


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_05808_amd import lt
    lt.load()
    return torch, lt


def _note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_mesh(gpu, lab, max_label=None):
    torch, lt = gpu
    max_label = int(lab.max()) if max_label is None else max_label
    t = torch.from_numpy(np.ascontiguousarray(lab)).cuda()
    out = lt.mesh_measures(t, max_label)
    lt.default_context().sync_status()
    return {k: v.cpu().numpy() for k, v in out.items()}


def compare(got, ref):
    n = len(ref["volume"])
    np.testing.assert_array_equal(got["volume"][:n].astype(np.int64), ref["volume"])
    ok = ref["volume"] > 0
    np.testing.assert_array_equal(got["area"][:n][~ok], 0.0)
    assert np.all(np.isnan(got["sphericity"][:n][~ok]))
    np.testing.assert_allclose(got["area"][:n][ok].astype(np.float64), ref["area"][ok], rtol=RTOL, atol=0)
    np.testing.assert_allclose(got["sphericity"][:n][ok].astype(np.float64), ref["sphericity"][ok],
                               rtol=RTOL, atol=0)


SHAPES = [(1, 1), (1, 37), (23, 1), (37, 70), (130, 67), (300, 260), (3, 5, 7), (9, 130, 67),
          (17, 33, 65), (40, 9, 77), (1, 50, 60), (45, 1, 1), (70, 66, 129)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dtype", [np.uint16, np.int32, np.uint32])
def test_random_labels(gpu, shape, dtype):
    """Touching labels, border contact and multi-component labels; several blocks
    along every axis for the larger shapes (64-cube chunks, 4-row blocks)."""
    rng = synth.rng_for(7000 + len(shape) * 100 + shape[-1])
    for blob, nl, pbg in [(1, 3, 0.3), (4, 5, 0.1), (8, 2, 0.0)]:
        lab = synth.random_labels(rng, shape, n_labels=nl, p_bg=pbg, blob=blob, dtype=dtype)
        _note(f"mesh random shape={shape} dtype={np.dtype(dtype).name} blob={blob}")
        compare(run_mesh(gpu, lab), M.mesh_measures(lab))


def test_many_labels_overflow_block_tables(gpu):
    """More labels per block than the block's label table holds (global fallback)."""
    rng = synth.rng_for(7100)
    lab = rng.integers(0, 1500, size=(10, 30, 70)).astype(np.int32)
    _note("mesh 1500 random labels")
    compare(run_mesh(gpu, lab), M.mesh_measures(lab))


def test_single_voxel_and_empty(gpu):
    for shape in [(8, 9), (5, 6, 7)]:
        lab = np.zeros(shape, dtype=np.int32)
        got = run_mesh(gpu, lab, max_label=3)
        assert np.all(got["volume"] == 0) and np.all(got["area"] == 0) and np.all(np.isnan(got["sphericity"]))
        lab.flat[len(lab.flat) // 2] = 2
        got = run_mesh(gpu, lab, max_label=3)
        expect = 1.5 * (1 + math.sqrt(2)) if len(shape) == 3 else 2 * math.sqrt(2)
        assert got["area"][2] == pytest.approx(expect, rel=1e-7)
        compare(got, M.mesh_measures(lab, max_label=3))


def test_full_image_one_label(gpu):
    """The whole image is one object: its surface is the padded border."""
    for shape in [(31, 47), (12, 20, 33), (65, 64, 63)]:
        lab = np.full(shape, 7, dtype=np.uint16)
        compare(run_mesh(gpu, lab), M.mesh_measures(lab))


def test_cfg1_and_cfg2(gpu):
    lab, _ = synth.cfg1()
    _note("mesh cfg1 256x256 int32")
    compare(run_mesh(gpu, lab), M.mesh_measures(lab))
    lab, meta = synth.cfg2()
    _note("mesh cfg2 128^3 int32")
    got = run_mesh(gpu, lab)
    compare(got, M.mesh_measures(lab))
    for o in meta["objects"]:                       # digital balls: S_mesh in the known bias band
        if o["kind"] == "ball":
            assert 0.7 < got["sphericity"][o["label"]] < 0.9


def test_sparse_labels_and_range_error(gpu):
    torch, lt = gpu
    lab = np.zeros((30, 40, 50), dtype=np.uint32)
    lab[2:10, 3:12, 4:20] = 100000
    lab[12:25, 20:35, 10:45] = 7
    compare(run_mesh(gpu, lab, max_label=100001), M.mesh_measures(lab, max_label=100001))
    t = torch.from_numpy(lab).cuda()
    lt.mesh_measures(t, 99999)
    with pytest.raises(lt.LTError) as e:
        lt.default_context().sync_status()
    assert e.value.status == 6


def test_512cube_every_object(gpu):
    """The 512^3 uint16 benchmark volume: every object against the oracle."""
    lab, meta = synth.cfg3()
    _note(f"mesh cfg3 512^3 uint16 objects={meta['n_objects']}")
    got = run_mesh(gpu, lab)
    ref = M.mesh_measures(lab)
    assert int((ref["volume"] > 0).sum()) == meta["n_objects"]
    compare(got, ref)
