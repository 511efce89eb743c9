"""GPU parity: the HIP path through the C ABI against the CPU oracle, in both
forms (lt_edt + lt_thickness + lt_object_measures, and the fused lt_pipeline).

Distances and local thickness are compared bit-exactly (integers); per-object
volume, shell count and max LT exactly; the FP32 measures within 1e-5 relative
of the FP64 oracle (the bound the method's FP32 outputs are held to; fixed-point
radius sums contribute <= 2^-24 absolute per voxel and the FP32 closed forms a
few ulp)."""
import math
import sys

import numpy as np
import pytest

from oracle import lt_oracle as O
from paper_2504_05808_amd import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-5
FLOAT_KEYS = ("mean_lt", "shell_mean_lt", "sphericity", "roundness")


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


def run_gpu(gpu, lab, max_label=None, hist=False, fused=None):
    """The path through the C ABI.  fused=None runs both forms (three calls and the
    one-call lt_pipeline), checks that they agree bit for bit and returns one."""
    if fused is None:
        a = run_gpu(gpu, lab, max_label, hist, fused=False)
        b = run_gpu(gpu, lab, max_label, hist, fused=True)
        for k in a:
            np.testing.assert_array_equal(a[k], b[k], err_msg=f"fused vs separate: {k}")
        return a
    torch, lt = gpu
    max_label = int(lab.max()) if max_label is None else max_label
    t = torch.from_numpy(np.ascontiguousarray(lab)).cuda()
    d, ltsq, m = (lt.pipeline if fused else lt.measure)(t, max_label, hist=hist)
    lt.default_context().sync_status()
    out = dict(dist_sq=d.cpu().numpy().astype(np.int64), lt_sq=ltsq.cpu().numpy().astype(np.int64))
    for k in ("volume", "shell_count", "max_lt_sq"):
        out[k] = getattr(m, k).cpu().numpy().astype(np.int64)
    for k in FLOAT_KEYS:
        out[k] = getattr(m, k).cpu().numpy().astype(np.float64)
    if hist:
        out["hist32"] = m.hist32.cpu().numpy().astype(np.float64)
    return out


def compare(got, ref, lab, fields=True):
    if fields:
        np.testing.assert_array_equal(got["dist_sq"], ref["dist_sq"])
        np.testing.assert_array_equal(got["lt_sq"], ref["lt_sq"])
    n = len(ref["volume"])
    for k in ("volume", "shell_count"):
        np.testing.assert_array_equal(got[k][:n], ref[k])
    np.testing.assert_array_equal(got["max_lt_sq"][:n], ref["max_lt_sq"])
    ok = ref["volume"] > 0
    for k in FLOAT_KEYS:
        g, r = got[k][:n], ref[k]
        assert np.all(np.isnan(g[~ok]))
        okk = ok & ~np.isnan(r)
        np.testing.assert_allclose(g[okk], r[okk], rtol=RTOL, atol=0, err_msg=k)


# ------------------------------------------------------------------ small random

SHAPES = [(1, 1), (1, 37), (23, 1), (37, 70), (130, 67), (65, 129), (3, 5, 7), (9, 130, 67),
          (17, 33, 65), (40, 9, 77), (1, 50, 60), (45, 1, 1)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dtype", [np.uint16, np.int32, np.uint32])
def test_random_labels_bit_exact(gpu, shape, dtype):
    rng = synth.rng_for(1000 + len(shape) * 100 + shape[-1])
    for blob, nl, pbg in [(1, 3, 0.3), (4, 5, 0.1), (8, 2, 0.0)]:
        lab = synth.random_labels(rng, shape, n_labels=nl, p_bg=pbg, blob=blob, dtype=dtype)
        _note(f"random shape={shape} dtype={np.dtype(dtype).name} blob={blob}")
        ref = O.measure(lab, per_object=False)
        got = run_gpu(gpu, lab)
        compare(got, ref, lab)


def test_cfg1_2d_ellipses(gpu):
    lab, meta = synth.cfg1()
    _note("cfg1 256x256 int32")
    ref = O.measure(lab, per_object=False)
    compare(run_gpu(gpu, lab), ref, lab)


def test_cfg2_3d_ellipsoids_and_balls(gpu):
    lab, meta = synth.cfg2()
    _note("cfg2 128^3 int32")
    ref = O.measure(lab)
    got = run_gpu(gpu, lab)
    compare(got, ref, lab)
    for o in meta["objects"]:
        if o["kind"] == "ball":
            l, r = o["label"], o["r"]
            assert np.all(got["lt_sq"][lab == l] == r * r + 1)
            assert got["roundness"][l] == pytest.approx(1.0, abs=1e-6)


# ------------------------------------------------------------------ edge cases

def test_empty_and_single_voxel(gpu):
    for shape in [(8, 9), (5, 6, 7)]:
        lab = np.zeros(shape, dtype=np.int32)
        got = run_gpu(gpu, lab, max_label=3)
        assert np.all(got["dist_sq"] == 0) and np.all(got["lt_sq"] == 0)
        assert np.all(got["volume"] == 0) and np.all(np.isnan(got["sphericity"]))
        lab.flat[len(lab.flat) // 2] = 2
        ref = O.measure(lab, max_label=3, per_object=False)
        compare(run_gpu(gpu, lab, max_label=3), ref, lab)


def test_full_volume_one_label(gpu):
    for shape in [(31, 47), (12, 20, 33)]:
        lab = np.full(shape, 7, dtype=np.uint16)
        ref = O.measure(lab, per_object=False)
        compare(run_gpu(gpu, lab), ref, lab)


def test_large_objects_span_tiles(gpu):
    """Objects wider than one 32x64 paint tile and with large balls."""
    m, _ = synth.disc_mask(60)
    lab = np.zeros((140, 150), dtype=np.int32)
    lab[5:5 + m.shape[0], 10:10 + m.shape[1]][m] = 1
    lab[:, 140:] = 2
    ref = O.measure(lab, per_object=False)
    compare(run_gpu(gpu, lab), ref, lab)
    lab3 = np.zeros((30, 90, 150), dtype=np.int32)
    m3, off = synth.ellipsoid_mask((70.0, 40.0, 12.0), np.eye(3), (0.3, 0.1, 0.2))
    o = np.array([15, 45, 75]) + off
    lab3[o[0]:o[0] + m3.shape[0], o[1]:o[1] + m3.shape[1], o[2]:o[2] + m3.shape[2]][m3] = 1
    lab3[:, 85:, :] = 3
    ref3 = O.measure(lab3)
    compare(run_gpu(gpu, lab3), ref3, lab3)


def _lt_sq_at(lab, D, p, reach):
    """LT^2 at voxel p from the definition: the largest D(c) over centres c of p's
    label whose open ball |q - c|^2 < D(c) contains p."""
    lo = [max(0, p[a] - reach) for a in range(3)]
    hi = [min(lab.shape[a], p[a] + reach + 1) for a in range(3)]
    sub = tuple(slice(lo[a], hi[a]) for a in range(3))
    zz, yy, xx = np.meshgrid(*[np.arange(lo[a], hi[a]) for a in range(3)], indexing="ij")
    d2 = (zz - p[0]) ** 2 + (yy - p[1]) ** 2 + (xx - p[2]) ** 2
    ok = (lab[sub] == lab[p]) & (d2 < D[sub])
    return int(D[sub][ok].max())


def test_thick_cylinder_column_rescans(gpu):
    """A cylinder of radius 34 along z (axis between voxels, end faces on the image
    border): the central columns hold D = 1109 from slice 33 to Z - 34, and each of
    those voxels is a kept centre (its neighbours' balls are no larger), so with reach
    33 the 64-slice chunk [128, 192) of such a column lists 64 + 2 * 33 = 130 > 128
    centres and the paint pass rescans the column there.  D is compared with the
    oracle in full; LT at sampled voxels with its definition (the oracle's full LT
    takes minutes here); volume, shell count and largest LT exactly."""
    Z, Y, X, r = 264, 72, 72, 34
    zz, yy, xx = np.meshgrid(np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    lab = (((yy - 35.5) ** 2 + (xx - 35.5) ** 2) < r * r).astype(np.uint16)
    _note(f"cylinder {lab.shape} r={r}")
    got = run_gpu(gpu, lab)
    D = O.edt_sq(lab).astype(np.int64)
    np.testing.assert_array_equal(got["dist_sq"], D)
    dmax = int(D.max())
    reach = math.isqrt(dmax - 1)
    assert dmax == 1109 and reach == 33
    assert np.count_nonzero(D[128 - reach:192 + reach, 35, 35] == dmax) == 130
    obj = np.argwhere(lab > 0)
    rng = np.random.default_rng(11)
    pick = obj[rng.choice(len(obj), 1500, replace=False)]
    extra = [[z, 35, 35] for z in (0, 1, 33, 63, 64, 127, 128, 160, 191, 192, 230, 263)]
    pick = np.concatenate([pick, extra, [[150, 35, 2], [150, 2, 35], [5, 35, 69]]])
    want = np.array([_lt_sq_at(lab, D, tuple(p), reach) for p in pick])
    np.testing.assert_array_equal(got["lt_sq"][tuple(pick.T)], want)
    assert np.all(got["lt_sq"][lab == 0] == 0)
    assert got["volume"][1] == int(lab.sum())
    assert got["shell_count"][1] == int(O.shell_mask(lab).sum())
    assert got["max_lt_sq"][1] == dmax


def test_sparse_label_values_and_large_max_label(gpu):
    rng = synth.rng_for(77)
    lab = synth.random_labels(rng, (20, 30, 40), n_labels=4, blob=5, dtype=np.uint32)
    lab = np.choose(lab, [0, 5, 60000, 70001, 3]).astype(np.uint32)
    ref = O.measure(lab, max_label=80000, per_object=False)
    compare(run_gpu(gpu, lab, max_label=80000), ref, lab)


def test_histogram_bins(gpu):
    lab, _ = synth.cfg2()
    got = run_gpu(gpu, lab, hist=True)
    ref = O.measure(lab)
    h = O.lt_histogram(lab, ref["lt_sq"], ref["max_lt_sq"])
    ok = ref["volume"] > 0
    np.testing.assert_allclose(got["hist32"][ok], h[ok], rtol=1e-6, atol=1e-7)


def test_label_above_max_label_sets_error(gpu):
    torch, lt = gpu
    lab = np.zeros((8, 8, 8), dtype=np.int32)
    lab[2:5, 2:5, 2:5] = 9
    t = torch.from_numpy(lab).cuda()
    d = lt.edt(t)
    x = lt.thickness(t, d, 4)
    with pytest.raises(lt.LTError) as e:
        lt.default_context().sync_status()
    assert e.value.status == 6
    lt.default_context().sync_status()          # the word was cleared


def test_label_above_max_label_sets_error_in_fused_call(gpu):
    """The fused call finds out-of-range labels while it records the boxes."""
    torch, lt = gpu
    lab = np.zeros((9, 10, 70), dtype=np.uint16)
    lab[2:5, 2:5, 60:68] = 3
    lab[6, 7, 1:4] = 11
    t = torch.from_numpy(lab).cuda()
    lt.pipeline(t, 4)
    with pytest.raises(lt.LTError) as e:
        lt.default_context().sync_status()
    assert e.value.status == 6
    lt.default_context().sync_status()


def test_deterministic_repeat(gpu):
    lab, _ = synth.cfg2()
    a = run_gpu(gpu, lab)
    b = run_gpu(gpu, lab)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])


def _ball_and_smalls():
    """A digital ball of radius 45 (largest D 2026: the banded paint list) and eight
    balls of radius 4..11 (the plain list) beside it in a 128^3 volume."""
    vol = np.zeros((128, 128, 128), dtype=np.int32)
    m, _ = synth.ball_mask(45)
    vol[1:1 + m.shape[0], 1:1 + m.shape[1], 1:1 + m.shape[2]][m] = 1
    for i, r in enumerate(range(4, 12)):
        m, _ = synth.ball_mask(r)
        z, y = 2 + 30 * (i // 2), 2 + 40 * (i % 2)
        vol[z:z + m.shape[0], y:y + m.shape[1], 98:98 + m.shape[2]][m] = i + 2
    return vol


@pytest.mark.parametrize("case", ["cfg2", "ball_and_smalls"])
def test_label_numbering_does_not_change_results(gpu, case):
    """The paint work items are ordered by estimated cost, not by label: renumbering
    the objects (random and reversed) leaves D and LT unchanged bit for bit and
    permutes the per-object measures with the labels."""
    lab = synth.cfg2()[0] if case == "cfg2" else _ball_and_smalls()
    k = int(lab.max())
    base = run_gpu(gpu, lab)
    if case == "ball_and_smalls":                 # a digital ball of radius r: LT^2 = r^2 + 1
        for l, r in [(1, 45)] + [(i + 2, r) for i, r in enumerate(range(4, 12))]:
            assert np.all(base["lt_sq"][lab == l] == r * r + 1)
    rng = np.random.default_rng(11)
    for name, perm in (("random", rng.permutation(k) + 1), ("reversed", np.arange(k, 0, -1))):
        _note(f"{case}: {name} numbering")
        lut = np.zeros(k + 1, dtype=lab.dtype)
        lut[1:] = perm
        got = run_gpu(gpu, lut[lab], max_label=k)
        np.testing.assert_array_equal(got["dist_sq"], base["dist_sq"])
        np.testing.assert_array_equal(got["lt_sq"], base["lt_sq"])
        for key in ("volume", "shell_count", "max_lt_sq") + FLOAT_KEYS:
            np.testing.assert_array_equal(got[key][perm], base[key][1:k + 1], err_msg=f"{name}: {key}")


def test_closed_forms_entry_fp32_vs_fp64(gpu):
    """The FP32 closed forms over a wide range of volumes and mean thickness,
    including near-spheres and extreme oblate / prolate spheroids."""
    torch, lt = gpu
    rng = np.random.default_rng(3)
    n = 4000
    V = np.concatenate([rng.integers(1, 10 ** 6, n - 8), [1, 7, 1000, 10 ** 6, 4169, 515, 2, 3]])
    r0 = (3 * V / (4 * np.pi)) ** (1 / 3)
    a = r0 * np.exp(rng.uniform(-2.5, 2.5, n))
    a[:40] = r0[:40] * (1 + rng.uniform(-1e-3, 1e-3, 40))
    a = np.maximum(a, 1.0)
    q = np.rint(a * V * 2.0 ** 23).astype(np.uint64)
    mx = np.rint(np.maximum(a, 1) ** 2 * 1.5).astype(np.int32)
    ns = np.maximum(V // 3, 1).astype(np.uint64)
    sq = np.rint(np.sqrt(mx * 0.8) * ns * 2.0 ** 23).astype(np.uint64)
    dev = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    for ndim in (2, 3):
        out = lt.closed_forms(dev(V.astype(np.uint64)), dev(q), dev(mx), dev(ns), dev(sq), ndim)
        torch.cuda.synchronize()
        mean = q.astype(np.float64) / 2.0 ** 23 / V
        f = O.sphericity_3d if ndim == 3 else O.sphericity_2d
        ref_s = np.array([f(float(v), float(m)) for v, m in zip(V, mean)])
        ref_r = (sq.astype(np.float64) / 2.0 ** 23 / ns) / np.sqrt(mx.astype(np.float64))
        np.testing.assert_allclose(out["sphericity"].cpu().numpy(), ref_s, rtol=RTOL)
        np.testing.assert_allclose(out["roundness"].cpu().numpy(), ref_r, rtol=RTOL)
        np.testing.assert_allclose(out["mean_lt"].cpu().numpy(), mean, rtol=RTOL)
