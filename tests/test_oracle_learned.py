"""Pins of the learned-correction oracles (mesh area, FP64 network) against facts
that do not come from them: exact flat-surface areas and volumes, symmetries of the
iso-surface, torch's bfloat16 rounding, and central finite differences."""
import math

import numpy as np
import pytest

from oracle import mesh_area as M
from oracle import mlp_ref as R
from paper_2504_05808_amd import synth


def test_flat_surface_area_and_volume_exact():
    """A half-space x <= k filling the whole y-z extent: the 0.5 iso-surface is the
    plane x = k + 1/2, so its area is (ny - 1)(nz - 1) and the enclosed volume
    (k + 1/2)(ny - 1)(nz - 1)."""
    for k, shape in [(3, (6, 7, 9)), (0, (4, 5, 3)), (5, (9, 4, 8))]:
        m = np.zeros(shape, bool)
        m[:, :, :k + 1] = True
        a = (shape[0] - 1) * (shape[1] - 1)
        assert M.iso_area(m, pad=False) == pytest.approx(a, abs=1e-12)
        assert M.iso_volume(m, pad=False) == pytest.approx((k + 0.5) * a, abs=1e-12)
    m = np.zeros((5, 8, 6), bool)
    m[:2] = True                                   # plane normal to z
    assert M.iso_area(m, pad=False) == pytest.approx(7 * 5, abs=1e-12)


def test_iso_surface_symmetries():
    """Axis permutations map the cube split onto itself, and the level 0.5 surface
    of a mask and of its complement coincide."""
    rng = np.random.default_rng(4)
    for _ in range(3):
        r = rng.random((7, 8, 9)) < 0.45
        a = M.iso_area(r)
        for perm in [(1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0)]:
            assert M.iso_area(r.transpose(perm)) == pytest.approx(a, rel=1e-12)
        assert M.iso_area(r, pad=False) == pytest.approx(M.iso_area(~r, pad=False), rel=1e-12)
        big = np.zeros((12, 13, 14), bool)
        big[2:9, 3:11, 4:13] = r
        assert M.iso_area(big) == pytest.approx(a, rel=1e-12)          # translation


def test_ball_area_bias_is_stable_and_volume_converges():
    """Digital balls: the enclosed volume tends to the voxel count and the area
    exceeds the equal-volume sphere's by a factor that settles (the fixed bias of
    a midpoint iso-surface of binary data)."""
    ratios = []
    for r in (10, 15, 20, 30):
        b, _ = synth.ball_mask(r)
        V = b.sum()
        re = (3 * V / (4 * math.pi)) ** (1 / 3)
        ratios.append(M.iso_area(b) / (4 * math.pi * re * re))
        assert abs(M.iso_volume(b) / V - 1) < 0.02 * 10 / r
    assert max(ratios) - min(ratios) < 0.02
    assert 1.2 < np.mean(ratios) < 1.35


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(5000) * 10 ** rng.uniform(-5, 5, 5000),
                        [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -0.0, 65504.0, 1e-40]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(R.bf16(x), ref)


def _small_net(seed=0):
    rng = np.random.default_rng(seed)
    w = {"W1": np.zeros((R.H, R.INP)), "W4": np.zeros((R.OUTP, R.H))}
    w["W1"][:, :R.IN] = rng.normal(0, 0.3, (R.H, R.IN))
    w["W2"] = rng.normal(0, 0.2, (R.H, R.H))
    w["W3"] = rng.normal(0, 0.2, (R.H, R.H))
    w["W4"][0] = rng.normal(0, 0.3, R.H)
    for k in ("b1", "b2", "b3"):
        w[k] = rng.normal(0, 0.1, R.H)
    w["b4"] = np.zeros(R.OUTP)
    w["b4"][0] = 0.05
    return R.pack(w)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(2)
    p = _small_net()
    x = rng.normal(0, 1, (24, R.IN))
    y = rng.normal(0, 1, 24)
    mean, inv = np.zeros(R.IN), np.ones(R.IN)
    g = R.backward(p, x, y, mean, inv, bf16_ops=False)
    used = np.nonzero(np.abs(g) > 0)[0]
    pick = rng.choice(used, 60, replace=False)
    for k in ("b4", "W4"):
        pick = np.append(pick, R.OFF[k][0])
    h = 1e-6
    for i in pick:
        e = np.zeros_like(p)
        e[i] = h
        fd = (R.loss(p + e, x, y, mean, inv) - R.loss(p - e, x, y, mean, inv)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-5, abs=1e-9)
    # padding parameters get no gradient
    W1 = R.unpack(g)["W1"]
    assert np.all(W1[:, R.IN:] == 0) and np.all(R.unpack(g)["W4"][1:] == 0)


def test_forward_special_cases():
    p = np.zeros(R.N_PARAM)
    p[R.OFF["b4"][0]] = 0.25
    pred, _ = R.forward(p, np.ones((3, R.IN)), np.zeros(R.IN), np.ones(R.IN))
    np.testing.assert_array_equal(pred, 0.25)
    assert R.silu(0.0) == 0.0 and R.silu(40.0) == pytest.approx(40.0)
    assert R.dsilu(0.0) == 0.5


def _ellipsoid_area(a, b, c):
    """Exact surface area of the ellipsoid (Legendre form with incomplete elliptic
    integrals), a >= b > c."""
    from scipy import special
    a, b, c = sorted([a, b, c], reverse=True)
    phi = math.acos(c / a)
    m = (a * a * (b * b - c * c)) / (b * b * (a * a - c * c))
    return 2 * math.pi * c * c + 2 * math.pi * a * b / math.sin(phi) * (
        special.ellipeinc(phi, m) * math.sin(phi) ** 2 + special.ellipkinc(phi, m) * math.cos(phi) ** 2)


def test_ellipsoid_mesh_area_against_exact_area():
    """Digital axis-aligned ellipsoids: the iso-surface area over the exact ellipsoid
    area shows the same staircase bias as digital balls (1.2-1.3: flat faces aligned
    with the lattice have less of it), and the enclosed volume tracks the voxel count.
    The exact-area formula itself is checked at a near-sphere against 4 pi a^2."""
    assert _ellipsoid_area(10.0, 10.0 - 1e-7, 10.0 - 2e-7) == pytest.approx(4 * math.pi * 100, rel=1e-6)
    for axes in [(20, 14, 9), (24, 10, 8), (16, 16, 8.001), (18, 12, 11.999), (22, 15, 6)]:
        m, _ = synth.ellipsoid_mask(np.array(axes, float), np.eye(3), (0.3, 0.2, 0.1))
        ratio = M.iso_area(m) / _ellipsoid_area(*axes)
        assert 1.18 < ratio < 1.30, (axes, ratio)
        assert M.iso_volume(m) == pytest.approx(m.sum(), rel=0.01)


def test_mesh_sphericity_single_voxels_hand_value():
    """One voxel: the 0.5 iso-surface is made of one triangle in each of the 24
    tetrahedra of the cube split around it, spanned by the midpoints of its three
    edges there.  Where the voxel is the split's (0,0,0) or (1,1,1) corner (12
    tetrahedra) the triangle's legs are e_j / 2 and (e_j + e_k) / 2: area 1/8; at
    the other six corners (2 tetrahedra each) the legs are (e_i + e_j) / 2 and
    (e_i + e_j + e_k) / 2: area sqrt(2)/8.  A = 3/2 (1 + sqrt 2), enclosed volume
    24 / 48 = 1/2.  Two separate voxels double the area and V = 2 (voxel count) in
    pi^(1/3) (6V)^(2/3) / A."""
    a1 = 1.5 * (1 + math.sqrt(2))
    one = np.zeros((1, 1, 1), bool)
    one[0, 0, 0] = True
    assert M.iso_area(one) == pytest.approx(a1, rel=1e-14)
    assert M.iso_volume(one) == pytest.approx(0.5, rel=1e-14)
    assert M.mesh_sphericity(one) == pytest.approx(math.pi ** (1 / 3) * 6 ** (2 / 3) / a1, rel=1e-14)
    two = np.zeros((1, 1, 4), bool)
    two[0, 0, 0] = two[0, 0, 3] = True
    assert M.mesh_sphericity(two) == pytest.approx(math.pi ** (1 / 3) * 12 ** (2 / 3) / (2 * a1), rel=1e-14)
