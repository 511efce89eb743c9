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


# --------------------------------------------------------------------------- 2D contour

def test_contour_single_pixel_rectangle_and_diagonal_pair():
    """Marching squares at 0.5 on zero-padded masks, worked by hand: one pixel is cut
    off in each of its 4 squares (4 x sqrt(2)/2); a w x h block has w - 1 + h - 1
    unit steps on each pair of sides plus 4 corner cuts, 2(w - 1) + 2(h - 1) +
    2 sqrt 2; two pixels touching at a corner share one square with both diagonal
    corners inside (sqrt 2) and have three single-corner squares each."""
    r2 = math.sqrt(2.0)
    one = np.ones((1, 1), bool)
    assert M.contour_length(one) == pytest.approx(2 * r2, rel=1e-15)
    for w, h in [(1, 1), (3, 5), (7, 2), (1, 6)]:
        m = np.ones((h, w), bool)
        assert M.contour_length(m) == pytest.approx(2 * (w - 1) + 2 * (h - 1) + 2 * r2, rel=1e-14)
    diag = np.eye(2, dtype=bool)
    assert M.contour_length(diag) == pytest.approx(3 * r2 + r2, rel=1e-14)
    # an L of three pixels (0, 0), (1, 0), (1, 1): tracing the crossings around it
    # gives the polygon (-1/2, 0) (0, 1/2) (1/2, 1) (1, 3/2) (3/2, 1) (3/2, 0) (1, -1/2)
    # (0, -1/2) in (y, x): six diagonal sides of sqrt(2)/2 and two unit sides
    ell = np.zeros((3, 3), bool)
    ell[0, 0] = ell[1, 0] = ell[1, 1] = True
    assert M.contour_length(ell) == pytest.approx(3 * r2 + 2, rel=1e-14)


def test_contour_symmetries_and_sphericity():
    rng = np.random.default_rng(8)
    for _ in range(4):
        r = rng.random((9, 13)) < 0.5
        a = M.contour_length(r)
        for t in (r.T, r[::-1], r[:, ::-1], r[::-1, ::-1].T):
            assert M.contour_length(t) == pytest.approx(a, rel=1e-13)
        assert M.contour_length(r, pad=False) == pytest.approx(M.contour_length(~r, pad=False), rel=1e-13)
    # a large digital disc: the midpoint contour is a chain of unit and diagonal
    # steps; a straight edge at angle t in [0, pi/4] costs cos t + (sqrt 2 - 1) sin t
    # per unit length, on average over t 8 (sqrt 2 - 1) / pi, so the perimeter
    # sphericity of a large disc tends to pi / (8 (sqrt 2 - 1)) = 0.94806
    lim = math.pi / (8 * (math.sqrt(2) - 1))
    errs = []
    for r in (100, 200, 400):
        m, _ = synth.disc_mask(r)
        errs.append(abs(M.contour_sphericity(m) - lim))
    assert errs[0] < 3e-3 and errs[1] < 1e-3 and errs[2] < 1e-3 and errs[2] < errs[0]
    assert M.contour_sphericity(np.ones((1, 1), bool)) == pytest.approx(2 * math.sqrt(math.pi) / (2 * math.sqrt(2)))


def test_mesh_measures_per_label():
    """Per-label mesh measures treat other labels as outside: an object's area does
    not change when another label touches it, and equals the single-mask area."""
    m, _ = synth.ball_mask(5)
    lab = np.pad(m.astype(np.int32), 2)
    alone = M.mesh_measures(lab)
    crowd = lab.copy()
    crowd[(crowd == 0) & (np.indices(crowd.shape)[0] < 7)] = 3
    both = M.mesh_measures(crowd, max_label=4)
    assert both["volume"][1] == alone["volume"][1] == m.sum()
    assert both["area"][1] == pytest.approx(M.iso_area(m), rel=1e-14)
    assert both["area"][1] == pytest.approx(alone["area"][1], rel=1e-14)
    assert both["sphericity"][1] == pytest.approx(M.mesh_sphericity(m), rel=1e-14)
    assert both["area"][3] == pytest.approx(M.iso_area(crowd == 3), rel=1e-14)
    assert np.isnan(both["sphericity"][2]) and np.isnan(both["sphericity"][4]) and both["volume"][2] == 0
    d, _ = synth.disc_mask(7)
    lab2 = np.pad(d.astype(np.uint16), 3)
    lab2[0, :] = 2
    r = M.mesh_measures(lab2)
    assert r["area"][1] == pytest.approx(M.contour_length(d), rel=1e-14)
    # label 2 is a 1 x w row of pixels: 2 (w - 1) + 2 sqrt 2
    assert r["area"][2] == pytest.approx(2 * (lab2.shape[1] - 1) + 2 * math.sqrt(2.0), rel=1e-14)
