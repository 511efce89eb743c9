"""Pins of the oracle's anisotropic-spacing form (squared voxel spacings w along
each axis; |o|^2 = sum_i w_i o_i^2).  The paper's volumes have unit spacing; the
weighted form extends its distance map and local thickness to voxels that are
longer along some axes, as micro-CT stacks often are.  Pinned against:
  * the literal definitions (tier 0, all pairs) on small random label images;
  * scipy's Euclidean distance transform with per-axis sampling sqrt(w);
  * homogeneity: weights (k, k, k) multiply D and LT by k; unit weights give the
    unweighted oracle;
  * axis permutations of the image with the weights permuted alike;
  * a digital weighted ball {q : |q|_w^2 <= R}: every voxel lies in the centre's
    ball, so LT equals the centre's D, the smallest weighted lattice norm above R
    (found here by plain enumeration);
  * the physical volume of that ball (voxel count times sqrt(prod w)) against
    4/3 pi R^(3/2), and its sphericity near 1."""
import itertools
import math

import numpy as np
import pytest
from scipy import ndimage

from oracle import lt_oracle as O
from paper_2504_05808_amd import synth

WEIGHTS3 = [(4, 1, 1), (1, 4, 1), (2, 3, 5), (9, 4, 1), (1, 1, 7)]
WEIGHTS2 = [(4, 1), (1, 9), (3, 5)]


def _blobby(rng, shape, n_labels, p_bg, blob):
    return synth.random_labels(rng, shape, n_labels=n_labels, p_bg=p_bg, blob=blob)


@pytest.mark.parametrize("shape,weights", [((7, 9, 11), w) for w in WEIGHTS3] +
                         [((13, 17), w) for w in WEIGHTS2])
def test_tier1_equals_literal_definition(shape, weights):
    rng = synth.rng_for(900 + sum(shape) + sum(weights))
    for blob, nl, pbg in [(3, 2, 0.0), (4, 3, 0.1), (2, 4, 0.2)]:
        lab = _blobby(rng, shape, nl, pbg, blob)
        D = O.edt_sq(lab, weights)
        np.testing.assert_array_equal(D, O.edt_sq_brute(lab, weights))
        LT = O.local_thickness_sq(D, weights=weights)
        np.testing.assert_array_equal(LT, O.local_thickness_sq_brute(lab, D, weights))
        obj = lab != 0
        assert np.all(LT[obj] >= D[obj]) and np.all(LT[~obj] == 0)


@pytest.mark.parametrize("weights", WEIGHTS3 + WEIGHTS2)
def test_distance_matches_scipy_sampling(weights):
    nd = len(weights)
    rng = synth.rng_for(950 + sum(weights))
    shape = (14, 19, 23)[-nd:] if nd == 3 else (31, 37)
    lab = _blobby(rng, shape, 3, 0.1, 5)
    D = O.edt_sq(lab, weights)
    samp = np.sqrt(np.asarray(weights, np.float64))
    for l in np.unique(lab):
        if l == 0:
            continue
        m = np.pad(lab == l, 1)                  # outside the image is background
        e = ndimage.distance_transform_edt(m, sampling=samp)[(slice(1, -1),) * nd]
        np.testing.assert_array_equal(D[lab == l], np.rint(e[lab == l] ** 2).astype(np.int64))


def test_homogeneity_and_unit_weights():
    rng = synth.rng_for(970)
    lab = _blobby(rng, (12, 15, 18), 3, 0.1, 4)
    D1 = O.edt_sq(lab)
    LT1 = O.local_thickness_sq(D1)
    np.testing.assert_array_equal(O.edt_sq(lab, (1, 1, 1)), D1)
    for k in (2, 3, 7):
        Dk = O.edt_sq(lab, (k, k, k))
        np.testing.assert_array_equal(Dk, k * D1)
        np.testing.assert_array_equal(O.local_thickness_sq(Dk, weights=(k, k, k)), k * LT1)


def test_axis_permutation():
    rng = synth.rng_for(980)
    lab = _blobby(rng, (9, 12, 15), 3, 0.1, 4)
    w = (2, 3, 5)
    D = O.edt_sq(lab, w)
    LT = O.local_thickness_sq(D, weights=w)
    for perm in itertools.permutations(range(3)):
        labp = np.ascontiguousarray(np.transpose(lab, perm))
        wp = tuple(w[i] for i in perm)
        Dp = O.edt_sq(labp, wp)
        np.testing.assert_array_equal(Dp, np.transpose(D, perm))
        np.testing.assert_array_equal(O.local_thickness_sq(Dp, weights=wp), np.transpose(LT, perm))


def _weighted_ball(weights, R):
    """{q : sum w_i q_i^2 <= R}, centred, padded by one voxel; and the smallest
    weighted lattice norm above R."""
    half = [int(math.isqrt(R // w)) for w in weights]
    grids = np.meshgrid(*[np.arange(-h - 1, h + 2) for h in half], indexing="ij")
    n2 = sum(w * g * g for w, g in zip(weights, grids))
    m = n2 <= R
    above = min(int(v) for v in n2.ravel() if v > R)
    # the enumeration box reaches one step past every axis: a norm just above R is
    # never farther than one step along some axis from the ball
    return m, above


@pytest.mark.parametrize("weights,R", [((4, 1, 1), 100), ((1, 4, 9), 150), ((2, 3, 5), 60), ((4, 1), 200),
                                       ((3, 7), 90)])
def test_weighted_ball_thickness_is_the_centre_distance(weights, R):
    m, above = _weighted_ball(weights, R)
    lab = m.astype(np.int32)
    D = O.edt_sq(lab, weights)
    centre = tuple(s // 2 for s in lab.shape)
    assert D[centre] == above == D.max()
    LT = O.local_thickness_sq(D, weights=weights)
    assert np.all(LT[m] == above) and np.all(LT[~m] == 0)


def test_weighted_ball_physical_volume_and_sphericity():
    for weights, R in (((4, 1, 1), 400), ((1, 9, 4), 900)):
        m, _ = _weighted_ball(weights, R)
        res = O.measure(m.astype(np.int32), per_object=False, weights=weights)
        vs = math.sqrt(math.prod(weights))
        assert res["volume"][1] == m.sum()
        v_phys = res["volume"][1] * vs
        assert v_phys == pytest.approx(4 / 3 * math.pi * R ** 1.5, rel=0.03)
        assert res["roundness"][1] == pytest.approx(1.0, abs=1e-12)
        assert 0.999 < res["sphericity"][1] <= 1.0 + 1e-9
    # 2D: a weighted digital disc is a physical disc of radius sqrt(R)
    m, _ = _weighted_ball((4, 1), 900)
    res = O.measure(m.astype(np.int32), per_object=False, weights=(4, 1))
    assert res["volume"][1] * 2.0 == pytest.approx(math.pi * 900, rel=0.02)
    assert 0.999 < res["sphericity"][1] <= 1.0 + 1e-9
