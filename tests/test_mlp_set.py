"""The stored training set of the learned correction (tests/golden/mlp_set.npz) was
written by tests/golden/make_mlp_set.py from the CPU oracles alone: every record
depends on its index only, so records re-made here must equal the stored ones (with
the storage precisions: histogram float16, the two extra features float32)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))

import make_mlp_set as G  # noqa: E402

SET = os.path.join(ROOT, "tests", "golden", "mlp_set.npz")


@pytest.fixture(scope="module")
def stored():
    return np.load(SET)


def test_size_and_kinds(stored):
    n = len(stored["s_lt"])
    assert n == 200000 and int(stored["seed0"]) == G.SEED0
    assert stored["hist"].shape == (n, 32) and stored["extra"].shape == (n, 2)
    # the recipe cycles balls, ellipsoids, superellipsoids, noisy superellipsoids
    np.testing.assert_array_equal(stored["kind"], np.arange(n) % 4)
    # histograms are fractions of the object's voxels
    np.testing.assert_allclose(stored["hist"].astype(np.float64).sum(axis=1), 1.0, atol=2e-2)


@pytest.mark.parametrize("i", [0, 1, 2, 3, 40001, 123457, 199998, 199999])
def test_records_remade_from_the_oracle(stored, i):
    feat, s_lt, s_mesh, v, kind = G.record(i)
    np.testing.assert_array_equal(stored["hist"][i], feat[:32].astype(np.float32).astype(np.float16))
    np.testing.assert_array_equal(stored["extra"][i], feat[32:].astype(np.float32))
    assert stored["s_lt"][i] == s_lt and stored["s_mesh"][i] == s_mesh
    assert stored["volume"][i] == v and stored["kind"][i] == kind
