"""The roofline accounting of bench.py: lattice-point counts and containment tables,
and the ball-cover work (sum over kept centres of the open-ball lattice counts),
checked against brute force on small labelled volumes."""
import itertools
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench                                   # noqa: E402
from oracle import lt_oracle as O             # noqa: E402
from paper_2504_05808_amd import synth        # noqa: E402

PTS = np.array(list(itertools.product(range(-9, 10), repeat=3)))
Q2 = (PTS ** 2).sum(1)


def test_lattice_tables_brute_force():
    N, T = bench.lattice_tables(70)
    for d in [0, 1, 2, 3, 4, 5, 9, 10, 17, 30, 50, 70]:
        assert N[d] == int((Q2 < d).sum())
        for c, o in enumerate([(1, 0, 0), (1, 1, 0), (1, 1, 1)]):
            sel = Q2 < d
            ref = int(((PTS[sel] - np.array(o)) ** 2).sum(1).max()) if sel.any() else -1
            assert T[c][d] == ref


@pytest.mark.parametrize("seed,shape,blob", [(1, (12, 13, 11), 3), (2, (9, 10, 14), 4), (3, (6, 15, 8), 2)])
def test_ball_cover_work_brute_force(seed, shape, blob):
    torch = pytest.importorskip("torch")
    lab = synth.random_labels(synth.rng_for(seed), shape, n_labels=3, p_bg=0.2, blob=blob)
    D = O.edt_sq(lab)
    assert D.max() < 81                         # the brute force below covers |q| <= 9
    work, kept = bench.ball_cover_work(torch.from_numpy(lab), torch.from_numpy(D.astype(np.int32)))
    W = K = 0
    Z, Y, X = lab.shape
    for z, y, x in zip(*np.nonzero(lab)):
        d = D[z, y, x]
        inside = PTS[Q2 < d]
        covered = False
        for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
            if (dz, dy, dx) == (0, 0, 0):
                continue
            zz, yy, xx = z + dz, y + dy, x + dx
            if not (0 <= zz < Z and 0 <= yy < Y and 0 <= xx < X) or lab[zz, yy, xx] != lab[z, y, x]:
                continue
            if ((inside - np.array([dx, dy, dz])) ** 2).sum(1).max() < D[zz, yy, xx]:
                covered = True
                break
        if not covered:
            K += 1
            W += len(inside)
    assert (work, kept) == (W, K)
