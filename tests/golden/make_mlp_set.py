"""Write the learned-correction data set from the CPU oracles only.

Each record is one isolated synthetic object (shape recipe of the 512^3 workload:
digital balls, ellipsoids, superellipsoids, and superellipsoids with value-noise
surfaces; semi-axes U[4,30]) measured by the CPU oracle: the 34 features of the
correction network (32-bin local-thickness histogram, log V, mean LT / V^(1/3)),
the closed-form sphericity S_LT, and the mesh sphericity S_mesh from the
marching-tetrahedra iso-surface.  Record i draws from seed 5_000_000 + i.

usage: python tests/golden/make_mlp_set.py N OUT.npz [workers]

If OUT.npz already holds the first M < N records, only records M..N-1 are computed
and appended (record i depends on i alone, so the result equals a fresh run).
"""
from __future__ import annotations

import math
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import lt_oracle as O          # noqa: E402
from oracle import mesh_area as M          # noqa: E402
from paper_2504_05808_amd import synth     # noqa: E402

SEED0 = 5_000_000


def shape(i: int):
    rng = synth.rng_for(SEED0 + i)
    kind = i % 4
    if kind == 0:
        m, _ = synth.ball_mask(int(rng.integers(4, 31)))
    elif kind == 1:
        axes = rng.uniform(4.0, 30.0, 3)
        m, _ = synth.ellipsoid_mask(axes, synth.haar_rotation(rng), rng.uniform(0, 1, 3))
    else:
        axes = rng.uniform(4.0, 30.0, 3)
        e1, e2 = rng.uniform(0.3, 1.0, 2)
        amp = 0.0 if kind == 2 else float(rng.uniform(0.0, 2.0))
        m, _ = synth.superellipsoid_mask(axes, float(e1), float(e2), synth.haar_rotation(rng), amp, rng,
                                         rng.uniform(0, 1, 3))
    idx = np.nonzero(m)
    sl = tuple(slice(int(a.min()), int(a.max()) + 1) for a in idx)
    return kind, m[sl]


def record(i: int):
    kind, m = shape(i)
    lab = np.pad(m.astype(np.int32), 1)
    D = O.edt_sq(lab)
    LT = O.local_thickness_sq(D)
    sums = O.object_sums(lab, LT, 1)
    cf = O.closed_forms(sums, 3)
    V = float(sums["volume"][1])
    hist = O.lt_histogram(lab, LT, sums["max_lt_sq"])[1]
    feat = np.concatenate([hist, [math.log(V), cf["mean_lt"][1] / V ** (1 / 3)]])
    return feat, cf["sphericity"][1], M.mesh_sphericity(m), V, kind


def main():
    n = int(sys.argv[1])
    out = sys.argv[2]
    workers = int(sys.argv[3]) if len(sys.argv) > 3 else os.cpu_count() or 1
    t0 = time.time()
    shard = 2000
    parts = _load(out) if os.path.exists(out) else []
    if len(parts) >= n:
        print(f"{out} already holds {len(parts)} records", flush=True)
        return
    with Pool(workers) as pool:
        for s0 in range(len(parts), n, shard):
            recs = pool.map(record, range(s0, min(n, s0 + shard)), chunksize=8)
            parts.extend(recs)
            print(f"{len(parts)}/{n} records, {time.time() - t0:.0f}s", flush=True)
            if len(parts) % 20000 == 0 or len(parts) == n:
                _save(out, parts)


def _load(out):
    d = np.load(out)
    if int(d["seed0"]) != SEED0:
        raise ValueError(f"{out} was written with another seed base")
    feat = np.concatenate([d["hist"].astype(np.float32), d["extra"]], axis=1)
    return [(feat[i], float(d["s_lt"][i]), float(d["s_mesh"][i]), float(d["volume"][i]), int(d["kind"][i]))
            for i in range(len(feat))]


def _save(out, parts):
    feat = np.stack([p[0] for p in parts]).astype(np.float32)
    np.savez_compressed(out + ".tmp.npz", hist=feat[:, :32].astype(np.float16), extra=feat[:, 32:],
                        s_lt=np.array([p[1] for p in parts]), s_mesh=np.array([p[2] for p in parts]),
                        volume=np.array([p[3] for p in parts]), kind=np.array([p[4] for p in parts], np.uint8),
                        seed0=SEED0)
    os.replace(out + ".tmp.npz", out)


if __name__ == "__main__":
    main()
