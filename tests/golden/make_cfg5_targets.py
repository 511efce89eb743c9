"""Write the mesh-sphericity targets of the learned correction's evaluation volume
from the CPU oracle only.

The volume is the seeded 1024^3 uint32 volume of ``synth.cfg5_volume`` (objects of
the 512^3 distribution).  For every present label the mesh sphericity S_mesh of
``oracle.mesh_area`` is computed on the object's own mask (bounding box, zero
padded).  The file also records the volume's digest so that a test can check that
it regenerated the same volume.

usage: python tests/golden/make_cfg5_targets.py OUT.npz [draws] [workers]
"""
from __future__ import annotations

import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mesh_area as M          # noqa: E402
from paper_2504_05808_amd import synth     # noqa: E402

_VOL = None


def _one(item):
    label, sl = item
    return label, M.mesh_sphericity(_VOL[sl] == label)


def main():
    global _VOL
    out = sys.argv[1]
    draws = int(sys.argv[2]) if len(sys.argv) > 2 else 5
    workers = int(sys.argv[3]) if len(sys.argv) > 3 else os.cpu_count() or 1
    t0 = time.time()
    vol, meta = synth.cfg5_volume(draws=draws, workers=workers, progress=print)
    print(f"volume {vol.shape} {meta['n_objects']} objects, {time.time() - t0:.0f}s", flush=True)
    from scipy import ndimage
    _VOL = vol
    boxes = ndimage.find_objects(vol.astype(np.int32))
    items = [(i + 1, sl) for i, sl in enumerate(boxes) if sl is not None]
    with Pool(workers) as pool:
        res = pool.map(_one, items, chunksize=16)
    labels = np.array([r[0] for r in res], dtype=np.int64)
    s_mesh = np.array([r[1] for r in res])
    np.savez_compressed(out, labels=labels, s_mesh=s_mesh, digest=synth.digest(vol),
                        n_objects=meta["n_objects"], draws=draws)
    print(f"{len(labels)} targets written, {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main()
