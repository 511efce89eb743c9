"""Mesh surface area of a binary object -- TEST INFRASTRUCTURE (CPU oracle).

The paper's sphericity baseline meshes each object (marching cubes in 3D,
marching squares in 2D, on the mask) and measures the mesh area or contour length
(Related work; Experiments, Benchmark methods).  This module gives project-written
equivalents, used as the oracle of the GPU mesh measures and as the training /
evaluation target of the learned sphericity correction: the iso-surface (3D) or
iso-line (2D) at level 0.5 of the zero-padded binary mask.  In 3D the surface is
built by marching tetrahedra; in 2D by marching squares.

Construction.  Every unit cube of the lattice is split into the six tetrahedra of
the Freudenthal (Kuhn) subdivision: for each ordering (i, j, k) of the three axes,
the tetrahedron 0 -> e_i -> e_i + e_j -> e_i + e_j + e_k.  Neighbouring cubes
share the split of their common faces, so the surface is closed.  In a tetrahedron
the iso-surface of the linearly interpolated 0/1 values at 0.5 passes through the
midpoints of the edges joining an inside and an outside corner: one corner apart
from the other three gives a triangle, two against two gives a parallelogram.
Since all tetrahedra have lattice corners, the area of every (tetrahedron, inside
pattern) pair is computed once from those midpoints, and the surface area is a sum
of table look-ups over all cubes.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

_PERMS = list(itertools.permutations(range(3)))        # axis orderings


def _tet_corners(perm):
    e = np.eye(3, dtype=np.int64)
    p0 = np.zeros(3, dtype=np.int64)
    p1 = p0 + e[perm[0]]
    p2 = p1 + e[perm[1]]
    p3 = p2 + e[perm[2]]
    return np.stack([p0, p1, p2, p3])                   # (x, y, z) offsets in the cube


def _pattern_area(corners: np.ndarray, inside: tuple) -> float:
    """Area of the 0.5 iso-surface in one tetrahedron for a given inside pattern."""
    ins = [i for i in range(4) if inside[i]]
    out = [i for i in range(4) if not inside[i]]
    if len(ins) in (0, 4):
        return 0.0
    c = corners.astype(np.float64)
    if len(ins) in (1, 3):
        lone = ins[0] if len(ins) == 1 else out[0]
        rest = [i for i in range(4) if i != lone]
        m = [(c[lone] + c[r]) / 2 for r in rest]
        return 0.5 * float(np.linalg.norm(np.cross(m[1] - m[0], m[2] - m[0])))
    u, v = ins
    a, b = out
    mua, mub, mvb, mva = (c[u] + c[a]) / 2, (c[u] + c[b]) / 2, (c[v] + c[b]) / 2, (c[v] + c[a]) / 2
    # the four midpoints form a parallelogram mua -> mub -> mvb -> mva
    return float(np.linalg.norm(np.cross(mub - mua, mva - mua)))


def _tables():
    tabs = []
    for perm in _PERMS:
        corners = _tet_corners(perm)
        t = np.zeros(16)
        for code in range(16):
            inside = tuple((code >> i) & 1 for i in range(4))
            t[code] = _pattern_area(corners, inside)
        tabs.append((corners, t))
    return tabs


_TABLES = _tables()


def iso_area(mask: np.ndarray, pad: bool = True) -> float:
    """Area of the iso-surface at 0.5 of the binary 3D mask ([z][y][x]), zero-padded
    by one voxel unless pad=False (then only the cubes inside the array count)."""
    m = np.asarray(mask, dtype=bool)
    m = (np.pad(m, 1) if pad else m).astype(np.int64)
    nz, ny, nx = m.shape
    total = 0.0
    for corners, tab in _TABLES:
        code = np.zeros((nz - 1, ny - 1, nx - 1), dtype=np.int64)
        for bit, (cx, cy, cz) in enumerate(corners):
            code |= m[cz:cz + nz - 1, cy:cy + ny - 1, cx:cx + nx - 1] << bit
        total += float((tab * np.bincount(code.ravel(), minlength=16)).sum())
    return total


def iso_volume(mask: np.ndarray, pad: bool = True) -> float:
    """Volume enclosed by the same surface: a tetrahedron (volume 1/6) contributes
    1/48 with one corner inside (the corner tetrahedron of half size), 1/6 - 1/48
    with three, half of 1/6 with two (the midpoint section halves it by symmetry of
    the two corner pairs), 1/6 with four."""
    m = np.asarray(mask, dtype=bool)
    m = (np.pad(m, 1) if pad else m).astype(np.int64)
    nz, ny, nx = m.shape
    frac = {0: 0.0, 1: 1 / 48, 2: 1 / 12, 3: 1 / 6 - 1 / 48, 4: 1 / 6}
    vol = 0.0
    for corners, _ in _TABLES:
        cnt = np.zeros((nz - 1, ny - 1, nx - 1), dtype=np.int64)
        for (cx, cy, cz) in corners:
            cnt += m[cz:cz + nz - 1, cy:cy + ny - 1, cx:cx + nx - 1]
        hist = np.bincount(cnt.ravel(), minlength=5)
        vol += sum(frac[k] * hist[k] for k in range(5))
    return vol


def mesh_sphericity(mask: np.ndarray) -> float:
    """Wadell sphericity pi^(1/3) (6V)^(2/3) / A with V the voxel count and A the
    iso-surface area (the mesh-based sphericity used as the learning target)."""
    V = float(np.count_nonzero(mask))
    return math.pi ** (1 / 3) * (6 * V) ** (2 / 3) / iso_area(mask)


# ---------------------------------------------------------------------------
# 2D: marching squares
# ---------------------------------------------------------------------------
#
# A unit square of the lattice has corners c0 = (0, 0), c1 = (0, 1), c2 = (1, 0),
# c3 = (1, 1) in (y, x).  The 0.5 iso-line of the linearly interpolated 0/1 values
# crosses every edge joining an inside and an outside corner at its midpoint.  Two
# crossings are joined by one segment.  Four crossings (two diagonal corners inside)
# are joined in two segments; of the two ways to pair them, each gives segments of
# length sqrt(2)/2 in a unit square, so the contour length does not depend on the
# choice: here each inside corner is cut off on its own.

_SQ_CORNERS = np.array([(0, 0), (0, 1), (1, 0), (1, 1)], dtype=np.float64)
_SQ_EDGES = [(0, 1), (0, 2), (1, 3), (2, 3)]           # corner pairs along the sides


def _square_length(inside: tuple) -> float:
    mids = {e: (_SQ_CORNERS[e[0]] + _SQ_CORNERS[e[1]]) / 2 for e in _SQ_EDGES if inside[e[0]] != inside[e[1]]}
    if not mids:
        return 0.0
    if len(mids) == 2:
        a, b = mids.values()
        return float(np.linalg.norm(a - b))
    total = 0.0                                          # saddle: cut off each inside corner
    for c in range(4):
        if inside[c]:
            a, b = [m for e, m in mids.items() if c in e]
            total += float(np.linalg.norm(a - b))
    return total


_SQ_TABLE = np.array([_square_length(tuple((code >> i) & 1 for i in range(4))) for code in range(16)])


def contour_length(mask: np.ndarray, pad: bool = True) -> float:
    """Length of the 0.5 iso-line of the binary 2D mask ([y][x]), zero-padded by one
    pixel unless pad=False (then only the squares inside the array count)."""
    m = np.asarray(mask, dtype=bool)
    m = (np.pad(m, 1) if pad else m).astype(np.int64)
    ny, nx = m.shape
    code = (m[:ny - 1, :nx - 1] | (m[:ny - 1, 1:] << 1) | (m[1:, :nx - 1] << 2) | (m[1:, 1:] << 3))
    return float((_SQ_TABLE * np.bincount(code.ravel(), minlength=16)).sum())


def contour_sphericity(mask: np.ndarray) -> float:
    """Perimeter sphericity P_c / P_o (Background) with P_o the marching-squares
    contour length and P_c = 2 sqrt(pi A) for A the pixel count."""
    A = float(np.count_nonzero(mask))
    return 2.0 * math.sqrt(math.pi * A) / contour_length(mask)


# ---------------------------------------------------------------------------
# per label
# ---------------------------------------------------------------------------

def mesh_measures(labels: np.ndarray, max_label: int | None = None) -> dict:
    """Per label 0..max_label of a 2D or 3D label image: voxel count V, mesh area
    (3D surface, 2D contour length) of the label's own mask (every other label and
    the outside are background), and the mesh sphericity (3D: pi^(1/3) (6V)^(2/3) / A;
    2D: 2 sqrt(pi V) / P).  Absent labels (and label 0) get V = 0, area 0 and NaN."""
    from scipy import ndimage
    lab = np.asarray(labels)
    if max_label is None:
        max_label = int(lab.max()) if lab.size else 0
    n = max_label + 1
    V = np.zeros(n, dtype=np.int64)
    area = np.zeros(n)
    sph = np.full(n, np.nan)
    work = lab.astype(np.int64)
    for i, sl in enumerate(ndimage.find_objects(work)):
        l = i + 1
        if sl is None or l >= n:
            continue
        m = work[sl] == l                         # the crop's zero padding is outside
        V[l] = int(m.sum())
        if lab.ndim == 3:
            area[l] = iso_area(m)
            sph[l] = math.pi ** (1 / 3) * (6 * V[l]) ** (2 / 3) / area[l]
        else:
            area[l] = contour_length(m)
            sph[l] = 2.0 * math.sqrt(math.pi * V[l]) / area[l]
    return dict(volume=V, area=area, sphericity=sph)
