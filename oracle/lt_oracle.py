"""CPU oracle for local-thickness sphericity and roundness -- TEST INFRASTRUCTURE.

Plain, slow, FP64 / int64, written from the paper's definitions so that it can be
checked against them by eye.  It shares no code with the GPU library and imports
nothing from it.  Only the test suite, the smoke check and the benchmark's CPU
baseline use it; the product path never does.

Two tiers:
  * tier 0 (this file, numpy): the literal definitions as exhaustive minima and
    maxima over all pairs -- for images of a few thousand voxels;
  * tier 1 (``lt_oracle.c``): the same definitions with an early exit over offsets
    sorted by length (distance transform) and an unpruned scatter of every ball
    (local thickness), run on whole small images or on one crop per object.

Paper passages followed (arXiv 2504.05808):
  * local thickness: radius of the largest circle/sphere inside the object that
    contains the point (Introduction; Method section, first paragraph);
  * 3D sphericity: Wadell's ratio pi^(1/3) (6V)^(2/3) / S (Background, Eq. 1), with S
    the surface of a spheroid whose two equal semi-axes are the mean local thickness
    and whose third semi-axis is 3V / (4 pi a^2) (Method, Sphericity: spheroid
    surface equations and the c_s equation);
  * 2D sphericity: perimeter sphericity P_c / P_o (Background, perimeter-sphericity
    equation), P_o from Ramanujan's first ellipse-perimeter approximation with
    a = mean local thickness, b = A / (pi a), and P_c = 2 sqrt(pi A) (Method,
    Sphericity, 2D equations);
  * roundness: mean local thickness over the contour (2D, 4-neighbourhood) or surface
    shell (3D, face neighbours) divided by the largest local thickness of the
    object, which is the radius of the maximal inscribed circle/sphere (Method,
    Roundness; Background, generic 3D roundness equation).

Readings where the text is silent or garbled (each is listed in the design notes):
  * the printed eccentricities lack a square root; e = sqrt(1 - c^2/a^2) (oblate) and
    e = sqrt(1 - a^2/c^2) (prolate) are the spheroid's eccentricities; at c == a the
    common limit S = 4 pi a^2 is used;
  * "P_o ... calculated from object area" in the 2D passage means P_c;
  * local thickness is a radius; squared values are kept as integers (LT_sq) and
    the radius is sqrt(LT_sq);
  * distances are between voxel centres, balls are open and lattice-centred,
    outside the image is background, and other labels count as background for each
    object (all objects at once, each on its own);
  * the 3D surface shell uses the 6 face neighbours, the analogue of 2D 4-connectivity;
  * mean local thickness is the arithmetic mean of sqrt(LT_sq) over all object voxels.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lt_oracle.c")
_LIB = os.path.join(_HERE, "_lt_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the tier-1 C oracle with gcc (plain -O2, no vectorisation flags)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        p64 = ctypes.POINTER(ctypes.c_int64)
        lib.oracle_edt.argtypes = [p64, ctypes.c_int, p64, p64, p64]
        lib.oracle_edt.restype = ctypes.c_int
        lib.oracle_lt.argtypes = [p64, ctypes.c_int, p64, p64, p64, p64]
        lib.oracle_lt.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p64(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _weights(weights, ndim: int):
    """Squared voxel spacings as an int64 array of ndim positive integers, or None
    for unit spacing."""
    if weights is None:
        return None
    w = np.ascontiguousarray(weights, dtype=np.int64)
    if w.shape != (ndim,) or np.any(w < 1):
        raise ValueError(f"weights must be {ndim} positive integers")
    return w


def _wptr(w):
    return _p64(w) if w is not None else None


# ---------------------------------------------------------------------------
# tier 1 (C): distance transform and local thickness on a whole image
# ---------------------------------------------------------------------------

def edt_sq(labels: np.ndarray, weights=None) -> np.ndarray:
    """Per-label squared EDT: D(p) = min |p - q|^2 over q outside the image or with
    L(q) != L(p); 0 on background.  int64.  With `weights` (the squared voxel
    spacings, ndim positive integers along (z, y, x) or (y, x)) |o|^2 is the weighted
    sum of the squared offsets."""
    lab = np.ascontiguousarray(labels, dtype=np.int64)
    if lab.ndim not in (2, 3):
        raise ValueError("labels must be 2D or 3D")
    w = _weights(weights, lab.ndim)
    out = np.empty(lab.shape, dtype=np.int64)
    shape = np.array(lab.shape, dtype=np.int64)
    if _load().oracle_edt(_p64(lab), lab.ndim, _p64(shape), _wptr(w), _p64(out)) != 0:
        raise RuntimeError("oracle_edt failed")
    return out


def local_thickness_sq(dist_sq: np.ndarray, return_work: bool = False, weights=None):
    """Squared local thickness: LT(p) = max{D(x) : |p - x|^2 < D(x)}; 0 on background
    (|.|^2 weighted as in edt_sq when `weights` is given)."""
    d = np.ascontiguousarray(dist_sq, dtype=np.int64)
    w = _weights(weights, d.ndim)
    out = np.empty(d.shape, dtype=np.int64)
    shape = np.array(d.shape, dtype=np.int64)
    work = np.zeros(1, dtype=np.int64)
    if _load().oracle_lt(_p64(d), d.ndim, _p64(shape), _wptr(w), _p64(out), _p64(work)) != 0:
        raise RuntimeError("oracle_lt failed")
    return (out, int(work[0])) if return_work else out


# ---------------------------------------------------------------------------
# tier 0 (numpy): literal minima / maxima over all pairs, tiny images only
# ---------------------------------------------------------------------------

def edt_sq_brute(labels: np.ndarray, weights=None) -> np.ndarray:
    """Literal D: for every object voxel, the minimum of |p - q|^2 (weighted by the
    squared spacings when given) over all q of the image grown by a one-voxel frame
    (the frame is outside, hence background; a nearest outside point along any
    direction first crosses the frame)."""
    lab = np.asarray(labels)
    w = np.ones(lab.ndim, np.int64) if weights is None else np.asarray(weights, np.int64)
    pad = np.pad(lab.astype(np.int64), 1, constant_values=0)
    qcoords = np.argwhere(np.ones(pad.shape, bool)) - 1          # image coordinates
    qlab = pad.ravel()
    out = np.zeros(lab.shape, dtype=np.int64)
    for p in np.argwhere(lab != 0):
        l = lab[tuple(p)]
        other = qcoords[qlab != l]
        out[tuple(p)] = int((w * (other - p) ** 2).sum(axis=1).min())
    return out


def local_thickness_sq_brute(labels: np.ndarray, dist_sq: np.ndarray, weights=None) -> np.ndarray:
    """Literal LT: for every object voxel p, the maximum D(x) over all x with
    D(x) > 0 and |p - x|^2 < D(x) (weighted as in edt_sq_brute)."""
    lab = np.asarray(labels)
    w = np.ones(lab.ndim, np.int64) if weights is None else np.asarray(weights, np.int64)
    d = np.asarray(dist_sq, dtype=np.int64)
    xs = np.argwhere(d > 0)
    dx = d[tuple(xs.T)]
    out = np.zeros(lab.shape, dtype=np.int64)
    for p in np.argwhere(lab != 0):
        dist2 = (w * (xs - p) ** 2).sum(axis=1)
        cover = dist2 < dx
        out[tuple(p)] = int(dx[cover].max())
    return out


# ---------------------------------------------------------------------------
# shell, per-object sums and closed forms (FP64)
# ---------------------------------------------------------------------------

def shell_mask(labels: np.ndarray) -> np.ndarray:
    """Contour / surface voxels: object voxels with a face neighbour (4 in 2D, 6 in
    3D) that lies outside the image or carries another label (Method, Roundness)."""
    lab = np.asarray(labels)
    pad = np.pad(lab, 1, constant_values=0)
    inner = tuple(slice(1, -1) for _ in range(lab.ndim))
    sh = np.zeros(lab.shape, dtype=bool)
    for ax in range(lab.ndim):
        for step in (-1, 1):
            nb = np.roll(pad, step, axis=ax)[inner]
            sh |= nb != lab
    return sh & (lab != 0)


def object_sums(labels: np.ndarray, lt_sq: np.ndarray, max_label: int | None = None) -> dict:
    """Per-label V, sum of LT radius, max LT_sq, shell count and shell LT sum.

    Arrays are indexed by label value 0..max_label; label 0 is background and its
    entries are zero."""
    lab = np.asarray(labels).astype(np.int64).ravel()
    lt = np.asarray(lt_sq, dtype=np.int64).ravel()
    if max_label is None:
        max_label = int(lab.max()) if lab.size else 0
    n = max_label + 1
    obj = lab != 0
    r = np.sqrt(lt.astype(np.float64))
    sh = shell_mask(np.asarray(labels)).ravel()
    V = np.bincount(lab[obj], minlength=n)[:n].astype(np.int64)
    sum_lt = np.bincount(lab[obj], weights=r[obj], minlength=n)[:n]
    max_lt = np.zeros(n, dtype=np.int64)
    np.maximum.at(max_lt, lab[obj], lt[obj])
    n_sh = np.bincount(lab[sh], minlength=n)[:n].astype(np.int64)
    sum_sh = np.bincount(lab[sh], weights=r[sh], minlength=n)[:n]
    return dict(volume=V, sum_lt=sum_lt, max_lt_sq=max_lt, shell_count=n_sh, shell_sum_lt=sum_sh)


def spheroid_surface(a: float, c: float) -> float:
    """Surface of a spheroid with two equal semi-axes a and third semi-axis c
    (Method, Sphericity: oblate branch c < a, prolate branch c > a; eccentricity
    read with its square root; c == a gives the sphere 4 pi a^2)."""
    if c < a:
        e = math.sqrt(1.0 - (c * c) / (a * a))
        return 2.0 * math.pi * a * a * (1.0 + (1.0 - e * e) / e * math.atanh(e))
    if c > a:
        e = math.sqrt(1.0 - (a * a) / (c * c))
        return 2.0 * math.pi * a * a * (1.0 + c / (a * e) * math.asin(e))
    return 4.0 * math.pi * a * a


def ramanujan_perimeter(a: float, b: float) -> float:
    """Ramanujan's first approximation of an ellipse perimeter (Method, Sphericity)."""
    return math.pi * (3.0 * (a + b) - math.sqrt((3.0 * a + b) * (a + 3.0 * b)))


def sphericity_3d(volume: float, mean_lt: float) -> float:
    """S_LT in 3D: a = mean LT, c = 3V / (4 pi a^2), pi^(1/3) (6V)^(2/3) / S(a, c)."""
    a = mean_lt
    c = 3.0 * volume / (4.0 * math.pi * a * a)
    return math.pi ** (1.0 / 3.0) * (6.0 * volume) ** (2.0 / 3.0) / spheroid_surface(a, c)


def sphericity_2d(area: float, mean_lt: float) -> float:
    """S_LT in 2D: a = mean LT, b = A / (pi a), P_c = 2 sqrt(pi A), P_c / P_o."""
    a = mean_lt
    b = area / (math.pi * a)
    return 2.0 * math.sqrt(math.pi * area) / ramanujan_perimeter(a, b)


def closed_forms(sums: dict, ndim: int, voxel_size: float = 1.0) -> dict:
    """Per-label FP64 mean LT, max LT, shell mean LT, sphericity and roundness.
    Entries with V = 0 (background, absent labels) are NaN.  `voxel_size` is the
    physical volume (area) of one voxel (pixel): with squared spacings w it is
    sqrt(prod w), and V (A) in the sphericity is the voxel count times it; local
    thickness values are already physical lengths."""
    V = sums["volume"].astype(np.float64)              # voxel counts
    Vp = V * float(voxel_size)                         # physical volume (area)
    n = len(V)
    mean_lt = np.full(n, np.nan)
    max_lt = np.full(n, np.nan)
    shell_mean = np.full(n, np.nan)
    sph = np.full(n, np.nan)
    rnd = np.full(n, np.nan)
    for l in range(n):
        if V[l] <= 0:
            continue
        mean_lt[l] = sums["sum_lt"][l] / V[l]
        max_lt[l] = math.sqrt(float(sums["max_lt_sq"][l]))
        if sums["shell_count"][l] > 0:
            shell_mean[l] = sums["shell_sum_lt"][l] / sums["shell_count"][l]
            rnd[l] = shell_mean[l] / max_lt[l]
        sph[l] = (sphericity_3d if ndim == 3 else sphericity_2d)(Vp[l], mean_lt[l])
    return dict(mean_lt=mean_lt, max_lt=max_lt, shell_mean_lt=shell_mean, sphericity=sph,
                roundness=rnd)


def lt_histogram(labels: np.ndarray, lt_sq: np.ndarray, max_lt_sq: np.ndarray) -> np.ndarray:
    """Normalised 32-bin histogram of sqrt(LT_sq) / R per label (R^2 = the object's
    largest LT_sq): bin(p) is the smallest k in 1..32 with 1024 LT_sq(p) <= k^2 R^2,
    decided in integers.  Row l holds the fractions of label l's voxels in bins
    1..32; rows of absent labels are NaN.  (Feature of the learned correction, not
    a quantity of the paper.)"""
    lab = np.asarray(labels).astype(np.int64).ravel()
    lt = np.asarray(lt_sq, dtype=np.int64).ravel()
    n = len(max_lt_sq)
    obj = lab != 0
    l, v = lab[obj], lt[obj]
    r2 = np.asarray(max_lt_sq, dtype=np.int64)[l]
    k = np.arange(1, 33, dtype=np.int64)
    ok = 1024 * v[:, None] <= (k[None, :] ** 2) * r2[:, None]
    bins = np.argmax(ok, axis=1)                    # first k satisfying the test
    counts = np.zeros((n, 32), dtype=np.int64)
    np.add.at(counts, (l, bins), 1)
    V = counts.sum(axis=1)
    out = np.full((n, 32), np.nan)
    out[V > 0] = counts[V > 0] / V[V > 0, None]
    return out


# ---------------------------------------------------------------------------
# roughness-filtered roundness and the 0-1 remap (extensions)
# ---------------------------------------------------------------------------
#
# The Discussion expects the influence of surface roughness on the contour /
# surface roundness to be controllable by filtering the shell values.  The filter
# used here: a shell voxel's LT is replaced by the largest shell LT found within
# half-width w along x, then y, then z (2D: x, then y), each step taking only
# positions that carry the voxel's own label.  Bumps narrower than w lose their
# small inscribed balls to the larger values around them; w = 0 is the paper's
# roundness.  The Results note that the observed minimum can map roundness to the
# standard 0-1 range: R' = (R - m) / (1 - m).

def filtered_shell_lt(labels: np.ndarray, lt_sq: np.ndarray, w: int) -> np.ndarray:
    """F_w: start from LT_sq on shell voxels and 0 elsewhere; along each axis in turn
    (x first, z last) a voxel takes the maximum of the current values at offsets
    -w..w along that axis whose voxel carries its label (outside the image counts as
    no voxel).  Returned on shell voxels (0 elsewhere)."""
    lab = np.asarray(labels).astype(np.int64)
    sh = shell_mask(lab)
    f = np.where(sh, np.asarray(lt_sq, dtype=np.int64), 0)
    for ax in reversed(range(lab.ndim)):                # x (last axis) first
        n = lab.shape[ax]
        out = f.copy()
        for o in range(-w, w + 1):
            if o == 0 or abs(o) >= n:
                continue
            src = [slice(None)] * lab.ndim
            dst = [slice(None)] * lab.ndim
            src[ax] = slice(max(0, o), n + min(0, o))       # position p + o
            dst[ax] = slice(max(0, -o), n - max(0, o))      # position p
            src, dst = tuple(src), tuple(dst)
            same = lab[src] == lab[dst]
            out[dst] = np.where(same, np.maximum(out[dst], f[src]), out[dst])
        f = out
    return np.where(sh & (lab != 0), f, 0)


def filtered_shell_lt_brute(labels: np.ndarray, lt_sq: np.ndarray, w: int) -> np.ndarray:
    """The same filter by its direct reading: for a shell voxel p of label l, the
    largest LT_sq(q) over shell voxels q of label l with |q - p| <= w per axis such
    that the axis-ordered path p -> p + (0,..,dz) -> p + (0, dy, dz) -> q (z step,
    then y, then x; 2D: y then x) stays on voxels of label l at its corners."""
    lab = np.asarray(labels).astype(np.int64)
    lt = np.asarray(lt_sq, dtype=np.int64)
    sh = shell_mask(lab)
    out = np.zeros(lab.shape, dtype=np.int64)
    shape = lab.shape
    rng = range(-w, w + 1)
    for p in np.argwhere(sh):
        p = tuple(int(v) for v in p)
        l = lab[p]
        best = 0
        offs = [(a, b, c) for a in rng for b in rng for c in rng] if lab.ndim == 3 else \
               [(a, b) for a in rng for b in rng]
        for o in offs:
            q = tuple(pi + oi for pi, oi in zip(p, o))
            if any(v < 0 or v >= n for v, n in zip(q, shape)) or not sh[q] or lab[q] != l:
                continue
            # corners of the staircase: change the first axes' coordinates first
            ok = True
            for k in range(1, lab.ndim):
                c = tuple(q[i] if i < k else p[i] for i in range(lab.ndim))
                if lab[c] != l:
                    ok = False
            if ok:
                best = max(best, int(lt[q]))
        out[p] = best
    return out


def filtered_roundness(labels: np.ndarray, lt_sq: np.ndarray, w: int, max_label: int | None = None) -> np.ndarray:
    """Per label: mean over shell voxels of sqrt(F_w) divided by sqrt(max LT_sq);
    NaN for absent labels."""
    lab = np.asarray(labels).astype(np.int64)
    if max_label is None:
        max_label = int(lab.max()) if lab.size else 0
    n = max_label + 1
    F = filtered_shell_lt(lab, lt_sq, w)
    sh = shell_mask(lab).ravel()
    l = lab.ravel()[sh]
    num = np.bincount(l, weights=np.sqrt(F.ravel()[sh].astype(np.float64)), minlength=n)[:n]
    cnt = np.bincount(l, minlength=n)[:n]
    mx = np.zeros(n, dtype=np.int64)
    obj = lab.ravel() != 0
    np.maximum.at(mx, lab.ravel()[obj], np.asarray(lt_sq, dtype=np.int64).ravel()[obj])
    out = np.full(n, np.nan)
    ok = cnt > 0
    out[ok] = num[ok] / cnt[ok] / np.sqrt(mx[ok].astype(np.float64))
    return out


def remap_roundness(r: np.ndarray, r_min: float | None = None) -> np.ndarray:
    """(R - m) / (1 - m) with m the given minimum, or the smallest finite R; NaN
    stays NaN.  When m = 1 every finite R is 1 and maps to 1."""
    r = np.asarray(r, dtype=np.float64)
    fin = np.isfinite(r)
    m = float(r[fin].min()) if r_min is None else float(r_min)
    out = np.full(r.shape, np.nan)
    out[fin] = 1.0 if m >= 1.0 else (r[fin] - m) / (1.0 - m)
    return out


# ---------------------------------------------------------------------------
# whole pipeline
# ---------------------------------------------------------------------------

def object_boxes(labels: np.ndarray):
    """Bounding box (lo, hi exclusive) per present label (scipy find_objects)."""
    from scipy import ndimage
    lab = np.asarray(labels)
    if lab.dtype.kind not in "iu" or lab.dtype.itemsize > 4 or lab.dtype == np.uint32:
        lab = lab.astype(np.int64)
    boxes = {}
    for i, sl in enumerate(ndimage.find_objects(lab)):
        if sl is not None:
            boxes[i + 1] = (tuple(s.start for s in sl), tuple(s.stop for s in sl))
    return boxes


def _crop_fields(lab: np.ndarray, l: int, box, weights=None):
    """D and LT of label l computed on its box grown by one voxel (clipped to the
    image).  Exact: the nearest non-l position of an l voxel always lies in that
    grown box (clamping any nearer candidate into the box keeps it non-l and no
    farther), and every ball covering an l voxel is centred on an l voxel."""
    lo = [max(0, a - 1) for a in box[0]]
    hi = [min(s, b + 1) for b, s in zip(box[1], lab.shape)]
    sl = tuple(slice(a, b) for a, b in zip(lo, hi))
    sub = (lab[sl] == l).astype(np.int64)
    d = edt_sq(sub, weights)
    lt, work = local_thickness_sq(d, return_work=True, weights=weights)
    return sl, sub.astype(bool), d, lt, work


def fields(labels: np.ndarray, per_object: bool | None = None, threads: int | None = None,
           labels_subset=None, weights=None):
    """D and LT for a whole label image, either directly or one object crop at a time
    (threads run crops in parallel; the C calls release the GIL).  With
    ``labels_subset`` only those labels are filled (other voxels stay -1)."""
    lab = np.asarray(labels)
    if per_object is None:
        per_object = lab.size > 64 ** 3 or labels_subset is not None
    if not per_object:
        d = edt_sq(lab, weights)
        lt, work = local_thickness_sq(d, return_work=True, weights=weights)
        return d, lt, work
    boxes = object_boxes(lab)
    todo = sorted(boxes) if labels_subset is None else [int(l) for l in labels_subset]
    fill = 0 if labels_subset is None else -1
    D = np.full(lab.shape, fill, dtype=np.int64)
    LT = np.full(lab.shape, fill, dtype=np.int64)
    works = 0
    with ThreadPoolExecutor(max_workers=threads or os.cpu_count() or 1) as ex:
        for sl, m, d, lt, work in ex.map(lambda l: _crop_fields(lab, l, boxes[l], weights), todo):
            D[sl][m] = d[m]
            LT[sl][m] = lt[m]
            works += work
    return D, LT, works


def measure(labels: np.ndarray, max_label: int | None = None, weights=None, **kw) -> dict:
    """Full oracle pipeline: D, LT, per-label sums and closed forms (FP64).  With
    `weights` (squared voxel spacings) distances are weighted and volumes are
    physical (voxel count times sqrt(prod weights))."""
    lab = np.asarray(labels)
    D, LT, work = fields(lab, weights=weights, **kw)
    sums = object_sums(lab, LT, max_label)
    out = dict(dist_sq=D, lt_sq=LT, ball_work=work)
    out.update(sums)
    vs = 1.0 if weights is None else math.sqrt(float(np.prod(np.asarray(weights, np.float64))))
    out.update(closed_forms(sums, lab.ndim, voxel_size=vs))
    return out
