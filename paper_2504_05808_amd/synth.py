"""Seeded synthetic label images and volumes.

Shapes only: ellipses, ellipsoids, digital balls and superellipsoids with a
value-noise surface perturbation, placed by voxel-level rejection into a label
array (C order, x contiguous, background 0, labels 1..K in placement order).

This module holds none of the distance, thickness or shape-measure arithmetic of
the method.  Both the CPU oracle tests and the GPU tests draw their inputs from
here, so the two sides see identical arrays.  Every generator is a pure function
of its seed (numpy ``Generator(PCG64(seed))``).

Workload recipes (sizes, distributions) stand in for the paper's unavailable
data: Krumbein charts and cell images (2D), and a labelled 400^3 micro-CT volume
of 15,503 fat objects of 27..130,000 voxels (3D; Experiments, Data section).
"""
from __future__ import annotations

import hashlib
import os

import numpy as np

__all__ = [
    "rng_for", "haar_rotation", "ellipse_mask", "ellipsoid_mask", "ball_mask",
    "superellipsoid_mask", "place_objects", "cfg1", "cfg2", "cfg3", "cfg4_volume", "cfg4_batch",
    "cfg4_sizes", "random_labels", "single_object_crops", "CFG3_SHAPE",
]

CFG3_SHAPE = (512, 512, 512)


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def haar_rotation(rng: np.random.Generator, d: int = 3) -> np.ndarray:
    """Uniformly random proper rotation: QR of a Gaussian matrix with sign fix."""
    g = rng.standard_normal((d, d))
    q, r = np.linalg.qr(g)
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


# ---------------------------------------------------------------------------
# local shape masks.  A mask is returned with the integer offset of its [0,0,..]
# element relative to the integer part of the shape centre.
# ---------------------------------------------------------------------------

def ellipse_mask(a: float, b: float, theta: float, frac=(0.0, 0.0)):
    """2D filled ellipse, semi-axes (a, b) rotated by theta; arrays are [y][x]."""
    c, s = np.cos(theta), np.sin(theta)
    rot = np.array([[c, -s], [s, c]])          # columns: ellipse axes in (x, y)
    half = np.abs(rot) @ np.array([a, b])      # extent along x, y
    ext_y, ext_x = int(np.ceil(half[1])) + 1, int(np.ceil(half[0])) + 1
    ys = np.arange(-ext_y, ext_y + 1, dtype=np.float64)[:, None] - frac[0]
    xs = np.arange(-ext_x, ext_x + 1, dtype=np.float64)[None, :] - frac[1]
    u = rot[0, 0] * xs + rot[1, 0] * ys
    v = rot[0, 1] * xs + rot[1, 1] * ys
    m = (u / a) ** 2 + (v / b) ** 2 <= 1.0
    return m, np.array([-ext_y, -ext_x])


def _rotated_coords(rot: np.ndarray, half: np.ndarray, frac):
    ext = np.ceil(half).astype(np.int64) + 1
    z = (np.arange(-ext[0], ext[0] + 1, dtype=np.float32) - np.float32(frac[0]))[:, None, None]
    y = (np.arange(-ext[1], ext[1] + 1, dtype=np.float32) - np.float32(frac[1]))[None, :, None]
    x = (np.arange(-ext[2], ext[2] + 1, dtype=np.float32) - np.float32(frac[2]))[None, None, :]
    r = rot.astype(np.float32)
    # q = R^T (p - c0); p - c0 has components (x, y, z) in R's row order (x, y, z)
    qx = r[0, 0] * x + r[1, 0] * y + r[2, 0] * z
    qy = r[0, 1] * x + r[1, 1] * y + r[2, 1] * z
    qz = r[0, 2] * x + r[1, 2] * y + r[2, 2] * z
    return ext, qx, qy, qz


def ellipsoid_mask(axes, rot, frac=(0.0, 0.0, 0.0)):
    """3D filled ellipsoid with semi-axes (a, b, c) along the rotated x', y', z'."""
    a, b, c = axes
    half = np.abs(rot) @ np.array([a, b, c])            # extent along x, y, z
    ext, qx, qy, qz = _rotated_coords(rot, half[::-1], frac)
    m = (qx / a) ** 2 + (qy / b) ** 2 + (qz / c) ** 2 <= 1.0
    return m, -ext


def ball_mask(r: int):
    """Digital ball {p : |p - c|^2 <= r^2} about an integer centre."""
    k = np.arange(-r - 1, r + 2)
    m = (k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2) <= r * r
    return m, np.array([-r - 1] * 3)


def disc_mask(r: int):
    """Digital disc {p : |p - c|^2 <= r^2} about an integer centre."""
    k = np.arange(-r - 1, r + 2)
    m = (k[:, None] ** 2 + k[None, :] ** 2) <= r * r
    return m, np.array([-r - 1] * 2)


def _value_noise_at(shape, pts, rng: np.random.Generator, cell: int = 6) -> np.ndarray:
    """Value noise in [-1, 1] at integer points ``pts`` (k x 3, local coordinates of a
    grid of ``shape``): U[-1, 1] values on a lattice of spacing ``cell`` covering the
    grid, trilinearly interpolated."""
    nl = [s // cell + 2 for s in shape]
    lat = rng.uniform(-1.0, 1.0, size=nl).astype(np.float32)
    u = pts.astype(np.float32) / np.float32(cell)
    i0 = np.floor(u).astype(np.int64)
    t = u - i0
    out = np.zeros(len(pts), dtype=np.float32)
    for dz in (0, 1):
        wz = t[:, 0] if dz else 1 - t[:, 0]
        for dy in (0, 1):
            wy = t[:, 1] if dy else 1 - t[:, 1]
            for dx in (0, 1):
                wx = t[:, 2] if dx else 1 - t[:, 2]
                out += wz * wy * wx * lat[i0[:, 0] + dz, i0[:, 1] + dy, i0[:, 2] + dx]
    return out


def superellipsoid_mask(axes, eps1: float, eps2: float, rot, amp: float,
                        rng: np.random.Generator, frac=(0.0, 0.0, 0.0), cell: int = 6):
    """Superellipsoid with value-noise radial perturbation.

    Inside iff F(q / s(p)) <= 1 with
    F(q) = (|qx/a|^(2/e2) + |qy/b|^(2/e2))^(e2/e1) + |qz/c|^(2/e1),
    q = R^T (p - c0), s(p) = 1 + amp * n(p) / min(a, b, c), n value noise.
    F is homogeneous of degree 2/e1, so the test is G(q) <= s with G = F^(e1/2).
    """
    a, b, c = axes
    smax = 1.0 + amp / min(a, b, c)
    half = np.abs(rot) @ np.array([a, b, c]) * smax     # along x, y, z
    ext, qx, qy, qz = _rotated_coords(rot, half[::-1], frac)
    with np.errstate(over="ignore", invalid="ignore", divide="ignore"):
        t1 = (np.abs(qx / a) ** (2.0 / eps2) + np.abs(qy / b) ** (2.0 / eps2)) ** (eps2 / eps1)
        f = t1 + np.abs(qz / c) ** (2.0 / eps1)
        g = f ** (eps1 / 2.0)
    m = g <= 1.0
    if amp > 0:
        # s(p) lies in [1 - amp/m, 1 + amp/m]: only that band of G needs the noise
        k = amp / min(a, b, c)
        band = np.argwhere((g > 1.0 - k) & (g <= 1.0 + k))
        n = _value_noise_at(g.shape, band, rng, cell)
        inside = g[band[:, 0], band[:, 1], band[:, 2]] <= 1.0 + np.float32(k) * n
        m[band[:, 0], band[:, 1], band[:, 2]] = inside
    return m, -ext


def _crop_true(mask: np.ndarray, off: np.ndarray):
    idx = np.nonzero(mask)
    if len(idx[0]) == 0:
        return mask, off
    lo = [int(i.min()) for i in idx]
    hi = [int(i.max()) + 1 for i in idx]
    sl = tuple(slice(l, h) for l, h in zip(lo, hi))
    return mask[sl], off + np.array(lo)


def _dilate_faces(mask: np.ndarray) -> np.ndarray:
    """Mask grown by one voxel along each axis (face neighbours), padded by 1."""
    p = np.pad(mask, 1)
    out = p.copy()
    for ax in range(mask.ndim):
        out |= np.roll(p, 1, axis=ax)
        out |= np.roll(p, -1, axis=ax)
    return out


def _hits(vol, vshape, pts) -> bool:
    """True if any in-image point of ``pts`` (k x ndim) is already labelled."""
    inb = np.all((pts >= 0) & (pts < vshape), axis=1)
    p = pts[inb]
    return bool(np.any(vol[tuple(p.T)]))


def place_objects(vol: np.ndarray, shapes, rng: np.random.Generator, *, attempts: int = 100,
                  margin: int = 0, forbid_adjacent: bool = False, label0: int = 1):
    """Place shapes (mask, offset) by rejection; returns the list of placed records.

    Each shape gets up to ``attempts`` uniformly drawn integer positions keeping its
    mask inside [margin, n - 1 - margin] on every axis; a position is accepted when
    none of its voxels (or, with ``forbid_adjacent``, none of its face neighbours)
    is already labelled.  Shapes that find no position are skipped.
    """
    placed = []
    label = label0
    nd = vol.ndim
    for rec in shapes:
        mask, off = _crop_true(rec["mask"], np.asarray(rec["offset"]))
        if mask.sum() == 0:
            continue
        ms = np.array(mask.shape)
        lo = margin - off                     # centre position range such that the
        hi = np.array(vol.shape) - 1 - margin - (off + ms - 1)  # mask stays in range
        if np.any(hi < lo):
            continue
        test = _dilate_faces(mask) if forbid_adjacent else mask
        toff = off - 1 if forbid_adjacent else off
        tpts = np.argwhere(test)                       # local coordinates of tested voxels
        sample = tpts[rng.permutation(len(tpts))[:64]] if len(tpts) > 256 else None
        vshape = np.array(vol.shape)
        ok = False
        for _ in range(attempts):
            c = np.array([rng.integers(l, h + 1) for l, h in zip(lo, hi)])
            o = c + toff
            if sample is not None and _hits(vol, vshape, sample + o):
                continue
            if not _hits(vol, vshape, tpts + o):
                ok = True
                break
        if not ok:
            continue
        o = c + off
        sub = tuple(slice(int(a), int(a + s)) for a, s in zip(o, ms))
        vol[sub][mask] = label
        r = {k: v for k, v in rec.items() if k not in ("mask", "offset")}
        r.update(label=label, origin=tuple(int(v) for v in o), size=tuple(int(v) for v in ms),
                 voxels=int(mask.sum()))
        placed.append(r)
        label += 1
    return placed


def _superellipsoid_params(rng: np.random.Generator):
    axes = rng.uniform(4.0, 30.0, 3)
    e1, e2 = rng.uniform(0.3, 1.0, 2)
    rot = haar_rotation(rng)
    amp = float(rng.uniform(0.0, 2.0))
    frac = rng.uniform(0.0, 1.0, 3)
    return axes, float(e1), float(e2), rot, amp, frac


def _ellipsoid_params(rng, lo=4.0, hi=20.0):
    axes = rng.uniform(lo, hi, 3)
    rot = haar_rotation(rng)
    frac = rng.uniform(0.0, 1.0, 3)
    return axes, rot, frac


# ---------------------------------------------------------------------------
# workload recipes
# ---------------------------------------------------------------------------

def cfg1(seed: int = 1):
    """2D 256x256 int32: 20 ellipses, semi-axes U[5,30], angle U[0,pi);
    no shared and no 4-adjacent pixels; bbox inside [1, 254]."""
    rng = rng_for(seed)
    vol = np.zeros((256, 256), dtype=np.int32)
    shapes = []
    objs = []
    while len(objs) < 20:
        a, b = rng.uniform(5.0, 30.0, 2)
        th = float(rng.uniform(0.0, np.pi))
        frac = rng.uniform(0.0, 1.0, 2)
        m, off = ellipse_mask(a, b, th, frac)
        got = place_objects(vol, [dict(mask=m, offset=off, kind="ellipse", a=float(a),
                                       b=float(b), theta=th)], rng, attempts=200,
                            margin=1, forbid_adjacent=True, label0=len(objs) + 1)
        objs += got
    return vol, dict(name="cfg1", objects=objs, n_objects=len(objs))


def cfg2(seed: int = 2):
    """3D 128^3 int32: 50 rotated ellipsoids (semi-axes U[4,20]) + 10 digital balls
    (r in 5..15, integer centres); non-overlapping and not face-adjacent."""
    rng = rng_for(seed)
    vol = np.zeros((128, 128, 128), dtype=np.int32)
    objs = []
    while len(objs) < 50:
        axes, rot, frac = _ellipsoid_params(rng)
        m, off = ellipsoid_mask(axes, rot, frac)
        objs += place_objects(vol, [dict(mask=m, offset=off, kind="ellipsoid",
                                         axes=[float(v) for v in axes])], rng,
                              attempts=200, forbid_adjacent=True, label0=len(objs) + 1)
    nb = 0
    while nb < 10:
        r = int(rng.integers(5, 16))
        m, off = ball_mask(r)
        got = place_objects(vol, [dict(mask=m, offset=off, kind="ball", r=r)], rng,
                            attempts=200, forbid_adjacent=True, label0=len(objs) + 1)
        objs += got
        nb += len(got)
    return vol, dict(name="cfg2", objects=objs, n_objects=len(objs))


def _cache_path(name: str) -> str | None:
    d = os.environ.get("LT_SYNTH_CACHE", "/tmp/lt_synth_cache")
    if d in ("", "0", "off"):
        return None
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, name)


def _superellipsoid_shapes(rng, n, kinds=("superellipsoid",)):
    for i in range(n):
        kind = kinds[i % len(kinds)]
        if kind == "superellipsoid":
            axes, e1, e2, rot, amp, frac = _superellipsoid_params(rng)
            m, off = superellipsoid_mask(axes, e1, e2, rot, amp, rng, frac)
            yield dict(mask=m, offset=off, kind=kind, axes=[float(v) for v in axes],
                       eps1=e1, eps2=e2, amp=amp)
        else:
            axes = rng.uniform(4.0, 30.0, 3)
            rot = haar_rotation(rng)
            frac = rng.uniform(0.0, 1.0, 3)
            m, off = ellipsoid_mask(axes, rot, frac)
            yield dict(mask=m, offset=off, kind=kind, axes=[float(v) for v in axes])


def _largest_first(shapes):
    """Shapes cropped to their true voxels and ordered by decreasing voxel count, so
    that rejection placement packs a dense volume (large objects go in first)."""
    recs = []
    for r in shapes:
        m, off = _crop_true(r["mask"], np.asarray(r["offset"]))
        r = dict(r, mask=m, offset=off)
        recs.append((-int(m.sum()), len(recs), r))
    recs.sort(key=lambda t: (t[0], t[1]))
    return [r for _, _, r in recs]


def _place_until(vol, rng, n_objects, kinds, batch: int = 250, max_shapes: int | None = None):
    """Draw shapes and place them largest-first with 100 attempts each; when some
    fail, keep drawing further batches (each placed largest-first) until
    ``n_objects`` are placed or ``max_shapes`` (default 2 * n_objects) were drawn."""
    max_shapes = max_shapes or 2 * n_objects
    objs = place_objects(vol, _largest_first(_superellipsoid_shapes(rng, n_objects, kinds)),
                         rng, attempts=100)
    drawn = n_objects
    while len(objs) < n_objects and drawn < max_shapes:
        k = min(batch, max_shapes - drawn)
        more = place_objects(vol, _largest_first(_superellipsoid_shapes(rng, k, kinds)), rng,
                             attempts=100, label0=len(objs) + 1)
        drawn += k
        objs += more[: n_objects - len(objs)]
    # labels beyond n_objects (if the last batch overshot) are cleared
    if len(objs) == n_objects:
        vol[vol > n_objects] = 0
    return objs


def cfg3(seed: int = 3, shape=CFG3_SHAPE, n_objects: int = 2000, dtype=np.uint16,
         use_cache: bool = True):
    """3D 512^3 uint16: ~2000 superellipsoids (semi-axes U[4,30], exponents
    U[0.3,1.0], value-noise amplitude U[0,2] voxels, lattice cell 6), placed largest
    first with at most 100 attempts each; touching allowed, no shared voxels."""
    key = f"cfg3_s{seed}_{'x'.join(map(str, shape))}_{n_objects}_{np.dtype(dtype).name}_v3"
    path = _cache_path(key + ".npz") if use_cache else None
    if path and os.path.exists(path):
        with np.load(path) as z:
            vol = z["vol"]
            n = int(z["n"])
        return vol, dict(name="cfg3", n_objects=n, cached=True)
    rng = rng_for(seed)
    vol = np.zeros(shape, dtype=dtype)
    objs = _place_until(vol, rng, n_objects, ("superellipsoid",))
    if path:
        tmp = path + f".tmp{os.getpid()}.npz"
        np.savez(tmp, vol=vol, n=len(objs))
        os.replace(tmp, path)
    return vol, dict(name="cfg3", objects=objs, n_objects=len(objs))


def cfg4_sizes(seed: int = 4, n_volumes: int = 64, edges=(96, 384), counts=(10, 500)):
    """Per-volume (edge, object count) for the batched workload."""
    rng = rng_for(seed)
    e = rng.integers(edges[0], edges[1] + 1, n_volumes)
    k = rng.integers(counts[0], counts[1] + 1, n_volumes)
    return [(int(a), int(b)) for a, b in zip(e, k)]


def cfg4_volume(i: int, seed: int = 4, n_volumes: int = 64, edges=(96, 384), counts=(10, 500)):
    """Volume i of the batch: cube of edge U{96..384} holding K ~ U{10..500} objects,
    half ellipsoids and half superellipsoids from the 512^3 distribution, uint16.
    Reduced batches (smaller edges / counts) use the same recipe."""
    edge, k = cfg4_sizes(seed, n_volumes, edges, counts)[i]
    rng = rng_for(seed * 100003 + i)
    vol = np.zeros((edge, edge, edge), dtype=np.uint16)
    objs = _place_until(vol, rng, k, ("ellipsoid", "superellipsoid"))
    return vol, dict(name=f"cfg4[{i}]", objects=objs, n_objects=len(objs))


def _cfg4_job(args):
    i, kw = args
    return i, cfg4_volume(i, **kw)[0]


def cfg4_batch(seed: int = 4, n_volumes: int = 64, edges=(96, 384), counts=(10, 500),
               workers: int | None = None):
    """Every volume of the batched workload (``cfg4_volume`` for i = 0..n_volumes-1),
    generated in parallel processes; returns the list in index order."""
    kw = dict(seed=seed, n_volumes=n_volumes, edges=edges, counts=counts)
    jobs = [(i, kw) for i in range(n_volumes)]
    workers = workers or min(16, os.cpu_count() or 1)
    vols = {}
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(workers) as pool:
            for i, v in pool.imap_unordered(_cfg4_job, jobs):
                vols[i] = v
    else:
        for j in jobs:
            i, v = _cfg4_job(j)
            vols[i] = v
    return [vols[i] for i in range(n_volumes)]


def _cfg5_block(args):
    seed, k, n_objects, edge, draws = args
    rng = rng_for(seed * 100003 + k)
    vol = np.zeros((edge, edge, edge), dtype=np.uint16)
    objs = _place_until(vol, rng, n_objects, ("superellipsoid",), max_shapes=draws * n_objects)
    return k, vol, len(objs)


def cfg5_volume(seed: int = 6, edge: int = 1024, n_objects: int = 20000, workers: int | None = None,
                use_cache: bool = True, draws: int = 5, progress=None):
    """Evaluation volume of the learned correction: edge^3 uint32 holding ~n_objects
    objects of the 512^3 distribution.  The volume is built as 4 x 4 x 4 independent
    blocks (each placed like the 512^3 volume with n_objects / 64 objects, seeded per
    block, objects never crossing a block face; at most draws * n_objects / 64 shapes
    drawn per block), generated in parallel processes; labels are numbered block by
    block in block order.  ``progress`` (optional) is called with a line of text as
    blocks complete."""
    key = f"cfg5_s{seed}_{edge}_{n_objects}_d{draws}_v2"
    path = _cache_path(key + ".npz") if use_cache else None
    if path and os.path.exists(path):
        with np.load(path) as z:
            return z["vol"], dict(name="cfg5", n_objects=int(z["n"]), cached=True)
    nb = 4
    h = edge // nb
    jobs = [(seed, k, n_objects // nb ** 3, h, draws) for k in range(nb ** 3)]
    workers = workers or min(16, os.cpu_count() or 1)
    parts = {}

    def done(k, v, n):
        parts[k] = (v, n)
        if progress and (len(parts) % 8 == 0 or len(parts) == len(jobs)):
            progress(f"blocks {len(parts)}/{len(jobs)}")

    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(workers) as pool:
            for k, v, n in pool.imap_unordered(_cfg5_block, jobs):
                done(k, v, n)
    else:
        for j in jobs:
            done(*_cfg5_block(j))
    vol = np.zeros((edge, edge, edge), dtype=np.uint32)
    base = 0
    for k in range(nb ** 3):
        v, n = parts[k]
        z0, y0, x0 = (k // (nb * nb)) * h, ((k // nb) % nb) * h, (k % nb) * h
        sub = v.astype(np.uint32)
        sub[sub != 0] += base
        vol[z0:z0 + h, y0:y0 + h, x0:x0 + h] = sub
        base += n
    if path:
        tmp = path + f".tmp{os.getpid()}.npz"
        np.savez(tmp, vol=vol, n=base)
        os.replace(tmp, path)
    return vol, dict(name="cfg5", n_objects=base)


def random_labels(rng: np.random.Generator, shape, n_labels: int = 4, p_bg: float = 0.3,
                  blob: int = 2, dtype=np.int32):
    """Small random label arrays for brute-force checks: blocky label patches with
    relabelling noise, so that runs, touching labels, border contact and
    multi-component labels all occur."""
    coarse = [max(1, (s + blob - 1) // blob) for s in shape]
    lab = rng.integers(1, n_labels + 1, size=coarse)
    lab = lab.repeat(blob, axis=0)
    for ax in range(1, len(shape)):
        lab = lab.repeat(blob, axis=ax)
    lab = lab[tuple(slice(0, s) for s in shape)]
    noise = rng.random(shape) < 0.15
    lab = np.where(noise, rng.integers(1, n_labels + 1, size=shape), lab)
    lab = np.where(rng.random(shape) < p_bg, 0, lab)
    return lab.astype(dtype)


def single_object_crops(vol: np.ndarray, labels, pad: int = 1):
    """Per-label crop (bbox +- pad, clipped) as a binary-relabelled array: the label
    keeps value 1, every other voxel becomes 0.  Returns (crop, slices)."""
    out = []
    for lab in labels:
        idx = np.nonzero(vol == lab)
        lo = [max(0, int(i.min()) - pad) for i in idx]
        hi = [min(s, int(i.max()) + 1 + pad) for i, s in zip(idx, vol.shape)]
        sl = tuple(slice(a, b) for a, b in zip(lo, hi))
        out.append(((vol[sl] == lab).astype(np.int32), sl))
    return out


def digest(arr: np.ndarray) -> str:
    return hashlib.sha1(np.ascontiguousarray(arr).view(np.uint8)).hexdigest()[:16]
