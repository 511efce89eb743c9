// Exact squared local thickness on gfx950.
//
// LT(p) = max{ D(x) : |p - x|^2 < D(x) } over lattice centres x (open balls of the
// per-label squared distance map D); LT = 0 on background.  The local-thickness
// definition (largest inscribed ball containing the point) is stated in the
// Introduction and the first paragraph of the Method section.
//
// Work is cut without changing the result:
//  1. Centre prune.  A ball whose lattice points all lie inside the open ball of a
//     26-neighbour (8 in 2D) with a larger D never decides a maximum, and the chain
//     of such containments ends at a kept ball, so only kept centres are used.
//     Containment is tested exactly with T_k[d] = max{|q - o|^2 : |q|^2 < d}.
//  2. z-fronts (3D).  For a voxel (z, y, x), the kept centres of its column (y, x)
//     whose ball reaches slice z give pairs (value D(c), residual b = D(c) - dz^2);
//     only the Pareto front over (value, residual) is kept, since a dominated pair
//     is covered by the dominating one in every later step.  A positive residual
//     means the ball holds (z, y, x) itself, so every pair of a front belongs to
//     the label of that voxel.  Fronts are computed by one thread per column walking
//     z (coalesced across x) and stored in up to three dense planes.
//  3. Disc painting.  In slice z, a front pair is a disc of squared radius b around
//     (y, x) carrying value D; each disc row is an interval along x.  Intervals are
//     max-painted into an LDS sparse table (two atomics per interval: the interval
//     is covered by two blocks of length 2^k), and a push-down over the levels
//     yields the per-voxel maximum.
// Work items are (object, 32x64 tile of the object's y-x bounding box) and run
// slice by slice over the object's z extent; the source columns of a tile are the
// tile grown by the object's largest ball reach, clipped to its bounding box.
#include "lt_internal.h"

namespace lt {

// ------------------------------------------------------------------ small kernels

__global__ void init_label_arrays(int32_t* bb, int32_t* maxd, uint32_t nlab) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlab) return;
    for (int k = 0; k < 3; ++k) {
        bb[(2 * k) * nlab + l] = 0x7fffffff;
        bb[(2 * k + 1) * nlab + l] = -1;
    }
    maxd[l] = 0;
}

// Bounding boxes from runs along x: the first voxel of each run scans to its end
// and updates the six extrema of its label.  bb layout: [zmin, zmax, ymin, ymax,
// xmin, xmax][nlab].
template <typename L>
__global__ void __launch_bounds__(256)
bbox_runs(const L* __restrict__ lab, int nx, int ny, uint32_t max_label, int32_t* bb,
          uint32_t nlab, uint32_t* err) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const int y = blockIdx.y, z = blockIdx.z;
    const L* r = lab + ((size_t)z * ny + y) * nx;
    const L l = r[x];
    if (l == 0) return;
    if (x > 0 && r[x - 1] == l) return;
    if (label_negative(l) || (uint64_t)l > max_label) {
        atomicOr(err, ERR_LABEL);
        return;
    }
    int e = x;
    while (e + 1 < nx && r[e + 1] == l) ++e;
    const uint32_t u = (uint32_t)l;
    atomicMin(&bb[0 * nlab + u], z);
    atomicMax(&bb[1 * nlab + u], z);
    atomicMin(&bb[2 * nlab + u], y);
    atomicMax(&bb[3 * nlab + u], y);
    atomicMin(&bb[4 * nlab + u], x);
    atomicMax(&bb[5 * nlab + u], e);
}

// ------------------------------------------------------------------ Pareto fronts

struct Front {
    int v[ZF_PLANES], b[ZF_PLANES], dz[ZF_PLANES];
    int n;
    bool overflow;
};

__device__ __forceinline__ void front_clear(Front& f) {
#pragma unroll
    for (int i = 0; i < ZF_PLANES; ++i) f.v[i] = f.b[i] = f.dz[i] = 0;
    f.n = 0;
    f.overflow = false;
}

// Insert (v, b) unless dominated; drop entries it dominates.  Empty slots hold v = 0,
// which no real pair (v >= 1) is dominated by.
__device__ __forceinline__ void front_insert(Front& f, int v, int b, int dz) {
    bool dom = false;
#pragma unroll
    for (int i = 0; i < ZF_PLANES; ++i) dom |= (f.v[i] >= v && f.b[i] >= b);
    if (dom) return;
#pragma unroll
    for (int i = 0; i < ZF_PLANES; ++i)
        if (f.v[i] != 0 && f.v[i] <= v && f.b[i] <= b) {
            f.v[i] = 0;
            f.b[i] = 0;
        }
    bool placed = false;
#pragma unroll
    for (int i = 0; i < ZF_PLANES; ++i)
        if (!placed && f.v[i] == 0) {
            f.v[i] = v;
            f.b[i] = b;
            f.dz[i] = dz;
            placed = true;
        }
    if (!placed) f.overflow = true;
}

__device__ __forceinline__ uint32_t zf_pack(int v, int dz) {
    return (uint32_t)v | ((uint32_t)(dz + 512) << ZF_DZ_SHIFT);
}

// ------------------------------------------------------------------ 3D column pass

// One thread per (y, x) column.  Walk 1: background LT = 0, centre prune, z-sorted
// list of kept centres, per-label maximum D.  Walk 2: z-front of every object voxel
// of the column from the kept centres within reach.
template <typename L>
__global__ void __launch_bounds__(256)
columns3d(const L* __restrict__ lab, const int32_t* __restrict__ D, int nx, int ny, int nz,
          uint32_t max_label, const int32_t* __restrict__ tab, uint32_t* __restrict__ clist,
          uint32_t* __restrict__ ccount, uint32_t* __restrict__ zf, int32_t* __restrict__ lt,
          int32_t* __restrict__ maxd, uint32_t* err) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const int y = blockIdx.y;
    const size_t plane = (size_t)ny * nx;
    const size_t col = (size_t)y * nx + x;
    const size_t n = plane * nz;
    uint32_t* list = clist + col * nz;
    const int32_t* t1 = tab;
    const int32_t* t2 = tab + (PRUNE_DCAP + 1);
    const int32_t* t3 = tab + 2 * (PRUNE_DCAP + 1);
    int cnt = 0, rmax = 0;
    for (int z = 0; z < nz; ++z) {
        const size_t i = z * plane + col;
        const int d = D[i];
        if (d <= 0) {
            lt[i] = 0;
            continue;
        }
        bool keep = true;
        if (d <= PRUNE_DCAP) {
            const int a1 = t1[d], a2 = t2[d], a3 = t3[d];
            for (int dz = -1; dz <= 1 && keep; ++dz) {
                if (z + dz < 0 || z + dz >= nz) continue;
                for (int dy = -1; dy <= 1 && keep; ++dy) {
                    if (y + dy < 0 || y + dy >= ny) continue;
                    const int32_t* rowp = D + (size_t)(z + dz) * plane + (size_t)(y + dy) * nx;
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int k = dz * dz + dy * dy + dx * dx;
                        if (k == 0 || x + dx < 0 || x + dx >= nx) continue;
                        const int thr = k == 1 ? a1 : (k == 2 ? a2 : a3);
                        if (rowp[x + dx] > thr) {
                            keep = false;
                            break;
                        }
                    }
                }
            }
        }
        if (keep) {
            if (d > (int)ZF_D_MASK) atomicOr(err, ERR_OVERFLOW);
            list[cnt++] = ((uint32_t)d << CL_Z_BITS) | (uint32_t)z;
            rmax = max(rmax, open_reach(d));
            const L l = lab[i];
            if (!label_negative(l) && (uint64_t)l <= max_label) atomicMax(&maxd[(uint32_t)l], d);
        }
    }
    ccount[col] = cnt;

    int lo = 0, hi = 0;
    for (int z = 0; z < nz; ++z) {
        while (hi < cnt && (int)(list[hi] & CL_Z_MASK) <= z + rmax) ++hi;
        while (lo < hi && (int)(list[lo] & CL_Z_MASK) < z - rmax) ++lo;
        const size_t i = z * plane + col;
        if (D[i] <= 0) continue;
        Front f;
        front_clear(f);
        for (int j = lo; j < hi; ++j) {
            const uint32_t e = list[j];
            const int dz = z - (int)(e & CL_Z_MASK);
            const int v = (int)(e >> CL_Z_BITS);
            const int b = v - dz * dz;
            if (b > 0) front_insert(f, v, b, dz);
        }
        // compact to the front of the planes
        int m = 0;
        uint32_t p[ZF_PLANES] = {0u, 0u, 0u};
#pragma unroll
        for (int k = 0; k < ZF_PLANES; ++k)
            if (f.v[k] != 0) {
                const uint32_t w = zf_pack(f.v[k], f.dz[k]);
                if (m == 0) p[0] = w;
                else if (m == 1) p[1] = w;
                else p[2] = w;
                ++m;
            }
        const uint32_t nfield = f.overflow ? 7u : (uint32_t)m;
        zf[i] = m ? (p[0] | (nfield << ZF_N_SHIFT)) : 0u;
        if (m >= 2) zf[n + i] = p[1];
        if (m >= 3) zf[2 * n + i] = p[2];
    }
}

// ------------------------------------------------------------------ 2D pixel pass

// One thread per pixel: background LT = 0, centre prune (8 neighbours), plane 0 =
// D | bit 31 for kept centres (a kept pixel is its own disc), per-label maximum D.
template <typename L>
__global__ void __launch_bounds__(256)
pixels2d(const L* __restrict__ lab, const int32_t* __restrict__ D, int nx, int ny,
         uint32_t max_label, const int32_t* __restrict__ tab, uint32_t* __restrict__ zf,
         int32_t* __restrict__ lt, int32_t* __restrict__ maxd) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= nx) return;
    const int y = blockIdx.y;
    const size_t i = (size_t)y * nx + x;
    const int d = D[i];
    if (d <= 0) {
        lt[i] = 0;
        return;
    }
    bool keep = true;
    if (d <= PRUNE_DCAP) {
        const int a1 = tab[d], a2 = tab[(PRUNE_DCAP + 1) + d];
        for (int dy = -1; dy <= 1 && keep; ++dy) {
            if (y + dy < 0 || y + dy >= ny) continue;
            for (int dx = -1; dx <= 1; ++dx) {
                const int k = dy * dy + dx * dx;
                if (k == 0 || x + dx < 0 || x + dx >= nx) continue;
                if (D[i + (ptrdiff_t)dy * nx + dx] > (k == 1 ? a1 : a2)) {
                    keep = false;
                    break;
                }
            }
        }
    }
    zf[i] = keep ? ((uint32_t)d | 0x80000000u) : 0u;
    if (keep) {
        const L l = lab[i];
        if (!label_negative(l) && (uint64_t)l <= max_label) atomicMax(&maxd[(uint32_t)l], d);
    }
}

// ------------------------------------------------------------------ planning

// Exclusive scan over labels of the number of paint tiles of each present object.
// toff has nlab + 1 entries; toff[nlab] is the total.  One block of 1024 threads.
__global__ void __launch_bounds__(1024)
plan_tiles(const int32_t* __restrict__ bb, uint32_t nlab, uint32_t* __restrict__ toff,
           uint32_t* __restrict__ counter) {
    __shared__ uint32_t s[1024];
    const int t = threadIdx.x;
    uint32_t running = 0;
    for (uint32_t base = 0; base < nlab; base += 1024) {
        const uint32_t l = base + t;
        uint32_t c = 0;
        if (l > 0 && l < nlab && bb[5 * nlab + l] >= 0) {
            const int by = bb[3 * nlab + l] - bb[2 * nlab + l] + 1;
            const int bx = bb[5 * nlab + l] - bb[4 * nlab + l] + 1;
            c = (uint32_t)((by + TILE_Y - 1) / TILE_Y) * (uint32_t)((bx + TILE_X - 1) / TILE_X);
        }
        s[t] = c;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const uint32_t v = t >= off ? s[t - off] : 0u;
            __syncthreads();
            s[t] += v;
            __syncthreads();
        }
        if (l < nlab) toff[l] = running + s[t] - c;
        running += s[1023];
        __syncthreads();
    }
    if (t == 0) {
        toff[nlab] = running;
        *counter = 0;
    }
}

// ------------------------------------------------------------------ painting

struct TileCtx {
    uint32_t* M;
    int H, W;            // tile extent
    int ty0, tx0;        // tile origin (absolute)
};

// Paint the open disc of squared radius b around (sy, sx) with value v, clipped to
// the tile, as one sparse-table update per disc row.
__device__ __forceinline__ void paint_disc(const TileCtx& t, int v, int b, int sy, int sx) {
    const int h = open_reach(b);
    const int dy0 = max(-h, t.ty0 - sy);
    const int dy1 = min(h, t.ty0 + t.H - 1 - sy);
    for (int dy = dy0; dy <= dy1; ++dy) {
        const int hw = open_reach(b - dy * dy);
        const int xs = max(sx - hw, t.tx0) - t.tx0;
        const int xe = min(sx + hw, t.tx0 + t.W - 1) - t.tx0;
        if (xs > xe) continue;
        const int len = xe - xs + 1;
        const int k = 31 - __clz(len);
        uint32_t* base = t.M + ((size_t)k * t.H + (sy + dy - t.ty0)) * t.W;
        atomicMax(base + xs, (uint32_t)v);
        atomicMax(base + xe - (1 << k) + 1, (uint32_t)v);
    }
}

__device__ __forceinline__ void paint_packed(const TileCtx& t, uint32_t e, int sy, int sx) {
    const int v = (int)(e & ZF_D_MASK);
    const int dz = (int)((e >> ZF_DZ_SHIFT) & ZF_DZ_MASK) - 512;
    paint_disc(t, v, v - dz * dz, sy, sx);
}

template <int NDIM, typename L>
__global__ void __launch_bounds__(256)
paint_tiles(const L* __restrict__ lab, const uint32_t* __restrict__ zf,
            const uint32_t* __restrict__ clist, const uint32_t* __restrict__ ccount,
            const int32_t* __restrict__ bb, const int32_t* __restrict__ maxd,
            const uint32_t* __restrict__ toff, uint32_t nlab, int nx, int ny, int nz,
            uint32_t* __restrict__ counter, int32_t* __restrict__ lt) {
    __shared__ uint32_t M[TILE_LEVELS * TILE_Y * TILE_X];
    __shared__ uint32_t s_item;
    const int tid = threadIdx.x;
    const int cx = tid & 63, ry = tid >> 6;
    const uint32_t total = toff[nlab];
    const size_t n = (size_t)nx * ny * nz;
    for (;;) {
        if (tid == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= total) break;
        // label: the largest l with toff[l] <= item
        uint32_t lo = 0, hi = nlab;               // toff[lo] <= item < toff[hi]
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (toff[mid] <= item) lo = mid;
            else hi = mid;
        }
        const uint32_t l = lo;
        const int z0 = bb[0 * nlab + l], z1 = bb[1 * nlab + l] + 1;
        const int y0 = bb[2 * nlab + l], y1 = bb[3 * nlab + l] + 1;
        const int x0 = bb[4 * nlab + l], x1 = bb[5 * nlab + l] + 1;
        const int R = open_reach(max(maxd[l], 1));
        const int tiles_x = (x1 - x0 + TILE_X - 1) / TILE_X;
        const int tt = (int)(item - toff[l]);
        TileCtx t;
        t.M = M;
        t.ty0 = y0 + (tt / tiles_x) * TILE_Y;
        t.tx0 = x0 + (tt % tiles_x) * TILE_X;
        t.H = min(TILE_Y, y1 - t.ty0);
        t.W = min(TILE_X, x1 - t.tx0);
        const int sy0 = max(y0, t.ty0 - R), sy1 = min(y1, t.ty0 + t.H + R);
        const int sx0 = max(x0, t.tx0 - R), sx1 = min(x1, t.tx0 + t.W + R);
        const int span = min(t.W, 2 * R + 1);
        const int nlev = 32 - __clz(span);        // levels 0 .. floor(log2(span))
        const int cells = t.H * t.W;
        for (int pz = (NDIM == 3 ? z0 : 0); pz < (NDIM == 3 ? z1 : 1); ++pz) {
            for (int q = tid; q < nlev * cells; q += 256) M[q] = 0u;
            __syncthreads();
            for (int sy = sy0 + ry; sy < sy1; sy += 4) {
                for (int sx = sx0 + cx; sx < sx1; sx += 64) {
                    const size_t i = ((size_t)pz * ny + sy) * nx + sx;
                    if ((uint64_t)lab[i] != (uint64_t)l) continue;
                    const uint32_t e0 = zf[i];
                    if (e0 == 0u) continue;
                    if (NDIM == 2) {
                        const int v = (int)(e0 & 0x7fffffffu);
                        paint_disc(t, v, v, sy, sx);
                        continue;
                    }
                    const uint32_t cnt = e0 >> ZF_N_SHIFT;
                    paint_packed(t, e0, sy, sx);
                    if (cnt >= 2) paint_packed(t, zf[n + i], sy, sx);
                    if (cnt >= 3) paint_packed(t, zf[2 * n + i], sy, sx);
                    if (cnt == 7) {
                        // front larger than the planes: paint every centre of the
                        // column that reaches this slice (a superset of the front)
                        const size_t c = (size_t)sy * nx + sx;
                        const uint32_t* list = clist + c * nz;
                        const int m = (int)ccount[c];
                        for (int j = 0; j < m; ++j) {
                            const uint32_t e = list[j];
                            const int dz = pz - (int)(e & CL_Z_MASK);
                            const int v = (int)(e >> CL_Z_BITS);
                            if (v - dz * dz > 0) paint_disc(t, v, v - dz * dz, sy, sx);
                        }
                    }
                }
            }
            __syncthreads();
            for (int k = nlev - 1; k >= 1; --k) {
                const int half = 1 << (k - 1);
                if (cx < t.W) {
                    for (int row = ry; row < t.H; row += 4) {
                        const uint32_t* src = M + ((size_t)k * t.H + row) * t.W;
                        uint32_t v = src[cx];
                        if (cx >= half) v = max(v, src[cx - half]);
                        uint32_t* dst = M + ((size_t)(k - 1) * t.H + row) * t.W;
                        dst[cx] = max(dst[cx], v);
                    }
                }
                __syncthreads();
            }
            if (cx < t.W) {
                for (int row = ry; row < t.H; row += 4) {
                    const uint32_t v = M[(size_t)row * t.W + cx];
                    if (v) lt[((size_t)pz * ny + (t.ty0 + row)) * nx + (t.tx0 + cx)] = (int32_t)v;
                }
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ host side

static inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct ThickLayout {
    size_t bb, maxd, toff, counter, zf, clist, ccount, total;
};

static ThickLayout thick_layout(const Geom& g, uint32_t max_label) {
    const size_t nlab = (size_t)max_label + 1;
    ThickLayout o;
    size_t at = 0;
    o.bb = at;      at += align256(6 * nlab * sizeof(int32_t));
    o.maxd = at;    at += align256(nlab * sizeof(int32_t));
    o.toff = at;    at += align256((nlab + 1) * sizeof(uint32_t));
    o.counter = at; at += 256;
    o.zf = at;      at += align256((g.ndim == 3 ? ZF_PLANES : 1) * g.n * sizeof(uint32_t));
    o.clist = at;   at += g.ndim == 3 ? align256(g.n * sizeof(uint32_t)) : 0;
    o.ccount = at;  at += g.ndim == 3 ? align256((size_t)g.ny * g.nx * sizeof(uint32_t)) : 0;
    o.total = at;
    return o;
}

size_t thickness_scratch_bytes(const Geom& g, uint32_t max_label) {
    return thick_layout(g, max_label).total;
}

template <typename L>
static lt_status thickness_typed(lt_ctx* ctx, const L* lab, const Geom& g, const int32_t* D,
                                 uint32_t max_label, int32_t* lt, hipStream_t s) {
    const ThickLayout lay = thick_layout(g, max_label);
    lt_status st = ensure_scratch(ctx, lay.total);
    if (st) return st;
    char* base = (char*)ctx->scratch.ptr;
    int32_t* bb = (int32_t*)(base + lay.bb);
    int32_t* maxd = (int32_t*)(base + lay.maxd);
    uint32_t* toff = (uint32_t*)(base + lay.toff);
    uint32_t* counter = (uint32_t*)(base + lay.counter);
    uint32_t* zf = (uint32_t*)(base + lay.zf);
    uint32_t* clist = (uint32_t*)(base + lay.clist);
    uint32_t* ccount = (uint32_t*)(base + lay.ccount);
    const uint32_t nlab = max_label + 1;

    {
        ProfScope _p(ctx, s, "init_label_arrays");
        init_label_arrays<<<(nlab + 255) / 256, 256, 0, s>>>(bb, maxd, nlab);
    }
    const dim3 block(256);
    const dim3 grid((g.nx + 255) / 256, g.ny, g.nz);
    {
        ProfScope _p(ctx, s, "bbox_runs");
        bbox_runs<L><<<grid, block, 0, s>>>(lab, g.nx, g.ny, max_label, bb, nlab, ctx->d_err);
    }
    if (g.ndim == 3) {
        ProfScope _p(ctx, s, "columns3d");
        columns3d<L><<<dim3((g.nx + 255) / 256, g.ny), block, 0, s>>>(
            lab, D, g.nx, g.ny, g.nz, max_label, ctx->d_prune3, clist, ccount, zf, lt, maxd,
            ctx->d_err);
    } else {
        ProfScope _p(ctx, s, "pixels2d");
        pixels2d<L><<<dim3((g.nx + 255) / 256, g.ny), block, 0, s>>>(
            lab, D, g.nx, g.ny, max_label, ctx->d_prune2, zf, lt, maxd);
    }
    {
        ProfScope _p(ctx, s, "plan_tiles");
        plan_tiles<<<1, 1024, 0, s>>>(bb, nlab, toff, counter);
    }
    const int blocks = ctx->n_cu * 2;
    {
        ProfScope _p(ctx, s, "paint_tiles");
        if (g.ndim == 3)
            paint_tiles<3, L><<<blocks, 256, 0, s>>>(lab, zf, clist, ccount, bb, maxd, toff, nlab,
                                                      g.nx, g.ny, g.nz, counter, lt);
        else
            paint_tiles<2, L><<<blocks, 256, 0, s>>>(lab, zf, clist, ccount, bb, maxd, toff, nlab,
                                                      g.nx, g.ny, 1, counter, lt);
    }
    return hip_check(hipGetLastError(), "thickness launch");
}

lt_status launch_thickness(lt_ctx* ctx, const void* labels, lt_dtype dt, const Geom& g,
                           const int32_t* dist_sq, uint32_t max_label, int32_t* lt_sq,
                           hipStream_t s) {
    switch (dt) {
        case LT_U16: return thickness_typed(ctx, (const uint16_t*)labels, g, dist_sq, max_label, lt_sq, s);
        case LT_I32: return thickness_typed(ctx, (const int32_t*)labels, g, dist_sq, max_label, lt_sq, s);
        case LT_U32: return thickness_typed(ctx, (const uint32_t*)labels, g, dist_sq, max_label, lt_sq, s);
    }
    return set_error(LT_E_DTYPE, "unknown dtype");
}

}  // namespace lt
