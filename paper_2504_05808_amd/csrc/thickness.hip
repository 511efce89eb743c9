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
#include <mutex>

#include "lt_internal.h"

namespace lt {

// ------------------------------------------------------------------ small kernels

__global__ void init_label_arrays(int32_t* bb, int32_t* maxd, uint32_t nlab, uint32_t* gmax) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l == 0) *gmax = 0u;
    if (l >= nlab) return;
    for (int k = 0; k < 3; ++k) {
        bb[(2 * k) * nlab + l] = 0x7fffffff;
        bb[(2 * k + 1) * nlab + l] = -1;
    }
    maxd[l] = 0;
}

// Bounding boxes from runs along x, one block per row.  Ballots mark where runs end;
// the first voxel of each run finds its end with bit scans (its own 64-wide chunk,
// else the next chunks' end masks kept in LDS) and updates the six extrema of its
// label.  bb layout: [zmin, zmax, ymin, ymax, xmin, xmax][nlab].
template <typename L>
__global__ void __launch_bounds__(1024)
bbox_runs(const L* __restrict__ lab, int nx, int ny, int nz, uint32_t max_label, int32_t* bb,
          uint32_t nlab, uint32_t* err) {
    __shared__ unsigned long long s_end[ROW_MAX_CHUNKS];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const int chunks = (nx + 63) >> 6;
    const int y = blockIdx.y;
  for (int z = blockIdx.z; z < nz; z += gridDim.z) {
    const L* r = lab + ((size_t)z * ny + y) * nx;
    for (int c = wid; c < chunks; c += nw) {
        const int x = c * 64 + lane;
        bool en = false;
        if (x < nx) en = x == nx - 1 || r[x + 1] != r[x];
        const unsigned long long me = __ballot(en);
        if (lane == 0) s_end[c] = me;
    }
    __syncthreads();
    for (int c = wid; c < chunks; c += nw) {
        const int x = c * 64 + lane;
        if (x >= nx) continue;
        const L l = r[x];
        if (l == 0 || (x > 0 && r[x - 1] == l)) continue;
        if (label_negative(l) || (uint64_t)l > max_label) {
            atomicOr(err, ERR_LABEL);
            continue;
        }
        const unsigned long long above = s_end[c] & ~((1ull << lane) - 1ull);
        int e;
        if (above) {
            e = c * 64 + __ffsll(above) - 1;
        } else {
            int cc = c + 1;
            while (s_end[cc] == 0ull) ++cc;                // the last chunk ends at x = nx - 1
            e = cc * 64 + __ffsll(s_end[cc]) - 1;
        }
        const uint32_t u = (uint32_t)l;
        atomicMin(&bb[0 * nlab + u], z);
        atomicMax(&bb[1 * nlab + u], z);
        atomicMin(&bb[2 * nlab + u], y);
        atomicMax(&bb[3 * nlab + u], y);
        atomicMin(&bb[4 * nlab + u], x);
        atomicMax(&bb[5 * nlab + u], e);
    }
    __syncthreads();                                     // the masks are reused by the next row
  }
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

// ------------------------------------------------------------------ 3D centre prune

// Running maximum of D per label: the lanes of a wave holding the same label fold
// their values first, so one atomic per (wave, label) reaches memory.
__device__ __forceinline__ void wave_label_max(uint32_t l, bool valid, int d, int32_t* maxd) {
    uint64_t active = __ballot(valid);
    while (active) {
        const int lead = __ffsll((unsigned long long)active) - 1;
        const uint32_t L0 = (uint32_t)__shfl((int)l, lead, 64);
        const bool in = valid && l == L0;
        int m = in ? d : 0;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) m = max(m, __shfl_xor(m, off, 64));
        if ((int)(threadIdx.x & 63) == lead) atomicMax(&maxd[L0], m);
        active &= ~__ballot(in);
    }
}

// Largest per-label maximum (the global reach used by the front pass); one block.
__global__ void __launch_bounds__(1024)
max_over_labels(const int32_t* __restrict__ maxd, uint32_t nlab, uint32_t* __restrict__ gmax) {
    __shared__ int s[1024];
    int m = 0;
    for (uint32_t l = threadIdx.x; l < nlab; l += 1024) m = max(m, maxd[l]);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int off = 512; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] = max(s[threadIdx.x], s[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *gmax = (uint32_t)s[0];
}

// One thread per voxel (blocks of 64 x 4 voxels in x, y share neighbour rows in L1):
// background LT = 0; a centre is kept unless a 26-neighbour's open ball contains
// its ball; kd = D for kept centres, 0 elsewhere; per-label and global max D.
template <typename L>
__global__ void __launch_bounds__(256)
prune3d(const L* __restrict__ lab, const int32_t* __restrict__ D, int nx, int ny, int nz,
        uint32_t max_label, const int32_t* __restrict__ tab, int32_t* __restrict__ kd,
        int32_t* __restrict__ lt, int32_t* __restrict__ maxd, uint32_t* err) {
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    const bool inside = x < nx && y < ny;
    const size_t plane = (size_t)ny * nx;
  for (int z = blockIdx.z; z < nz; z += gridDim.z) {
    const size_t i = inside ? (size_t)z * plane + (size_t)y * nx + x : 0;
    const int d = inside ? D[i] : 0;
    bool keep = false;
    uint32_t l = 0;
    if (d > 0) {
        const L raw = lab[i];
        keep = true;
        if (d <= PRUNE_DCAP) {
            const int a1 = tab[d], a2 = tab[(PRUNE_DCAP + 1) + d], a3 = tab[2 * (PRUNE_DCAP + 1) + d];
#pragma unroll
            for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
                for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                    for (int dx = -1; dx <= 1; ++dx) {
                        const int k = dz * dz + dy * dy + dx * dx;
                        if (k == 0) continue;
                        const bool inb = z + dz >= 0 && z + dz < nz && y + dy >= 0 && y + dy < ny &&
                                         x + dx >= 0 && x + dx < nx;
                        const int dn = inb ? D[(ptrdiff_t)i + dz * (ptrdiff_t)plane + dy * nx + dx] : 0;
                        keep = keep && !(dn > (k == 1 ? a1 : (k == 2 ? a2 : a3)));
                    }
        }
        if (keep && d > (int)ZF_D_MASK) atomicOr(err, ERR_OVERFLOW);
        if (label_negative(raw) || (uint64_t)raw > max_label) keep = false;   // flagged elsewhere
        l = (uint32_t)raw;
    }
    if (inside) {
        kd[i] = keep ? d : 0;
        if (d <= 0) lt[i] = 0;
    }
    wave_label_max(l, keep, d, maxd);
  }
}

// ------------------------------------------------------------------ 3D z-fronts

constexpr int FR_CAP = 48;          // kept centres per thread held in LDS

// One thread per (column, chunk of `chunk` slices).  The kept centres of the
// column within the chunk grown by the global reach R are gathered (batched loads)
// into the thread's LDS list in z order; then for each slice of the chunk the
// Pareto front over (value D, residual D - dz^2 > 0) of the centres within reach is
// formed from a sliding window of that list and stored in the front planes.  A
// list that would exceed FR_CAP marks the chunk's fronts as "rescan" (count 7);
// the paint pass then takes every centre of the column instead (same result).
__global__ void __launch_bounds__(256)
fronts3d(const int32_t* __restrict__ kd, int nx, int ny, int nz, int chunk,
         const uint32_t* __restrict__ gmax, uint32_t* __restrict__ zf) {
    __shared__ uint32_t s_list[256 * FR_CAP];
    const int tid = threadIdx.y * 64 + threadIdx.x;
    uint32_t* list = s_list + tid;                 // stride 256: lane-interleaved, no bank conflicts
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= nx || y >= ny) return;
    const int c0 = blockIdx.z * chunk, c1 = min(nz, c0 + chunk);
    const int R = open_reach(max((int)*gmax, 1));
    const int zlo = max(0, c0 - R), zhi = min(nz, c1 + R);
    const size_t plane = (size_t)ny * nx;
    const size_t col = (size_t)y * nx + x;
    const size_t n = plane * nz;
    int cnt = 0;
    bool full = false;
    for (int zb = zlo; zb < zhi; zb += 8) {
        int v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = zb + u < zhi ? kd[(size_t)(zb + u) * plane + col] : 0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (v[u] > 0) {
                if (cnt < FR_CAP) list[cnt * 256] = ((uint32_t)v[u] << CL_Z_BITS) | (uint32_t)(zb + u);
                else full = true;
                ++cnt;
            }
    }
    if (full) {
        for (int z = c0; z < c1; ++z) zf[(size_t)z * plane + col] = 7u << ZF_N_SHIFT;
        return;
    }
    // the column's own reach bounds the window (the gathered range used the global one)
    int Rc = 0;
    for (int j = 0; j < cnt; ++j) Rc = max(Rc, (int)(list[j * 256] >> CL_Z_BITS));
    Rc = cnt ? open_reach(Rc) : 0;
    int lo = 0, hi = 0;
    for (int z = c0; z < c1; ++z) {
        while (hi < cnt && (int)(list[hi * 256] & CL_Z_MASK) <= z + Rc) ++hi;
        while (lo < hi && (int)(list[lo * 256] & CL_Z_MASK) < z - Rc) ++lo;
        Front f;
        front_clear(f);
        for (int j = lo; j < hi; ++j) {
            const uint32_t e = list[j * 256];
            const int dz = z - (int)(e & CL_Z_MASK);
            const int v = (int)(e >> CL_Z_BITS);
            const int b = v - dz * dz;
            if (b > 0) front_insert(f, v, b, dz);
        }
        int m = 0;
        uint32_t p[ZF_PLANES];
#pragma unroll
        for (int k = 0; k < ZF_PLANES; ++k) p[k] = 0u;
#pragma unroll
        for (int k = 0; k < ZF_PLANES; ++k)
            if (f.v[k] != 0) {
                const uint32_t w = zf_pack(f.v[k], f.dz[k]);
#pragma unroll
                for (int q = 0; q < ZF_PLANES; ++q)
                    if (q == m) p[q] = w;
                ++m;
            }
        const size_t i = (size_t)z * plane + col;
        const uint32_t nfield = f.overflow ? 7u : (uint32_t)m;
        zf[i] = m ? (p[0] | (nfield << ZF_N_SHIFT)) : 0u;
#pragma unroll
        for (int q = 1; q < ZF_PLANES; ++q)
            if (m > q) zf[q * n + i] = p[q];
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
    const int y = blockIdx.y;
    const size_t i = (size_t)y * nx + x;
    const int d = x < nx ? D[i] : 0;
    bool keep = false;
    uint32_t l = 0;
    if (d > 0) {
        const L raw = lab[i];
        keep = true;
        if (d <= PRUNE_DCAP) {
            const int a1 = tab[d], a2 = tab[(PRUNE_DCAP + 1) + d];
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const int k = dy * dy + dx * dx;
                    if (k == 0) continue;
                    const bool inb = y + dy >= 0 && y + dy < ny && x + dx >= 0 && x + dx < nx;
                    const int dn = inb ? D[(ptrdiff_t)i + (ptrdiff_t)dy * nx + dx] : 0;
                    keep = keep && !(dn > (k == 1 ? a1 : a2));
                }
        }
        zf[i] = keep ? ((uint32_t)d | 0x80000000u) : 0u;
        if (label_negative(raw) || (uint64_t)raw > max_label) keep = false;
        l = (uint32_t)raw;
    } else if (x < nx) {
        lt[i] = 0;
    }
    wave_label_max(l, keep, d, maxd);              // every lane reaches this call
}

// ------------------------------------------------------------------ planning

// Exclusive scan over labels of the number of paint tiles of each present object.
// toff has nlab + 1 entries; toff[nlab] is the total.  One block of 1024 threads.
__global__ void __launch_bounds__(1024)
plan_tiles(const int32_t* __restrict__ bb, uint32_t nlab, int tile_y, uint32_t* __restrict__ toff,
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
            c = (uint32_t)((by + tile_y - 1) / tile_y) * (uint32_t)((bx + TILE_X - 1) / TILE_X);
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

// open_reach(w) = floor(sqrt(w - 1)) for 1 <= w < REACH_TAB, looked up in LDS.
constexpr int REACH_TAB = 4096;

struct TileCtx {
    uint32_t* M;
    const uint8_t* reach;  // LDS table of open_reach
    int H, W;              // tile extent
    int ty0, tx0;          // tile origin (absolute)
    int lstride;           // words per level = H * TILE_STRIDE
};

__device__ __forceinline__ int reach_of(const TileCtx& t, int w) {
    return w < REACH_TAB ? (int)t.reach[w] : open_reach(w);
}

// Sparse-table update of one interval [xs, xe] (tile-relative, xs <= xe) of row
// `row` with value v: the interval is the union of the two blocks of length 2^k
// starting at xs and ending at xe, k = floor(log2(len)).
__device__ __forceinline__ void paint_interval(const TileCtx& t, int row, int xs, int xe, uint32_t v) {
    const int k = 31 - __clz(xe - xs + 1);
    uint32_t* base = t.M + k * t.lstride + row * TILE_STRIDE;
    atomicMax(base + xs, v);
    atomicMax(base + xe - (1 << k) + 1, v);
}

// Discs held by the lanes in `mask` (all centred in source row sy, at the lane's
// column sx) are painted two at a time: lanes 0..31 take one disc, lanes 32..63 the
// next, and each half sweeps its disc's rows (clipped to the tile) 32 at a time.
__device__ __forceinline__ void paint_mask(const TileCtx& t, uint64_t mask, int v, int b, int sx,
                                           int sy, int lane) {
    const int r = lane & 31;
    const bool upper = lane >= 32;
    while (mask) {
        const int d1 = __ffsll((unsigned long long)mask) - 1;
        mask &= mask - 1;
        int d2 = -1;
        if (mask) {
            d2 = __ffsll((unsigned long long)mask) - 1;
            mask &= mask - 1;
        }
        const int v1 = __builtin_amdgcn_readlane(v, d1), b1 = __builtin_amdgcn_readlane(b, d1);
        const int x1 = __builtin_amdgcn_readlane(sx, d1);
        int v2 = 0, b2 = 0, x2 = 0;
        if (d2 >= 0) {
            v2 = __builtin_amdgcn_readlane(v, d2);
            b2 = __builtin_amdgcn_readlane(b, d2);
            x2 = __builtin_amdgcn_readlane(sx, d2);
        }
        const bool mine = !upper || d2 >= 0;
        const int pv = upper ? v2 : v1, pb = upper ? b2 : b1;
        const int pxr = (upper ? x2 : x1) - t.tx0;          // centre column, tile-relative
        const int h = mine ? reach_of(t, pb) : 0;
        const int dlo = max(-h, t.ty0 - sy);
        const int dhi = mine ? min(h, t.ty0 + t.H - 1 - sy) : dlo - 1;
        const int rowoff = sy - t.ty0;
        for (int dyb = dlo; dyb <= dhi; dyb += 32) {
            const int dy = dyb + r;
            if (dy <= dhi) {
                const int hw = reach_of(t, pb - dy * dy);
                const int xs = max(pxr - hw, 0);
                const int xe = min(pxr + hw, t.W - 1);
                if (xs <= xe) paint_interval(t, rowoff + dy, xs, xe, (uint32_t)pv);
            }
        }
    }
}

template <int NDIM, typename L>
__global__ void __launch_bounds__(PAINT_THREADS)
paint_tiles(const L* __restrict__ lab, const uint32_t* __restrict__ zf,
            const int32_t* __restrict__ kd, const int32_t* __restrict__ bb, const int32_t* __restrict__ maxd,
            const uint32_t* __restrict__ toff, uint32_t nlab, int nx, int ny, int nz, int tile_y,
            uint32_t* __restrict__ counter, int32_t* __restrict__ lt) {
    extern __shared__ uint32_t M[];               // [TILE_LEVELS][tile_y][TILE_STRIDE]
    __shared__ uint32_t s_item;
    __shared__ uint8_t s_reach[REACH_TAB];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int nwaves = blockDim.x >> 6;
    const uint32_t total = toff[nlab];
    const size_t n = (size_t)nx * ny * nz;
    // The table is all zero between slices: every cell a slice uses is cleared by
    // the wave that reads it out.
    for (int q = tid; q < TILE_LEVELS * tile_y * TILE_STRIDE; q += blockDim.x) M[q] = 0u;
    for (int w = tid; w < REACH_TAB; w += blockDim.x) s_reach[w] = (uint8_t)(w > 0 ? open_reach(w) : 0);
    for (;;) {
        if (tid == 0) s_item = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        __syncthreads();
        if (item >= total) break;
        // label: the largest l with toff[l] <= item
        uint32_t lo = 0, hi = nlab;
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
        t.reach = s_reach;
        t.ty0 = y0 + (tt / tiles_x) * tile_y;
        t.tx0 = x0 + (tt % tiles_x) * TILE_X;
        t.H = min(tile_y, y1 - t.ty0);
        t.W = min(TILE_X, x1 - t.tx0);
        t.lstride = t.H * TILE_STRIDE;
        const int sy0 = max(y0, t.ty0 - R), sy1 = min(y1, t.ty0 + t.H + R);
        const int sx0 = max(x0, t.tx0 - R), sx1 = min(x1, t.tx0 + t.W + R);
        const int nlev = 32 - __clz(min(t.W, 2 * R + 1));   // levels 0 .. floor(log2(span))
        for (int pz = (NDIM == 3 ? z0 : 0); pz < (NDIM == 3 ? z1 : 1); ++pz) {
            for (int sy = sy0 + wid; sy < sy1; sy += nwaves) {
                // labels and plane-0 fronts of the whole source row, loaded together
                constexpr int MAXC = 3;                   // source rows span <= 64 + 2 * 64 columns
                L lv[MAXC];
                uint32_t ev[MAXC];
                const size_t rowi = ((size_t)pz * ny + sy) * nx;
#pragma unroll
                for (int c = 0; c < MAXC; ++c) {
                    const int sx = sx0 + c * 64 + lane;
                    const bool in = sx < sx1;
                    lv[c] = in ? lab[rowi + sx] : L(0);
                    ev[c] = in ? zf[rowi + sx] : 0u;
                }
                for (int c = 0; c * 64 < sx1 - sx0; ++c) {
                    const int sx = sx0 + c * 64 + lane;
                    L lc;
                    uint32_t ec;
                    if (c == 0) {
                        lc = lv[0];
                        ec = ev[0];
                    } else if (c == 1) {
                        lc = lv[1];
                        ec = ev[1];
                    } else if (c == 2) {
                        lc = lv[2];
                        ec = ev[2];
                    } else {                              // very wide objects only
                        lc = sx < sx1 ? lab[rowi + sx] : L(0);
                        ec = sx < sx1 ? zf[rowi + sx] : 0u;
                    }
                    const bool own = sx < sx1 && (uint64_t)lc == (uint64_t)l;
                    const uint32_t e0 = own ? ec : 0u;
                    uint32_t e[ZF_PLANES];
                    e[0] = e0;
#pragma unroll
                    for (int q = 1; q < ZF_PLANES; ++q) e[q] = 0u;
                    int nent = 0;
                    bool ovf = false;
                    if (NDIM == 2) {
                        nent = e0 ? 1 : 0;
                    } else if (e0) {
                        const int cc = (int)(e0 >> ZF_N_SHIFT);
                        ovf = cc == 7;
                        nent = ovf ? 0 : cc;
#pragma unroll
                        for (int q = 1; q < ZF_PLANES; ++q)
                            if (nent > q) e[q] = zf[q * n + rowi + sx];
                    }
                    // stored front entries, one disc per lane per pass
#pragma unroll
                    for (int p = 0; p < ZF_PLANES; ++p) {
                        const bool has = p < nent;
                        const uint64_t mask = __ballot(has);
                        if (!mask) break;
                        int v = 0, b = 0;
                        if (has) {
                            if (NDIM == 2) {
                                v = b = (int)(e[p] & 0x7fffffffu);
                            } else {
                                v = (int)(e[p] & ZF_D_MASK);
                                const int dz = (int)((e[p] >> ZF_DZ_SHIFT) & ZF_DZ_MASK) - 512;
                                b = v - dz * dz;
                            }
                        }
                        paint_mask(t, mask, v, b, sx, sy, lane);
                    }
                    // fronts larger than the planes: every kept centre of the column
                    // (within the object's z range) that reaches this slice -- a superset
                    // of the front.  The wave walks the offsets dz = -R..R together, four
                    // independent loads at a time, and paints each offset's discs.
                    if (NDIM == 3 && __ballot(ovf)) {
                        const size_t col = (size_t)sy * nx + sx;
                        const size_t pl = (size_t)nx * ny;
                        for (int d0 = -R; d0 <= R; d0 += 4) {
                            int kv[4];
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const int zc = pz + d0 + u;
                                kv[u] = (ovf && d0 + u <= R && zc >= z0 && zc < z1) ? kd[(size_t)zc * pl + col] : 0;
                            }
#pragma unroll
                            for (int u = 0; u < 4; ++u) {
                                const int dz = d0 + u;
                                const int b = kv[u] - dz * dz;
                                const bool has = kv[u] > 0 && b > 0;
                                const uint64_t mask = __ballot(has);
                                if (mask) paint_mask(t, mask, kv[u], b, sx, sy, lane);
                            }
                        }
                    }
                }
            }
            __syncthreads();
            // push-down of the sparse table, one wave per row: level k-1 at column c
            // takes the blocks of level k starting at c and c - 2^(k-1); then write the
            // painted cells and clear every level of the row
            for (int row = wid; row < t.H; row += nwaves) {
                uint32_t val[TILE_LEVELS];
#pragma unroll
                for (int k = 0; k < TILE_LEVELS; ++k)
                    val[k] = (k < nlev && lane < t.W) ? t.M[k * t.lstride + row * TILE_STRIDE + lane] : 0u;
#pragma unroll
                for (int k = TILE_LEVELS - 1; k >= 1; --k) {
                    if (k < nlev) {
                        const int half = 1 << (k - 1);
                        const uint32_t up = __shfl_up(val[k], (unsigned)half, 64);
                        const uint32_t vk = lane >= half ? max(val[k], up) : val[k];
                        val[k - 1] = max(val[k - 1], vk);
                    }
                }
                if (lane < t.W) {
                    if (val[0]) lt[((size_t)pz * ny + (t.ty0 + row)) * nx + (t.tx0 + lane)] = (int32_t)val[0];
#pragma unroll
                    for (int k = 0; k < TILE_LEVELS; ++k)
                        if (k < nlev) t.M[k * t.lstride + row * TILE_STRIDE + lane] = 0u;
                }
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------------ host side

static inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct ThickLayout {
    size_t bb, maxd, toff, counter, zf, kd, total;
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
    o.kd = at;      at += g.ndim == 3 ? align256(g.n * sizeof(int32_t)) : 0;
    o.total = at;
    return o;
}

size_t thickness_scratch_bytes(const Geom& g, uint32_t max_label) {
    return thick_layout(g, max_label).total;
}

// Tile rows of the paint pass: 64 when the device lets one block hold the 64-row
// table (7 levels x 64 x 65 words = 116,480 B), else 32.
constexpr size_t PAINT_DYN64 = (size_t)TILE_LEVELS * 64 * TILE_STRIDE * sizeof(uint32_t);

int paint_tile_rows(lt_ctx* ctx) {
    const size_t dyn64 = PAINT_DYN64;
    static std::once_flag once;
    std::call_once(once, [] {
        const void* fns[] = {(const void*)paint_tiles<3, uint16_t>, (const void*)paint_tiles<3, int32_t>,
                             (const void*)paint_tiles<3, uint32_t>, (const void*)paint_tiles<2, uint16_t>,
                             (const void*)paint_tiles<2, int32_t>, (const void*)paint_tiles<2, uint32_t>};
        for (const void* f : fns)
            (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)PAINT_DYN64);
    });
    // dynamic table + static reach table and work-item word
    const bool fits64 = ctx->lds_per_block >= dyn64 + REACH_TAB + 64;
    if (ctx->tune.paint_tile_rows == 32) return 32;
    return fits64 ? 64 : 32;
}

template <typename L>
static lt_status thickness_typed(lt_ctx* ctx, const L* lab, const Geom& g, const int32_t* D,
                                 uint32_t max_label, int32_t* lt, void* scratch, hipStream_t s) {
    const ThickLayout lay = thick_layout(g, max_label);
    char* base = (char*)scratch;
    int32_t* bb = (int32_t*)(base + lay.bb);
    int32_t* maxd = (int32_t*)(base + lay.maxd);
    uint32_t* toff = (uint32_t*)(base + lay.toff);
    uint32_t* counter = (uint32_t*)(base + lay.counter);
    uint32_t* zf = (uint32_t*)(base + lay.zf);
    int32_t* kd = (int32_t*)(base + lay.kd);
    uint32_t* gmax = counter + 1;
    const uint32_t nlab = max_label + 1;

    {
        ProfScope _p(ctx, s, "init_label_arrays");
        init_label_arrays<<<(nlab + 255) / 256, 256, 0, s>>>(bb, maxd, nlab, gmax);
    }
    const dim3 block(256);
    const dim3 grid((g.nx + 255) / 256, g.ny, g.nz);
    {
        ProfScope _p(ctx, s, "bbox_runs");
        const int threads = min(1024, ((g.nx + 63) / 64) * 64);
        bbox_runs<L><<<dim3(1, g.ny, loop_extent(g.nz, g.ny, ctx)), threads, 0, s>>>(
            lab, g.nx, g.ny, g.nz, max_label, bb, nlab, ctx->d_err);
    }
    if (g.ndim == 3) {
        const dim3 b2(64, 4);
        {
            ProfScope _p(ctx, s, "prune3d");
            const long pb = (long)((g.nx + 63) / 64) * ((g.ny + 3) / 4);
            prune3d<L><<<dim3((g.nx + 63) / 64, (g.ny + 3) / 4, loop_extent(g.nz, pb, ctx)), b2, 0, s>>>(
                lab, D, g.nx, g.ny, g.nz, max_label, ctx->d_prune3, kd, lt, maxd, ctx->d_err);
        }
        {
            ProfScope _p(ctx, s, "max_over_labels");
            max_over_labels<<<1, 1024, 0, s>>>(maxd, nlab, gmax);
        }
        {
            ProfScope _p(ctx, s, "fronts3d");
            const int chunk = ctx->tune.front_chunk > 0 ? ctx->tune.front_chunk : 64;
            fronts3d<<<dim3((g.nx + 63) / 64, (g.ny + 3) / 4, (g.nz + chunk - 1) / chunk), b2, 0, s>>>(
                kd, g.nx, g.ny, g.nz, chunk, gmax, zf);
        }
    } else {
        ProfScope _p(ctx, s, "pixels2d");
        pixels2d<L><<<dim3((g.nx + 255) / 256, g.ny), block, 0, s>>>(
            lab, D, g.nx, g.ny, max_label, ctx->d_prune2, zf, lt, maxd);
    }
    const int tile_y = paint_tile_rows(ctx);
    {
        ProfScope _p(ctx, s, "plan_tiles");
        plan_tiles<<<1, 1024, 0, s>>>(bb, nlab, tile_y, toff, counter);
    }
    const size_t lds = (size_t)TILE_LEVELS * tile_y * TILE_STRIDE * sizeof(uint32_t);
    // two blocks per CU only when two 32-row tables fit in the LDS
    const size_t per_block = lds + REACH_TAB + 64;
    const int per_cu = (ctx->tune.paint_blocks_per_cu >= 2 && 2 * per_block <= ctx->lds_per_block) ? 2 : 1;
    const int blocks = ctx->n_cu * per_cu;
    {
        ProfScope _p(ctx, s, "paint_tiles");
        if (g.ndim == 3)
            paint_tiles<3, L><<<blocks, PAINT_THREADS, lds, s>>>(lab, zf, kd, bb, maxd, toff,
                                                               nlab, g.nx, g.ny, g.nz, tile_y, counter, lt);
        else
            paint_tiles<2, L><<<blocks, PAINT_THREADS, lds, s>>>(lab, zf, kd, bb, maxd, toff,
                                                               nlab, g.nx, g.ny, 1, tile_y, counter, lt);
    }
    return hip_check(hipGetLastError(), "thickness launch");
}

lt_status launch_thickness(lt_ctx* ctx, const void* labels, lt_dtype dt, const Geom& g,
                           const int32_t* dist_sq, uint32_t max_label, int32_t* lt_sq,
                           void* scratch, hipStream_t s) {
    switch (dt) {
        case LT_U16: return thickness_typed(ctx, (const uint16_t*)labels, g, dist_sq, max_label, lt_sq, scratch, s);
        case LT_I32: return thickness_typed(ctx, (const int32_t*)labels, g, dist_sq, max_label, lt_sq, scratch, s);
        case LT_U32: return thickness_typed(ctx, (const uint32_t*)labels, g, dist_sq, max_label, lt_sq, scratch, s);
    }
    return set_error(LT_E_DTYPE, "unknown dtype");
}

}  // namespace lt
