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
//     the label of that voxel.  Fronts are computed per column with lanes along z
//     and stored in up to four dense planes; a longer front goes whole to a spill
//     region of its block or to a shared pool (only with no spill space left is the
//     column rescanned by the paint pass); columns with more kept centres than the
//     front pass lists in LDS are finished by a long-list pass.
//  3. Disc painting.  In slice z, a front pair is a disc of squared radius b around
//     (y, x) carrying value D; each disc row is an interval along x.  Intervals are
//     max-painted into an LDS sparse table (two atomics per interval: the interval
//     is covered by two blocks of length 2^k), and a push-down over the levels
//     yields the per-voxel maximum.
//  4. Bands (objects of large reach).  Source groups are taken in bands of a bound
//     on their values, and a group or disc whose bound does not exceed the smallest
//     value already painted over the object's cells of the tile is skipped.
// Work items are (object, 64x64 or 32x64 tile of the object's y-x bounding box) and run
// slice by slice over the object's z extent (objects of large reach: 16 slices per
// item); the source columns of a tile are the tile grown by the object's largest ball
// reach, clipped to its bounding box.
#include <stdlib.h>

#include <mutex>

#include "lt_internal.h"

namespace lt {

// ------------------------------------------------------------------ small kernels

// counter words: [0] paint work items (set by plan_tiles), [1] largest D, [2] long-list
// work items, [3] long-list items taken, [4..5] spill pool words requested (64-bit).
__global__ void init_label_arrays(int32_t* bb, int32_t* maxd, uint32_t nlab, uint32_t* counter, int32_t* colmax,
                                  size_t ncol) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t c = l; c < ncol; c += (size_t)gridDim.x * blockDim.x) colmax[c] = 0;
    if (l < 5) counter[1 + l] = 0u;
    if (l >= nlab) return;
    if (bb) init_box(bb, nlab, l);
    maxd[l] = 0;
}

constexpr int BB_TAB = 128;           // labels per block table
constexpr int BB_ROWS_Y = 16, BB_ROWS_Z = 8;

// Bounding boxes from runs along x.  A block takes BB_ROWS_Y x BB_ROWS_Z rows; each
// wave walks whole rows.  Per row, a first sweep ballots the run ends of every
// 64-voxel chunk (lane c keeps chunk c's mask); a second sweep gives each run's
// first voxel its end (its own chunk's mask, else the first later chunk with an
// end) and merges (z, y, x_first, x_last) into the block's label table with LDS
// atomics.  The table is flushed to the global boxes once per block.
// bb layout: [zmin, zmax, ymin, ymax, xmin, xmax][nlab].
template <typename L>
__global__ void __launch_bounds__(1024)
bbox_runs(const L* __restrict__ lab, int nx, int ny, int nz, uint32_t max_label, int32_t* bb,
          uint32_t nlab, uint32_t* err) {
    __shared__ uint32_t s_key[BB_TAB];
    __shared__ int s_bb[6][BB_TAB];
    const int tid = threadIdx.x;
    for (int t = tid; t < BB_TAB; t += blockDim.x) {
        s_key[t] = 0u;
        s_bb[0][t] = s_bb[2][t] = s_bb[4][t] = 0x7fffffff;
        s_bb[1][t] = s_bb[3][t] = s_bb[5][t] = -1;
    }
    __syncthreads();
    const int lane = tid & 63, wid = __builtin_amdgcn_readfirstlane(tid >> 6), nw = blockDim.x >> 6;
    const int chunks = (nx + 63) >> 6;                   // <= 64
    const int y0 = blockIdx.y * BB_ROWS_Y, z0 = blockIdx.z * BB_ROWS_Z;
    const int rows = BB_ROWS_Y * BB_ROWS_Z;
    for (int r = wid; r < rows; r += nw) {
        const int y = y0 + r % BB_ROWS_Y, z = z0 + r / BB_ROWS_Y;
        if (y >= ny || z >= nz) continue;                // wave-uniform
        const L* row = lab + ((size_t)z * ny + y) * nx;
        unsigned long long mine = 0ull;
        for (int c = 0; c < chunks; ++c) {
            const int x = c * 64 + lane;
            const bool en = x < nx && (x == nx - 1 || row[x + 1] != row[x]);
            const unsigned long long me = __ballot(en);
            if (lane == c) mine = me;
        }
        for (int c = 0; c < chunks; ++c) {
            const int x = c * 64 + lane;
            const L l = x < nx ? row[x] : (L)0;
            bool start = l != 0 && (x == 0 || row[x - 1] != l);
            const unsigned long long cm = __shfl(mine, c, 64);
            const unsigned long long later = __ballot(lane > c && lane < chunks && mine != 0ull);
            const int cc = later ? __ffsll(later) - 1 : c;
            const unsigned long long nm = __shfl(mine, cc, 64);
            if (!start) continue;
            if (label_negative(l) || (uint64_t)l > max_label) {
                atomicOr(err, ERR_LABEL);
                continue;
            }
            const unsigned long long above = cm & ~((1ull << lane) - 1ull);
            const int e = above ? c * 64 + __ffsll(above) - 1 : cc * 64 + __ffsll(nm) - 1;
            const uint32_t u = (uint32_t)l;
            const int slot = lds_slot<BB_TAB>(s_key, u);
            if (slot >= 0) {
                atomicMin(&s_bb[0][slot], z);
                atomicMax(&s_bb[1][slot], z);
                atomicMin(&s_bb[2][slot], y);
                atomicMax(&s_bb[3][slot], y);
                atomicMin(&s_bb[4][slot], x);
                atomicMax(&s_bb[5][slot], e);
            } else {
                atomicMin(&bb[0 * nlab + u], z);
                atomicMax(&bb[1 * nlab + u], z);
                atomicMin(&bb[2 * nlab + u], y);
                atomicMax(&bb[3 * nlab + u], y);
                atomicMin(&bb[4 * nlab + u], x);
                atomicMax(&bb[5 * nlab + u], e);
            }
        }
    }
    __syncthreads();
    for (int t = tid; t < BB_TAB; t += blockDim.x) {
        const uint32_t u = s_key[t];
        if (u == 0u) continue;
        atomicMin(&bb[0 * nlab + u], s_bb[0][t]);
        atomicMax(&bb[1 * nlab + u], s_bb[1][t]);
        atomicMin(&bb[2 * nlab + u], s_bb[2][t]);
        atomicMax(&bb[3 * nlab + u], s_bb[3][t]);
        atomicMin(&bb[4 * nlab + u], s_bb[4][t]);
        atomicMax(&bb[5 * nlab + u], s_bb[5][t]);
    }
}

// ------------------------------------------------------------------ Pareto fronts

__device__ __forceinline__ uint32_t zf_pack(int v, int dz) {
    return (uint32_t)v | ((uint32_t)(dz + 512) << ZF_DZ_SHIFT);
}

// ------------------------------------------------------------------ wave helpers

// Inclusive scans over the 64 lanes of a wave with DPP moves (VALU only, no LDS
// traffic): row_shr by 1, 2, 4, 8 within each row of 16 lanes, then row_bcast:15
// (rows 1 and 3 take the last lane of the row before) and row_bcast:31 (rows 2 and 3
// take lane 31).  Lanes without a source take the identity.
__device__ __forceinline__ int wave_scan_add(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31
    return x;
}

__device__ __forceinline__ uint32_t wave_scan_or(uint32_t x) {
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
    x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
    return x;
}

// Inclusive maximum scan of non-negative values (identity 0, so each step folds into
// one DPP max).
__device__ __forceinline__ int wave_scan_max(int x) {
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false));
    return x;
}

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ------------------------------------------------------------------ 3D centre prune

// Running maximum of D per label: the lanes of a wave holding the same label fold
// their values first, so one atomic per (wave, label) reaches memory.
__device__ __forceinline__ void wave_label_max(uint32_t l, bool valid, int d, int32_t* maxd) {
    uint64_t active = __ballot(valid);
    while (active) {
        const int lead = __ffsll((unsigned long long)active) - 1;
        const uint32_t L0 = (uint32_t)__builtin_amdgcn_readlane((int)l, lead);
        const bool in = valid && l == L0;
        const int m = __builtin_amdgcn_readlane(wave_scan_max(in ? d : 0), 63);
        if ((int)(threadIdx.x & 63) == lead) atomicMax(&maxd[L0], m);
        active &= ~__ballot(in);
    }
}


// One thread per voxel: background LT = 0; a centre is kept unless a 26-neighbour's
// open ball contains its ball; kd = D for kept centres, 0 elsewhere, stored
// column-major ([y][x][z], each column's slices contiguous) for the z-front pass;
// per-label max of the kept D.
constexpr int PR_TY = 4, PR_ZB = 16, PR_W = 66, PR_H = PR_TY + 2, PR_TAB = 64;
constexpr int PR_NT = PR_TY * 64;        // threads per block
constexpr int PR_KS = PR_TY * 64 + 1;    // slice stride of the block's kept-field buffer (odd: no bank conflicts)

// With W (anisotropic spacing) the table has one row per offset class (which of
// z, y, x the offset moves along: 7 classes), since a weighted ball's containment
// depends on the axes, not only on |o|^2.
template <typename L, bool W = false>
__global__ void __launch_bounds__(PR_NT)
prune3d(const L* __restrict__ lab, const int32_t* __restrict__ D, int nx, int ny, int nz,
        uint32_t max_label, const int32_t* __restrict__ tab, int32_t* __restrict__ kd,
        int32_t* __restrict__ lt, int32_t* __restrict__ maxd, int32_t* __restrict__ colmax, uint32_t* err,
        int wz = 1, int wy = 1, int wx = 1) {
    // a block walks PR_ZB consecutive slices of a 64 x PR_TY tile; D of the slices
    // below, at and above the current one (tile + 1 voxel halo) rotate through LDS
    __shared__ int32_t s_d[3][PR_H][PR_W];
    __shared__ int32_t s_kd[PR_ZB * PR_KS];             // kept field of the block, [z][y][x]
    __shared__ uint32_t s_key[PR_TAB];
    __shared__ int s_max[PR_TAB];
    const int tx = threadIdx.x;                                   // 64 x PR_TY: one wave per ty
    const int ty = __builtin_amdgcn_readfirstlane((int)threadIdx.y), tid = ty * 64 + tx;
    const int x0 = blockIdx.x * 64, y0 = blockIdx.y * PR_TY;
    const int x = x0 + tx, y = y0 + ty;
    const bool inside = x < nx && y < ny;
    const size_t plane = (size_t)ny * nx;
    const int zs = blockIdx.z * PR_ZB, ze = min(nz, zs + PR_ZB);
    if (tid < PR_TAB) {
        s_key[tid] = 0u;
        s_max[tid] = 0;
    }
    // each thread moves (at most) two words of a halo plane: loaded into registers
    // one slice ahead, stored to LDS at the top of the next iteration
    constexpr int PR_N = PR_H * PR_W;
    static_assert(2 * PR_NT >= PR_N, "two words per thread cover a halo plane");
    int pv[2];
    auto fetch = [&](int z) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int q = tid + u * PR_NT;
            const int hy = q / PR_W, hx = q - hy * PR_W;
            const int gy = y0 - 1 + hy, gx = x0 - 1 + hx;
            pv[u] = (q < PR_N && z >= 0 && z < nz && gy >= 0 && gy < ny && gx >= 0 && gx < nx)
                        ? D[(size_t)z * plane + (size_t)gy * nx + gx]
                        : 0;
        }
    };
    auto store = [&](int z) {
        const int slot = (z + 3) % 3;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int q = tid + u * PR_NT;
            if (q < PR_N) (&s_d[slot][0][0])[q] = pv[u];
        }
    };
    fetch(zs - 1);
    store(zs - 1);
    fetch(zs);
    store(zs);
    fetch(zs + 1);
    int cmax = 0;                                        // largest kept D of this column's slices
    for (int z = zs; z < ze; ++z) {
        store(z + 1);
        __syncthreads();
        fetch(z + 2);                                    // in flight while slice z is tested
        const int sc = (z + 3) % 3;
        const int d = inside ? s_d[sc][ty + 1][tx + 1] : 0;
        const size_t i = inside ? (size_t)z * plane + (size_t)y * nx + x : 0;
        bool keep = false;
        uint32_t l = 0;
        if (d > 0) {
            const L raw = lab[i];
            keep = true;
            if (!W) {
                // thresholds from the (interleaved) tables, or beyond them the
                // containment bound
                int a1, a2, a3;
                if (d <= PRUNE_DCAP) {
                    const int4 a = ((const int4*)tab)[d];
                    a1 = a.x;
                    a2 = a.y;
                    a3 = a.z;
                } else {
                    a1 = prune_bound(d, 1);
                    a2 = prune_bound(d, 2);
                    a3 = prune_bound(d, 3);
                }
                // largest D over the face, edge and corner neighbours: the centre is
                // dropped when one class exceeds its table value
                int m1 = 0, m2 = 0, m3 = 0;
#pragma unroll
                for (int dz = -1; dz <= 1; ++dz) {
                    const int sl = (z + dz + 3) % 3;
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int k = dz * dz + dy * dy + dx * dx;
                            if (k == 0) continue;
                            const int dn = s_d[sl][ty + 1 + dy][tx + 1 + dx];
                            if (k == 1) m1 = max(m1, dn);
                            else if (k == 2) m2 = max(m2, dn);
                            else m3 = max(m3, dn);
                        }
                }
                keep = m1 <= a1 && m2 <= a2 && m3 <= a3;
            } else {
                // class c = 4 (dz != 0) + 2 (dy != 0) + (dx != 0) - 1
                int mc[7] = {0, 0, 0, 0, 0, 0, 0};
#pragma unroll
                for (int dz = -1; dz <= 1; ++dz) {
                    const int sl = (z + dz + 3) % 3;
#pragma unroll
                    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                        for (int dx = -1; dx <= 1; ++dx) {
                            const int c = 4 * (dz != 0) + 2 * (dy != 0) + (dx != 0) - 1;
                            if (c < 0) continue;
                            mc[c] = max(mc[c], s_d[sl][ty + 1 + dy][tx + 1 + dx]);
                        }
                }
                const bool in_tab = d <= PRUNE_DCAP;
#pragma unroll
                for (int c = 0; c < 7; ++c) {
                    const int b = c + 1;                      // squared weighted length of the class offset
                    const int kw = ((b >> 2) & 1) * wz + ((b >> 1) & 1) * wy + (b & 1) * wx;
                    keep &= mc[c] <= (in_tab ? tab[c * (PRUNE_DCAP + 1) + d] : prune_bound(d, kw));
                }
            }
            if (keep && d > (int)ZF_D_MASK) atomicOr(err, ERR_OVERFLOW);
            if (label_negative(raw) || (uint64_t)raw > max_label) keep = false;   // flagged elsewhere
            l = (uint32_t)raw;
        }
        s_kd[(z - zs) * PR_KS + ty * 64 + tx] = keep ? d : 0;
        if (inside && d <= 0) lt[i] = 0;
        if (keep) cmax = max(cmax, d);
        // per-label largest kept D: wave maxima merged in the block table
        uint64_t active = __ballot(keep);
        while (active) {
            const int lead = __ffsll((unsigned long long)active) - 1;
            const uint32_t L0 = (uint32_t)__builtin_amdgcn_readlane((int)l, lead);
            const bool in = keep && l == L0;
            const int m = __builtin_amdgcn_readlane(wave_scan_max(in ? d : 0), 63);
            if (tx == lead) {
                const int slot = lds_slot<PR_TAB>(s_key, L0);
                if (slot >= 0) atomicMax(&s_max[slot], m);
                else atomicMax(&maxd[L0], m);
            }
            active &= ~__ballot(in);
        }
        __syncthreads();                                 // the slot of z - 1 is reloaded next
    }
    if (tid < PR_TAB && s_key[tid] != 0u) atomicMax(&maxd[s_key[tid]], s_max[tid]);
    if (cmax > 0) atomicMax(&colmax[(size_t)y * nx + x], cmax);
    // the kept field goes out column-major ([y][x][z]): 16 lanes write one column's
    // PR_ZB slices as one contiguous run
#pragma unroll
    for (int it = 0; it < PR_ZB; ++it) {
        const int idx = it * PR_NT + tid;
        const int c = idx / PR_ZB, zo = idx % PR_ZB;     // column of the tile, slice offset
        const int cy = c >> 6, cx = c & 63;
        const int gx = x0 + cx, gy = y0 + cy, gz = zs + zo;
        if (gx < nx && gy < ny && gz < ze)
            kd[((size_t)gy * nx + gx) * nz + gz] = s_kd[zo * PR_KS + cy * 64 + cx];
    }
}

// ------------------------------------------------------------------ 3D z-fronts

constexpr int FZ_CAP = 128;         // listed centres per column (two per lane)
constexpr int FZ_LIST = FZ_CAP + 4; // list words per wave (zero padding for 4-wide reads)
constexpr int FZ_STRIDE = 65;       // output-tile row stride in words (conflict-free columns)
constexpr int FZ_WAVE = 2 * FZ_LIST + FZ_CAP / 4;   // LDS words per wave: list / pairs, D of every fourth

static size_t fronts3d_lds(int chunk) {
    return (size_t)(4 * FZ_WAVE + chunk * FZ_STRIDE) * sizeof(uint32_t);
}

// Pareto front of one column's list at slice z of each lane.  ent holds the entries
// as (zc, A = v - zc^2) by decreasing (D << 11) | zc, padded to cnt4 (a multiple of
// four) with entries no slice takes.  An entry (v, zc) is taken when its residual
// b = v - (z - zc)^2 exceeds maxb, the largest residual taken so far: with
// t = b + z^2 = A + 2 z zc (one 24-bit multiply-add) and the lane's threshold
// mz = maxb + z^2 (INT_MAX: a lane that takes no part) the test is t > mz.  A taken
// entry goes to the front at once: a larger residual of the same D as the lane's
// last member replaces that member (a group of equal D contributes only its largest
// residual; of equal residuals the first, the larger zc, stays), any other is
// appended.  Entries come four at a time (LDS broadcasts); four that no lane takes
// cost one test.  dq[i] holds the D of entry
// 4 i + 3; the wave stops once no lane has maxb below it.  Members go to p, newest first, or with
// SPILL to out[0..k).  Returns the front length k.
// With W the residual is v - wz (z - zc)^2: A = v - wz zc^2, t = A + 2 wz z zc and the
// threshold maxb + wz z^2 (full 32-bit products).
template <bool SPILL, bool W = false>
__device__ __forceinline__ int front_scan(const uint4* ent, const int* dq, int cnt4, int z, bool act,
                                          uint32_t (&p)[ZF_PLANES], uint32_t* out, int wz = 1) {
    const int z2 = W ? 2 * wz * z : 2 * z, zsq = W ? wz * z * z : __mul24(z, z);
    int mz = act ? zsq : INT_MAX;
    int k = 0, lastv = 0;                 // front length, D of the last member
    bool more = true;                     // wave-uniform: a lane with maxb < D
    for (int j = 0; more && j < cnt4; j += 4) {
        const uint4 qa = ent[j >> 1], qb = ent[(j >> 1) + 1];
        const int d4 = dq[j >> 2];
        const int zc[4] = {(int)qa.x, (int)qa.z, (int)qb.x, (int)qb.z};
        const int A[4] = {(int)qa.y, (int)qa.w, (int)qb.y, (int)qb.w};
        int t[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) t[u] = (W ? z2 * zc[u] : __mul24(z2, zc[u])) + A[u];
        if (__ballot(max(max(t[0], t[1]), max(t[2], t[3])) > mz)) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const bool em = t[u] > mz;
                if (__ballot(em)) {       // selects over the whole wave
                    const int v = (W ? wz : 1) * zc[u] * zc[u] + A[u];
                    const bool app = em && lastv != v;
                    const uint32_t w = zf_pack(v, z - zc[u]);
                    if (SPILL) {
                        if (em) out[app ? k : k - 1] = w;
                    } else {
#pragma unroll
                        for (int q = ZF_PLANES - 1; q >= 1; --q) p[q] = app ? p[q - 1] : p[q];
                        p[0] = em ? w : p[0];
                    }
                    k += app ? 1 : 0;
                    lastv = em ? v : lastv;
                    mz = em ? t[u] : mz;
                }
            }
        }
        more = __ballot(mz < d4 + zsq) != 0ull;   // maxb below the D of the fourth
    }
    return k;
}

// Pool space for the lanes with `need` (a front of m words each) that found no room
// in their block's region: one global atomic per wave; a lane whose front fits sets
// at (word offset in the pool) and where = 2.  Called by the whole wave.
__device__ __forceinline__ void pool_take(const SpillPool& pool, bool need, int m, int lane, uint32_t& at,
                                          int& where) {
    if (!__ballot(need)) return;
    const int want = need ? m : 0;
    const int incl = wave_scan_add(want);
    const int tot = __builtin_amdgcn_readlane(incl, 63);
    unsigned long long b = 0ull;
    if (lane == 0) b = atomicAdd(pool.used, (unsigned long long)tot);
    b = ((unsigned long long)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32)) << 32) |
        (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const unsigned long long mine = b + (unsigned long long)(incl - want);
    if (need && mine + (unsigned long long)m <= pool.cap) {
        at = (uint32_t)mine;
        where = 2;
    }
}

// Plane-0 word of a front longer than ZF_PLANES: spilled (block region or pool) or,
// with no spill space or more members than the length field holds, rescan.
__device__ __forceinline__ uint32_t long_front_word(int m, uint32_t at, int where) {
    if (where == 0 || m > ZF_LONG_MAX) return 7u << ZF_N_SHIFT;
    return (7u << ZF_N_SHIFT) | ZF_SPILL | ((uint32_t)m << 16) | (where == 2 ? ZF_POOL : at);
}

// One block per (row y, 64 columns, chunk of `chunk` slices), four waves.  Each
// wave takes whole columns, lanes along z: the column's kept centres within the
// chunk grown by the column's own reach R, read straight from the column-major kept
// field (contiguous along z), are compacted (ballots) into the wave's list when
// their ball reaches a slice of the chunk, ranked by D (each entry's rank counted
// against the whole list) and stored by rank as (zc, D - zc^2) pairs.  For each
// slice (one per lane) a scan of the pairs (front_scan) yields the Pareto front over
// (value D, residual D - dz^2 > 0): by decreasing D, a group of equal D contributes
// its largest residual when that exceeds every residual of larger D; slices no
// listed ball reaches take no part.  A front of up to ZF_PLANES members goes to the
// planes (plane 0 through an LDS tile, written out coalesced along x); a longer one
// is written whole to the block's spill region, or when that is full to the shared
// pool (second scan).  A list longer than FZ_CAP goes to the work list of the
// long-list pass (fronts3d_long), which overwrites the column's slices of the chunk;
// a front that finds no spill space is marked "rescan" (count 7 without ZF_SPILL):
// the paint pass then takes every centre of the column (same result).
template <bool WG = false>
__global__ void __launch_bounds__(256)
fronts3d(const int32_t* __restrict__ kd, int nx, int ny, int nz, int chunk,
         const int32_t* __restrict__ colmax, uint32_t* __restrict__ zf, uint32_t* __restrict__ spill,
         uint32_t* __restrict__ work, uint32_t* __restrict__ nwork, uint32_t wcap, SpillPool pool,
         uint32_t* __restrict__ bmap, uint32_t region_cap, int wz = 1) {
    extern __shared__ __align__(16) uint32_t S[];
    __shared__ int s_cm[64];
    __shared__ int s_bm[128];                         // per slice: bound on the block's front values
    __shared__ uint32_t s_used;                       // words of the block's spill region in use
    const int tid = threadIdx.x, lane = tid & 63;
    const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);    // wave-uniform, in a scalar register
    const int x0 = blockIdx.x * 64, y = blockIdx.y;
    const int W = min(64, nx - x0);
    const int c0 = blockIdx.z * chunk, c1 = min(nz, c0 + chunk);
    const size_t plane = (size_t)ny * nx;
    const size_t n = plane * nz;
    const size_t rowi = (size_t)y * nx + x0;          // column of lane 0
    if (wid == 0) {
        s_cm[lane] = lane < W ? colmax[rowi + lane] : 0;
        if (lane == 0) s_used = 0u;
    }
    if (tid < 128) s_bm[tid] = 0;
    __syncthreads();
    const int zs = c0;                                // first slice of the output tile
    uint32_t* tile = S + 4 * FZ_WAVE;
    uint32_t* list = S + wid * FZ_WAVE;               // compacted keys, then ranked pairs
    int* dq = (int*)(list + 2 * FZ_LIST);             // D of the entries 3, 7, 11, ... by rank
    const uint32_t cap = min((uint32_t)(SPILL_ROW_SLICE * chunk), region_cap);
    uint32_t* region = spill + ((size_t)blockIdx.z * ny + y) * gridDim.x * (size_t)cap + (size_t)blockIdx.x * cap;
    const unsigned long long below = (1ull << lane) - 1ull;
    int bacc0 = 0, bacc1 = 0;                         // the wave's group bounds of slices c0 + lane, + 64
    for (int cx = wid; cx < W; cx += 4) {
        const int cm = __builtin_amdgcn_readfirstlane(s_cm[cx]);
        uint32_t* out = tile + cx;                    // plane-0 words: out[(z - zs) * FZ_STRIDE]
        if (cm == 0) {                                // no kept centre in the column
            for (int z = c0 + lane; z < c1; z += 64) out[(z - zs) * FZ_STRIDE] = 0u;
            continue;
        }
        const size_t col = rowi + cx;
        const int R = WG ? open_reach_w(cm, wz) : open_reach(cm);   // no ball of the column reaches farther
        const int lo = max(0, c0 - R), hi = min(nz, c1 + R);
        int cnt = 0;
        const int32_t* kcol = kd + col * (size_t)nz;  // the column's kept field (column-major)
        for (int zb = lo; zb < hi; zb += 128) {      // two loads in flight per round
            int v[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int z = zb + 64 * u + lane;
                v[u] = z < hi ? kcol[z] : 0;
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                // a centre listed only when its ball reaches a slice of the chunk
                const int z = zb + 64 * u + lane;
                const int d = max(max(c0 - z, z - (c1 - 1)), 0);
                const bool keep = v[u] > (WG ? wz * d * d : __mul24(d, d));
                const unsigned long long m = __ballot(keep);
                if (keep) {
                    const int pos = cnt + __popcll(m & below);
                    if (pos < FZ_CAP) list[pos] = ((uint32_t)v[u] << CL_Z_BITS) | (uint32_t)z;
                }
                cnt += __popcll(m);
            }
        }
        if (cnt > FZ_CAP) {                           // the long-list pass takes the column
            if (lane == 0) {
                const uint32_t k = atomicAdd(nwork, 1u);
                if (k < wcap) work[k] = ((uint32_t)blockIdx.z << 20) | (uint32_t)col;
            }
            for (int z = c0 + lane; z < c1; z += 64) out[(z - zs) * FZ_STRIDE] = 7u << ZF_N_SHIFT;
            bacc0 = max(bacc0, cm);                   // bound for the long-list pass's fronts
            bacc1 = max(bacc1, cm);
            continue;
        }
        if (cnt == 0) {                               // no listed ball reaches the chunk
            for (int z = c0 + lane; z < c1; z += 64) out[(z - zs) * FZ_STRIDE] = 0u;
            continue;
        }
        if (lane < 4) list[cnt + lane] = 0u;          // padding: keys 0 count for no entry
        wave_lds_sync();
        // rank of each entry = number of larger keys (keys are distinct: one z each)
        const uint32_t e0 = lane < cnt ? list[lane] : 0u;
        const uint32_t e1 = lane + 64 < cnt ? list[lane + 64] : 0u;
        int r0 = 0, r1 = 0;
        if (cnt > 64) {                               // two entries per lane
            for (int k = 0; k < cnt; k += 4) {
                const uint4 q = *(const uint4*)(list + k);
                r0 += (q.x > e0) + (q.y > e0) + (q.z > e0) + (q.w > e0);
                r1 += (q.x > e1) + (q.y > e1) + (q.z > e1) + (q.w > e1);
            }
        } else {
            for (int k = 0; k < cnt; k += 4) {
                const uint4 q = *(const uint4*)(list + k);
                r0 += (q.x > e0) + (q.y > e0) + (q.z > e0) + (q.w > e0);
            }
        }
        // the list area now takes the entries by rank as (zc, v - zc^2), padded to a
        // multiple of four with entries no slice takes
        const int cnt4 = (cnt + 3) & ~3;
        uint2* ent = (uint2*)list;
        wave_lds_sync();                              // every lane has read the keys
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint32_t e = h ? e1 : e0;
            const int r = h ? r1 : r0, zc = (int)(e & CL_Z_MASK), v = (int)(e >> CL_Z_BITS);
            if (lane + 64 * h < cnt) {
                ent[r] = make_uint2((uint32_t)zc, (uint32_t)(v - (WG ? wz : 1) * zc * zc));
                if ((r & 3) == 3) dq[r >> 2] = v;
            }
        }
        if (lane < cnt4 - cnt) {                      // padding: never taken, ends the scan
            ent[cnt + lane] = make_uint2(0u, 0xc0000000u);
            if (((cnt + lane) & 3) == 3) dq[(cnt + lane) >> 2] = INT_MIN / 2;
        }
        wave_lds_sync();
        // slices each listed ball reaches, per 64-slice round
        for (int zr = c0; zr < c1; zr += 64) {
            unsigned long long cov = 0ull;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint32_t e = h ? e1 : e0;       // order is free here
                if (lane + 64 * h < cnt) {
                    const int ev = (int)(e >> CL_Z_BITS);
                    const int r = WG ? open_reach_w(ev, wz) : open_reach(ev), zc = (int)(e & CL_Z_MASK);
                    const int a = max(zc - r, zr) - zr, b = min(zc + r, zr + 63) - zr;
                    if (a <= b) {
                        const int len = b - a + 1;
                        cov |= (len == 64 ? ~0ull : ((1ull << len) - 1ull)) << a;
                    }
                }
            }
            const uint32_t clo = (uint32_t)__builtin_amdgcn_readlane((int)wave_scan_or((uint32_t)cov), 63);
            const uint32_t chi = (uint32_t)__builtin_amdgcn_readlane((int)wave_scan_or((uint32_t)(cov >> 32)), 63);
            const int z = zr + lane;
            const bool live = z < c1 && (((lane < 32 ? clo >> lane : chi >> (lane - 32)) & 1u) != 0u);
            uint32_t p[ZF_PLANES];
#pragma unroll
            for (int q = 0; q < ZF_PLANES; ++q) p[q] = 0u;
            int m = 0;
            uint32_t at = 0;
            int where = 0;                            // long front: 1 block region, 2 pool, 0 rescan
            if (__ballot(live)) {
                m = front_scan<false, WG>((const uint4*)ent, dq, cnt4, z, live, p, nullptr, wz);
                if (__ballot(m > ZF_PLANES)) {        // long fronts in the wave
                    if (m > ZF_PLANES) {
                        at = atomicAdd(&s_used, (uint32_t)m);
                        where = at + (uint32_t)m <= cap ? 1 : 0;
                    }
                    pool_take(pool, m > ZF_PLANES && where == 0, m, lane, at, where);
                    const bool again = where != 0;    // second scan: the whole front to the spill
                    if (__ballot(again))
                        front_scan<true, WG>((const uint4*)ent, dq, cnt4, z, again, p,
                                             (where == 2 ? pool.base : region) + at, wz);
                }
            }
            // group bound of this slice: the column's largest kept D (every disc it adds,
            // front or rescan, has no larger value)
            if (m > 0) {
                if (zr == c0) bacc0 = max(bacc0, cm);
                else bacc1 = max(bacc1, cm);
            }
            if (z < c1) {
                uint32_t w0;
                const size_t i = (size_t)z * plane + col;
                if (m > ZF_PLANES) {
                    w0 = long_front_word(m, at, where);
                    if (where == 2) zf[n + i] = at;
                } else {
                    w0 = m ? (p[0] | ((uint32_t)m << ZF_N_SHIFT)) : 0u;
#pragma unroll
                    for (int q = 1; q < ZF_PLANES; ++q)
                        if (m > q) zf[q * n + i] = p[q];
                }
                out[(z - zs) * FZ_STRIDE] = w0;
            }
        }
    }
    if (c0 + lane < c1) atomicMax(&s_bm[lane], bacc0);
    if (c0 + 64 + lane < c1) atomicMax(&s_bm[64 + lane], bacc1);
    __syncthreads();
    for (int q = wid; q < c1 - c0; q += 4)
        if (lane < W) zf[(size_t)(c0 + q) * plane + rowi + lane] = tile[q * FZ_STRIDE + lane];
    for (int q = tid; q < c1 - c0; q += 256)
        bmap[((size_t)(c0 + q) * ny + y) * gridDim.x + blockIdx.x] = (uint32_t)s_bm[q];
}

// Columns whose list outgrew FZ_CAP: the same fronts from a per-wave list that holds
// a whole column (FZ_BIG >= the largest extent), 16 entries per lane.  A persistent
// grid; each wave takes (chunk << 20 | column) items from the front pass's work list
// and rewrites that column's plane-0 words of the chunk (one word per slice, so the
// writes are not coalesced: these columns are few).  Long fronts go to the pool.
constexpr int FZ_BIG = 1024;
constexpr int FZ_BIG_E = FZ_BIG / 64;                // entries per lane
constexpr int FZ_BIG_WAVE = 2 * (FZ_BIG + 4) + FZ_BIG / 4;

static size_t fronts3d_long_lds() { return (size_t)4 * FZ_BIG_WAVE * sizeof(uint32_t); }

template <bool WG = false>
__global__ void __launch_bounds__(256)
fronts3d_long(const int32_t* __restrict__ kd, int nx, int ny, int nz, int chunk,
              const int32_t* __restrict__ colmax, uint32_t* __restrict__ zf, const uint32_t* __restrict__ work,
              const uint32_t* __restrict__ nwork, uint32_t wcap, uint32_t* __restrict__ take, SpillPool pool,
              int wz = 1) {
    extern __shared__ __align__(16) uint32_t S[];
    const int lane = threadIdx.x & 63;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    uint32_t* list = S + wid * FZ_BIG_WAVE;
    int* dq = (int*)(list + 2 * (FZ_BIG + 4));
    const size_t plane = (size_t)ny * nx;
    const size_t n = plane * nz;
    const uint32_t total = min(*nwork, wcap);        // final: the front pass has ended
    if (total == 0u) return;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (;;) {
        uint32_t it = 0u;
        if (lane == 0) it = atomicAdd(take, 1u);
        it = (uint32_t)__builtin_amdgcn_readfirstlane((int)it);
        if (it >= total) break;
        const uint32_t item = work[it];
        const size_t col = item & 0xfffffu;
        const int c0 = (int)(item >> 20) * chunk, c1 = min(nz, c0 + chunk);
        const int cm = colmax[col];
        const int R = WG ? open_reach_w(cm, wz) : open_reach(cm);
        const int lo = max(0, c0 - R), hi = min(nz, c1 + R);
        const int32_t* kcol = kd + col * (size_t)nz;
        int cnt = 0;                                  // <= hi - lo <= nz <= FZ_BIG
        for (int zb = lo; zb < hi; zb += 64) {
            const int z = zb + lane;
            const int v = z < hi ? kcol[z] : 0;
            const int d = max(max(c0 - z, z - (c1 - 1)), 0);
            const bool keep = v > (WG ? wz * d * d : __mul24(d, d));
            const unsigned long long m = __ballot(keep);
            if (keep) list[cnt + __popcll(m & below)] = ((uint32_t)v << CL_Z_BITS) | (uint32_t)z;
            cnt += __popcll(m);
        }
        if (lane < 4) list[cnt + lane] = 0u;
        wave_lds_sync();
        const int nh = (cnt + 63) >> 6;               // wave-uniform: entries held per lane
        uint32_t e[FZ_BIG_E];
        int r[FZ_BIG_E];
#pragma unroll
        for (int h = 0; h < FZ_BIG_E; ++h) {
            e[h] = lane + 64 * h < cnt ? list[lane + 64 * h] : 0u;
            r[h] = 0;
        }
        for (int k = 0; k < cnt; k += 4) {
            const uint4 q = *(const uint4*)(list + k);
#pragma unroll
            for (int h = 0; h < FZ_BIG_E; ++h)
                if (h < nh) r[h] += (q.x > e[h]) + (q.y > e[h]) + (q.z > e[h]) + (q.w > e[h]);
        }
        const int cnt4 = (cnt + 3) & ~3;
        uint2* ent = (uint2*)list;
        wave_lds_sync();
#pragma unroll
        for (int h = 0; h < FZ_BIG_E; ++h) {
            if (lane + 64 * h < cnt) {
                const int zc = (int)(e[h] & CL_Z_MASK), v = (int)(e[h] >> CL_Z_BITS);
                ent[r[h]] = make_uint2((uint32_t)zc, (uint32_t)(v - (WG ? wz : 1) * zc * zc));
                if ((r[h] & 3) == 3) dq[r[h] >> 2] = v;
            }
        }
        if (lane < cnt4 - cnt) {
            ent[cnt + lane] = make_uint2(0u, 0xc0000000u);
            if (((cnt + lane) & 3) == 3) dq[(cnt + lane) >> 2] = INT_MIN / 2;
        }
        wave_lds_sync();
        for (int zr = c0; zr < c1; zr += 64) {
            unsigned long long cov = 0ull;
#pragma unroll
            for (int h = 0; h < FZ_BIG_E; ++h) {
                if (lane + 64 * h < cnt) {
                    const int ev = (int)(e[h] >> CL_Z_BITS);
                    const int rr = WG ? open_reach_w(ev, wz) : open_reach(ev), zc = (int)(e[h] & CL_Z_MASK);
                    const int a = max(zc - rr, zr) - zr, b = min(zc + rr, zr + 63) - zr;
                    if (a <= b) {
                        const int len = b - a + 1;
                        cov |= (len == 64 ? ~0ull : ((1ull << len) - 1ull)) << a;
                    }
                }
            }
            const uint32_t clo = (uint32_t)__builtin_amdgcn_readlane((int)wave_scan_or((uint32_t)cov), 63);
            const uint32_t chi = (uint32_t)__builtin_amdgcn_readlane((int)wave_scan_or((uint32_t)(cov >> 32)), 63);
            const int z = zr + lane;
            const bool live = z < c1 && (((lane < 32 ? clo >> lane : chi >> (lane - 32)) & 1u) != 0u);
            uint32_t p[ZF_PLANES];
#pragma unroll
            for (int q = 0; q < ZF_PLANES; ++q) p[q] = 0u;
            int m = 0;
            uint32_t at = 0;
            int where = 0;
            if (__ballot(live)) {
                m = front_scan<false, WG>((const uint4*)ent, dq, cnt4, z, live, p, nullptr, wz);
                pool_take(pool, m > ZF_PLANES && m <= ZF_LONG_MAX, m, lane, at, where);
                const bool again = where != 0;
                if (__ballot(again))
                    front_scan<true, WG>((const uint4*)ent, dq, cnt4, z, again, p, pool.base + at, wz);
            }
            if (z < c1) {
                const size_t i = (size_t)z * plane + col;
                uint32_t w0;
                if (m > ZF_PLANES) {
                    w0 = long_front_word(m, at, where);
                    if (where == 2) zf[n + i] = at;
                } else {
                    w0 = m ? (p[0] | ((uint32_t)m << ZF_N_SHIFT)) : 0u;
#pragma unroll
                    for (int q = 1; q < ZF_PLANES; ++q)
                        if (m > q) zf[q * n + i] = p[q];
                }
                zf[i] = w0;
            }
        }
        wave_lds_sync();                              // the next item reuses the list
    }
}

// ------------------------------------------------------------------ 2D pixel pass

// One thread per pixel: background LT = 0, centre prune (8 neighbours), plane 0 =
// D | bit 31 for kept centres (a kept pixel is its own disc), per-label maximum D, and
// the banded launch's group bounds (largest kept D per row and 64-column group).
template <typename L, bool W = false>
__global__ void __launch_bounds__(256)
pixels2d(const L* __restrict__ lab, const int32_t* __restrict__ D, int nx, int ny,
         uint32_t max_label, const int32_t* __restrict__ tab, uint32_t* __restrict__ zf,
         int32_t* __restrict__ lt, int32_t* __restrict__ maxd, uint32_t* __restrict__ bmap, int wy = 1,
         int wx = 1) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    const size_t i = (size_t)y * nx + x;
    const int d = x < nx ? D[i] : 0;
    bool keep = false, kept = false;
    uint32_t l = 0;
    if (d > 0) {
        const L raw = lab[i];
        keep = true;
        {
            // classes: unweighted by |o|^2 (edge, corner); with W by the axes moved
            // along (c = 2 (dy != 0) + (dx != 0) - 1); thresholds from the tables, or
            // beyond them the containment bound
            int mc[3] = {0, 0, 0};
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
                for (int dx = -1; dx <= 1; ++dx) {
                    const int k = dy * dy + dx * dx;
                    if (k == 0) continue;
                    const bool inb = y + dy >= 0 && y + dy < ny && x + dx >= 0 && x + dx < nx;
                    const int dn = inb ? D[(ptrdiff_t)i + (ptrdiff_t)dy * nx + dx] : 0;
                    const int c = W ? 2 * (dy != 0) + (dx != 0) - 1 : k - 1;
                    mc[c] = max(mc[c], dn);
                }
            const bool in_tab = d <= PRUNE_DCAP;
            const int k0 = W ? wx : 1, k1 = W ? wy : 2, k2 = wx + wy;
            keep = mc[0] <= (in_tab ? tab[d] : prune_bound(d, k0)) &&
                   mc[1] <= (in_tab ? tab[(PRUNE_DCAP + 1) + d] : prune_bound(d, k1));
            if (W) keep = keep && mc[2] <= (in_tab ? tab[2 * (PRUNE_DCAP + 1) + d] : prune_bound(d, k2));
        }
        zf[i] = keep ? ((uint32_t)d | 0x80000000u) : 0u;
        kept = keep;
        if (label_negative(raw) || (uint64_t)raw > max_label) keep = false;
        l = (uint32_t)raw;
    } else if (x < nx) {
        lt[i] = 0;
    }
    // group bound of the banded paint launch: the largest kept D of the wave's 64 pixels
    // (one row, an aligned group of 64 columns)
    int gb = kept ? d : 0;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) gb = max(gb, __shfl_xor(gb, off, 64));
    if ((threadIdx.x & 63) == 0 && x < nx) bmap[(size_t)y * ((nx + 63) / 64) + (x >> 6)] = (uint32_t)gb;
    wave_label_max(l, keep, d, maxd);              // every lane reaches this call
}

// ------------------------------------------------------------------ planning

// Objects whose balls reach at least this far along y or x are painted by the
// banded launch: value bands with a tile floor (their source region spans several
// tiles' worth of columns).
constexpr int BAND_REACH = 32;
constexpr int BAND_ZCHUNK = 16;      // slices per banded work item (a large object alone fills the chip)
constexpr int NBANDS = 3;            // value bands of the banded launch

// Paint work items of the present objects, split by size: objects whose largest D
// exceeds band_d (balls reaching BAND_REACH or more along y or x) go to toff_big and
// the banded paint launch, one item per (tile, BAND_ZCHUNK slices); the rest go to
// toff, one item per (tile, run of slices): an object of bz slices is cut into
// ceil(bz / PLAIN_ZCHUNK) runs of ceil(bz / runs) slices, the last one shorter.
// Both launches run a persistent grid that takes items in list order, so the lists
// are ordered by estimated cost, longest first, whatever the numbering of the labels
// (list scheduling ends evenly when the long items go first): each present object
// gets a key, the quarter-octave class of its per-item work (slices x rows x columns
// of one item times the reach of its largest ball, plus one); positions are given
// out key by key from the costliest down (in arrival order within a key),
// ord[position] = label, and toff / toff_big are exclusive scans over positions of
// the objects' item counts.  Positions past the present objects hold no items.  toff
// and toff_big have nlab + 1 entries; entry nlab is the total.  One block of 1024
// threads.
constexpr int PLAN_KEYS = 1024;            // one per thread of the block
constexpr int PLAIN_ZCHUNK = 24;

__device__ __forceinline__ void plan_items(const int32_t* __restrict__ bb, const int32_t* __restrict__ maxd,
                                           uint32_t nlab, int tile_y, int band_d, uint32_t l, uint32_t& c,
                                           bool& big, int& key) {
    // every load issued before any test, so that several labels' loads are in flight
    const bool in = l > 0u && l < nlab;
    const uint32_t li = in ? l : 0u;
    const int z0 = bb[0 * nlab + li], z1 = bb[1 * nlab + li];
    const int y0 = bb[2 * nlab + li], y1 = bb[3 * nlab + li];
    const int x0 = bb[4 * nlab + li], x1 = bb[5 * nlab + li];
    const int md = max(maxd[li], 1);
    c = 0u;
    big = false;
    key = 0;
    if (!in || x1 < 0) return;                         // label 0, or absent
    const int bz = z1 - z0 + 1, by = y1 - y0 + 1, bx = x1 - x0 + 1;
    const int ty = (by + tile_y - 1) / tile_y, tx = (bx + TILE_X - 1) / TILE_X;
    c = (uint32_t)(ty * tx);
    big = md > band_d;
    int zi = bz;                                       // slices of one item
    if (big) {
        c *= (uint32_t)((bz + BAND_ZCHUNK - 1) / BAND_ZCHUNK);
        zi = min(bz, BAND_ZCHUNK);
    } else {
        const int nzc = (bz + PLAIN_ZCHUNK - 1) / PLAIN_ZCHUNK;
        c *= (uint32_t)nzc;
        zi = (bz + nzc - 1) / nzc;
    }
    const unsigned long long cost = (unsigned long long)zi * (unsigned long long)((by + ty - 1) / ty) *
                                    (unsigned long long)((bx + tx - 1) / tx) *
                                    (unsigned long long)(open_reach(md) + 1);
    const int e = 63 - __clzll(cost);                  // cost >= 1
    const int frac = (int)((e >= 2 ? cost >> (e - 2) : cost << (2 - e)) & 3ull);
    key = min(PLAN_KEYS - 1, (e << 2) | frac);
}

// Exclusive scan of (a0, a1) over the 1024 threads of the block in thread order (wave
// scans, then the 16 wave totals from LDS); tot0 / tot1 are the block totals.  Every
// thread calls it; it ends with a barrier, so s_w can be used again at once.
__device__ __forceinline__ void plan_block_scan(uint32_t a0, uint32_t a1, uint32_t& e0, uint32_t& e1,
                                                uint32_t& tot0, uint32_t& tot1, uint32_t (*s_w)[16]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t i0 = (uint32_t)wave_scan_add((int)a0), i1 = (uint32_t)wave_scan_add((int)a1);
    if (lane == 63) {
        s_w[0][w] = i0;
        s_w[1][w] = i1;
    }
    __syncthreads();
    uint32_t o0 = 0u, o1 = 0u;
    tot0 = tot1 = 0u;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const uint32_t v0 = s_w[0][q], v1 = s_w[1][q];
        o0 += q < w ? v0 : 0u;
        o1 += q < w ? v1 : 0u;
        tot0 += v0;
        tot1 += v1;
    }
    e0 = o0 + i0 - a0;
    e1 = o1 + i1 - a1;
    __syncthreads();
}

__global__ void __launch_bounds__(1024)
plan_tiles(const int32_t* __restrict__ bb, const int32_t* __restrict__ maxd, uint32_t nlab, int tile_y,
           int band_d, uint32_t* __restrict__ toff, uint32_t* __restrict__ toff_big, uint32_t* __restrict__ ord,
           uint32_t* __restrict__ counter) {
    constexpr int PU = 4;                              // labels per thread per round
    __shared__ uint32_t s_key[PLAN_KEYS];              // objects per key, then the key's next position
    __shared__ uint32_t s_w[2][16];
    __shared__ uint32_t s_np;
    const int t = threadIdx.x;
    s_key[t] = 0u;
    __syncthreads();
    for (uint32_t base = 0; base < nlab; base += PU * 1024) {
        uint32_t c[PU];
        bool big[PU];
        int key[PU];
#pragma unroll
        for (int u = 0; u < PU; ++u) plan_items(bb, maxd, nlab, tile_y, band_d, base + u * 1024 + t, c[u], big[u], key[u]);
#pragma unroll
        for (int u = 0; u < PU; ++u)
            if (c[u]) atomicAdd(&s_key[key[u]], 1u);
    }
    __syncthreads();
    {                                                  // first position of each key, costliest first
        const uint32_t m = s_key[PLAN_KEYS - 1 - t];
        uint32_t e, e_, tot, tot_;
        plan_block_scan(m, 0u, e, e_, tot, tot_, s_w);
        s_key[PLAN_KEYS - 1 - t] = e;
        if (t == 0) s_np = tot;
    }
    __syncthreads();
    for (uint32_t base = 0; base < nlab; base += PU * 1024) {
        uint32_t c[PU];
        bool big[PU];
        int key[PU];
#pragma unroll
        for (int u = 0; u < PU; ++u) plan_items(bb, maxd, nlab, tile_y, band_d, base + u * 1024 + t, c[u], big[u], key[u]);
#pragma unroll
        for (int u = 0; u < PU; ++u)
            if (c[u]) {
                const uint32_t p = atomicAdd(&s_key[key[u]], 1u);
                ord[p] = base + u * 1024 + t;
                toff[p] = big[u] ? 0u : c[u];          // item counts by position, scanned below
                toff_big[p] = big[u] ? c[u] : 0u;
            }
    }
    __syncthreads();                                   // the block's counts are visible to it
    const uint32_t np = s_np;
    uint32_t run0 = 0u, run1 = 0u;                     // the same in every thread
    uint32_t base = 0;
    for (; base < np; base += 1024) {
        const uint32_t p = base + t;
        const uint32_t a0 = p < np ? toff[p] : 0u, a1 = p < np ? toff_big[p] : 0u;
        uint32_t e0, e1, t0, t1;
        plan_block_scan(a0, a1, e0, e1, t0, t1, s_w);
        if (p < nlab) {
            toff[p] = run0 + e0;
            toff_big[p] = run1 + e1;
        }
        run0 += t0;
        run1 += t1;
    }
    for (uint32_t p = base + t; p < nlab; p += 1024) {   // positions past the objects: no items
        toff[p] = run0;
        toff_big[p] = run1;
    }
    if (t == 0) {
        toff[nlab] = run0;
        toff_big[nlab] = run1;
        counter[0] = 0u;                               // work items of the two paint launches
        counter[6] = 0u;
    }
}

// ------------------------------------------------------------------ painting

// open_reach(w) = floor(sqrt(w - 1)) for 1 <= w < REACH_TAB, looked up in LDS.
constexpr int REACH_TAB = 4096;

struct TileCtx {
    uint32_t* M;
    int* disc;             // the wave's disc list in LDS: [4][DL_CAP] (pair end, v, b, x | shift), owner [64]
    const uint8_t* reach;  // LDS table of open_reach
    int H, W;              // tile extent
    int ty0, tx0;          // tile origin (absolute)
    int lstride;           // words per level = H * TILE_STRIDE + 1 (the odd word staggers
                           // the levels over the LDS banks)
    unsigned long long* dirty;   // LDS mask of the tile rows painted in the current slice
    int wy, wx;                  // squared spacings along y and x (anisotropic form)
};

__device__ __forceinline__ int reach_of(const TileCtx& t, int w) {
    return w < REACH_TAB ? (int)t.reach[w] : open_reach(w);
}

// Reach along y (rows a disc of residual b spans) and along x (half-width of the
// interval of residual b on a row): the unit-spacing table, or the weighted reach.
template <bool W>
__device__ __forceinline__ int reach_y(const TileCtx& t, int b) {
    return W ? open_reach_w(b, t.wy) : reach_of(t, b);
}
template <bool W>
__device__ __forceinline__ int reach_x(const TileCtx& t, int b) {
    return W ? open_reach_w(b, t.wx) : reach_of(t, b);
}

// Sparse-table update of one interval [xs, xe] (tile-relative, xs <= xe) of row
// `row` with value v: the interval is the union of the two blocks of length 2^k
// starting at xs and ending at xe, k = floor(log2(len)).
__device__ __forceinline__ void paint_interval(const TileCtx& t, int row, int xs, int xe, uint32_t v) {
    const int k = 31 - __clz(xe - xs + 1);
    uint32_t* base = t.M + __mul24(k, t.lstride) + __mul24(row, TILE_STRIDE);
    atomicMax(base + xs, v);
    atomicMax(base + xe - (1 << k) + 1, v);
}

constexpr int DL_CAP = 128;          // discs per wave list


// Paint the n discs of the wave's list (all centred in source row sy).  Every
// (disc, row) pair clipped to the tile is one interval; the pairs are spread over
// all 64 lanes: each lane sizes two list entries and an inclusive scan over the
// lanes orders the pairs.  For each window of 64 pairs, the entries whose first
// pair falls inside it mark that slot in the wave's owner array; a running maximum
// over the lanes (seeded with the previous window's last owner) then gives each
// lane the entry its pair belongs to.
// In 3D the list may hold discs of several source rows of the wave: bits 19..31
// of an entry's b word hold its source row relative to the tile (+ 4096); in 2D
// (b up to 2^21) every listed disc is centred in source row sy.
template <int NDIM>
__device__ __forceinline__ void disc_unpack(const TileCtx& t, int w, int sy, int& b, int& ro) {
    if (NDIM == 3) {
        b = w & (int)ZF_D_MASK;
        ro = (int)((uint32_t)w >> ZF_D_BITS) - 4096;
    } else {
        b = w;
        ro = sy - t.ty0;
    }
}

template <int NDIM, bool W>
__device__ void disc_flush(const TileCtx& t, int n, int sy, int lane) {
    int* e_end = t.disc;
    int* e_v = t.disc + DL_CAP;
    int* e_b = t.disc + 2 * DL_CAP;
    int* e_x = t.disc + 3 * DL_CAP;
    int* own = t.disc + 4 * DL_CAP;                 // [64]
    wave_lds_sync();
    int cnt[2], dl[2], st[2], local = 0;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int j = 2 * lane + q;
        cnt[q] = 0;
        dl[q] = 0;
        if (j < n) {
            int b, ro;
            disc_unpack<NDIM>(t, e_b[j], sy, b, ro);
            const int h = reach_y<W>(t, b);
            dl[q] = max(-h, -ro);
            const int dhi = min(h, t.H - 1 - ro);
            cnt[q] = max(0, dhi - dl[q] + 1);
        }
        local += cnt[q];
    }
    const int incl = wave_scan_add(local);
    const int total = __builtin_amdgcn_readlane(incl, 63);
    {                                               // rows these discs paint
        unsigned long long rows = 0ull;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int j = 2 * lane + q;
            if (j < n && cnt[q] > 0) {
                int b, ro;
                disc_unpack<NDIM>(t, e_b[j], sy, b, ro);
                const int r0 = ro + dl[q];
                const unsigned long long span = cnt[q] >= 64 ? ~0ull : ((1ull << cnt[q]) - 1ull);
                rows |= span << r0;
            }
        }
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)wave_scan_or((uint32_t)rows), 63);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)wave_scan_or((uint32_t)(rows >> 32)), 63);
        rows = ((unsigned long long)hi << 32) | lo;
        if (lane == 0 && rows) atomicOr(t.dirty, rows);
    }
    int run = incl - local;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int j = 2 * lane + q;
        st[q] = run;
        if (j < n) {
            e_end[j] = run + cnt[q];
            // dy of pair i is i + (dlo - first pair index of the disc)
            e_x[j] = (e_x[j] & 0xfff) | ((dl[q] - run + 16384) << 12);
        }
        run += cnt[q];
    }
    int carry = 0;
    for (int base = 0; base < total; base += 64) {
        own[lane] = 0;                              // entry 0 is the smallest owner anyway
        wave_lds_sync();
#pragma unroll
        for (int q = 0; q < 2; ++q)
            if (cnt[q] > 0 && st[q] >= base && st[q] < base + 64) own[st[q] - base] = 2 * lane + q;
        wave_lds_sync();
        int o = wave_scan_max(own[lane]);
        o = min(max(o, carry), n - 1);
        carry = __builtin_amdgcn_readlane(o, 63);
        const int j = base + lane;
        if (j < total) {
            const int xw = e_x[o];
            const int pxr = (xw & 0xfff) - 2048;
            const int dy = j + (xw >> 12) - 16384;
            int b, ro;
            disc_unpack<NDIM>(t, e_b[o], sy, b, ro);
            const int hw = reach_x<W>(t, b - (W ? t.wy * dy * dy : __mul24(dy, dy)));
            const int xs = max(pxr - hw, 0);
            const int xe = min(pxr + hw, t.W - 1);
            if (xs <= xe) paint_interval(t, ro + dy, xs, xe, (uint32_t)e_v[o]);
        }
        wave_lds_sync();
    }
}

// Append the discs of the lanes with `has` (value v, squared radius b, centre
// column sx) to the wave's list (n: wave-uniform length), painting the list first
// when they would not fit.
template <int NDIM, bool W>
__device__ __forceinline__ void disc_push(const TileCtx& t, int& n, bool has, int v, int b, int sx, int sy,
                                          int lane) {
    const uint64_t m = __ballot(has);
    if (!m) return;
    const int k = __popcll(m);
    if (n + k > DL_CAP) {
        disc_flush<NDIM, W>(t, n, sy, lane);
        n = 0;
    }
    if (has) {
        const int r = n + __popcll(m & ((1ull << lane) - 1ull));
        t.disc[DL_CAP + r] = v;
        t.disc[2 * DL_CAP + r] =
            NDIM == 3 ? (int)((uint32_t)b | ((uint32_t)(sy - t.ty0 + 4096) << ZF_D_BITS)) : b;
        t.disc[3 * DL_CAP + r] = sx - t.tx0 + 2048;        // 12 bits: |sx - tx0| < 2048
    }
    n += k;
}

// With W (anisotropic spacing) the residual of a front entry is v - wz dz^2, discs
// span the rows with wy dy^2 < b and intervals the columns with wx dx^2 < b - wy dy^2;
// the fused shell test reads the face neighbours' labels (D = 1 identifies the
// shell only at unit spacing).
template <int NDIM, typename L, bool W = false, bool BAND = false>
__global__ void __launch_bounds__(PAINT_THREADS)
paint_tiles(const L* __restrict__ lab, const uint32_t* __restrict__ zf,
            const int32_t* __restrict__ kd, const int32_t* __restrict__ bb, const int32_t* __restrict__ maxd,
            const uint32_t* __restrict__ toff, const uint32_t* __restrict__ ord, uint32_t nlab, int nx, int ny,
            int nz, int tile_y,
            uint32_t* __restrict__ counter, int32_t* __restrict__ lt, const uint32_t* __restrict__ spill,
            const uint32_t* __restrict__ pool, const uint32_t* __restrict__ bmap,
            const int32_t* __restrict__ colmax, int chunk, MeasureSums ms, const int32_t* __restrict__ Dmap,
            Spacing spc = Spacing()) {
    // dynamic LDS: the sparse table [TILE_LEVELS][tile_y][TILE_STRIDE], then one disc
    // list per wave
    extern __shared__ uint32_t M[];
    __shared__ uint32_t s_item, s_pos;
    __shared__ unsigned long long s_dirty[2];      // painted rows, by slice parity
    __shared__ int s_floor[2];                     // tile floors of the banded passes
    __shared__ uint8_t s_reach[REACH_TAB];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const int nwaves = blockDim.x >> 6;
    const uint32_t total = toff[nlab];
    if (total == 0u) return;                       // no item for this launch
    const size_t n = (size_t)nx * ny * nz;
    const int ngroups = (nx + 63) / 64;
    // The table is all zero between slices: every cell a slice uses is cleared by
    // the wave that reads it out.
    for (int q = tid; q < TILE_LEVELS * (tile_y * TILE_STRIDE + 1); q += blockDim.x) M[q] = 0u;
    for (int w = tid; w < REACH_TAB; w += blockDim.x) s_reach[w] = (uint8_t)(w > 0 ? open_reach(w) : 0);
    // push-down shifts: level k reads lane - 2^(k-1) (byte index for ds_bpermute);
    // the lanes below that offset read themselves, which leaves their maximum as it is
    uint32_t pd_idx[TILE_LEVELS];
#pragma unroll
    for (int k = 1; k < TILE_LEVELS; ++k) {
        const int half = 1 << (k - 1);
        pd_idx[k] = (uint32_t)(lane >= half ? lane - half : lane) << 2;
    }
    pd_idx[0] = 0u;
    for (;;) {
        if (wid == 0) {
            // next item, and its position in the list: the largest p with toff[p] <= item,
            // by a 64-way search (each round one load per lane narrows the range 64-fold)
            uint32_t item = 0u;
            if (lane == 0) item = atomicAdd(counter, 1u);
            item = (uint32_t)__builtin_amdgcn_readfirstlane((int)item);
            uint32_t lo = 0u;
            if (item < total) {
                uint32_t hi = nlab;                  // toff[lo] <= item < toff[hi]
                while (hi - lo > 1u) {
                    const uint32_t step = (hi - lo + 63u) >> 6;
                    const uint32_t q = lo + (uint32_t)lane * step;
                    const unsigned long long le = __ballot(q < hi && toff[q] <= item);
                    lo += (uint32_t)(63 - __clzll(le)) * step;
                    hi = min(hi, lo + step);
                }
            }
            if (lane == 0) {
                s_item = item;
                s_pos = lo;
                s_dirty[0] = s_dirty[1] = 0ull;
                s_floor[0] = s_floor[1] = INT_MAX;
            }
        }
        __syncthreads();
        const uint32_t item = s_item, pos = s_pos;
        __syncthreads();
        if (item >= total) break;
        const uint32_t l = ord[pos];
        const int z0 = bb[0 * nlab + l], z1 = bb[1 * nlab + l] + 1;
        const int y0 = bb[2 * nlab + l], y1 = bb[3 * nlab + l] + 1;
        const int x0 = bb[4 * nlab + l], x1 = bb[5 * nlab + l] + 1;
        const int mdl = max(maxd[l], 1);
        const int R = W ? 0 : open_reach(mdl);
        const int Rz = W ? open_reach_w(mdl, spc.wz) : R;     // reach of the object's balls per axis
        const int Ry = W ? open_reach_w(mdl, spc.wy) : R;
        const int Rx = W ? open_reach_w(mdl, spc.wx) : R;
        const int tiles_x = (x1 - x0 + TILE_X - 1) / TILE_X;
        int tt = (int)(item - toff[pos]);
        int pz0 = NDIM == 3 ? z0 : 0, pz1 = NDIM == 3 ? z1 : 1;
        if (NDIM == 3) {                             // the item's run of slices
            const int ntile = tiles_x * ((y1 - y0 + tile_y - 1) / tile_y);
            int zl = BAND_ZCHUNK;                    // banded: runs of BAND_ZCHUNK
            if (!BAND) {                             // plain: ceil(bz / PLAIN_ZCHUNK) equal runs
                const int nzc = (z1 - z0 + PLAIN_ZCHUNK - 1) / PLAIN_ZCHUNK;
                zl = (z1 - z0 + nzc - 1) / nzc;
            }
            pz0 = z0 + (tt / ntile) * zl;
            pz1 = min(z1, pz0 + zl);
            tt %= ntile;
        }
        TileCtx t;
        t.M = M;
        t.disc = (int*)(M + TILE_LEVELS * (tile_y * TILE_STRIDE + 1)) + wid * (4 * DL_CAP + 64);
        t.reach = s_reach;
        t.ty0 = y0 + (tt / tiles_x) * tile_y;
        t.tx0 = x0 + (tt % tiles_x) * TILE_X;
        t.H = min(tile_y, y1 - t.ty0);
        t.W = min(TILE_X, x1 - t.tx0);
        t.lstride = t.H * TILE_STRIDE + 1;
        t.wy = spc.wy;
        t.wx = spc.wx;
        const int sy0 = max(y0, t.ty0 - Ry), sy1 = min(y1, t.ty0 + t.H + Ry);
        const int sx0 = max(x0, t.tx0 - Rx), sx1 = min(x1, t.tx0 + t.W + Rx);
        // Floor of the tile in slice pz after a band: the table is pushed down to level
        // 0 (the cells keep their values, the upper levels are cleared, so later bands
        // paint on), and the smallest value over the object's cells is taken (0 while
        // one is unpainted; INT_MAX when the slice holds none).
        auto tile_floor = [&](int slot, int pz) -> int {
            __syncthreads();                            // every wave's discs are in the table
            // the other slot is next band's: every thread has read its last floor
            if (tid == 0) s_floor[slot ^ 1] = INT_MAX;
            for (int row = wid; row < t.H; row += nwaves) {
                uint32_t val[TILE_LEVELS];
#pragma unroll
                for (int k = 0; k < TILE_LEVELS; ++k)
                    val[k] = lane < t.W ? t.M[k * t.lstride + row * TILE_STRIDE + lane] : 0u;
#pragma unroll
                for (int k = TILE_LEVELS - 1; k >= 1; --k) {
                    const uint32_t up = (uint32_t)__builtin_amdgcn_ds_bpermute((int)pd_idx[k], (int)val[k]);
                    val[k - 1] = max(val[k - 1], max(val[k], up));
                }
                int mn = INT_MAX;
                if (lane < t.W) {
                    t.M[row * TILE_STRIDE + lane] = val[0];
#pragma unroll
                    for (int k = 1; k < TILE_LEVELS; ++k) t.M[k * t.lstride + row * TILE_STRIDE + lane] = 0u;
                    const L lv = lab[((size_t)pz * ny + t.ty0 + row) * nx + t.tx0 + lane];
                    if ((uint64_t)lv == (uint64_t)l) mn = (int)val[0];
                }
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) mn = min(mn, __shfl_xor(mn, off, 64));
                if (lane == 0 && mn != INT_MAX) atomicMin(&s_floor[slot], mn);
            }
            __syncthreads();
            return s_floor[slot];
        };
        // fused measures: this thread's share of the item's volume, radius sums,
        // largest LT and shell terms (every painted cell is a voxel of label l)
        uint32_t a_n = 0, a_sn = 0;
        uint64_t a_q = 0, a_sq = 0;
        int a_mx = 0;
        for (int pz = pz0; pz < pz1; ++pz) {
            t.dirty = &s_dirty[pz & 1];
            int nlist = 0;                                // listed discs (wave-uniform)
            int sylast = sy0;
            // Discs of one source column (lane) in this slice: the stored front, the
            // spilled front or a rescan of the column.  Only discs that reach the
            // tile (b > need) with a value above the floor fl are listed.
            auto column = [&](L lc, uint32_t ec, int sx, int sy, size_t rowi, int need, int fl)
                              __attribute__((always_inline)) {
                const bool own = sx < sx1 && (uint64_t)lc == (uint64_t)l;
                const uint32_t e0 = own ? ec : 0u;
                uint32_t e[ZF_PLANES];
                e[0] = e0;
#pragma unroll
                for (int q = 1; q < ZF_PLANES; ++q) e[q] = 0u;
                int nent = 0;
                bool rescan = false, spilled = false;
                if (NDIM == 2) {
                    nent = e0 ? 1 : 0;
                } else if (e0) {
                    const int cc = (int)(e0 >> ZF_N_SHIFT);
                    spilled = cc == 7 && (e0 & ZF_SPILL);
                    rescan = cc == 7 && !spilled;
                    nent = cc == 7 ? 0 : cc;
#pragma unroll
                    for (int q = 1; q < ZF_PLANES; ++q)
                        if (nent > q) e[q] = zf[q * n + rowi + sx];
                }
                // stored front entries
#pragma unroll
                for (int p = 0; p < ZF_PLANES; ++p) {
                    const bool has = p < nent;
                    if (!__ballot(has)) break;
                    int v = 0, b = 0;
                    if (has) {
                        if (NDIM == 2) {
                            v = b = (int)(e[p] & 0x7fffffffu);
                        } else {
                            v = (int)(e[p] & ZF_D_MASK);
                            const int dz = (int)((e[p] >> ZF_DZ_SHIFT) & ZF_DZ_MASK) - 512;
                            b = v - (W ? spc.wz : 1) * dz * dz;
                        }
                    }
                    disc_push<NDIM, W>(t, nlist, has && b > need && v > fl, v, b, sx, sy, lane);
                }
                // long fronts kept in the front pass's spill region or the pool
                if (NDIM == 3 && __ballot(spilled)) {
                    int m = 0;
                    const uint32_t* sp = spill;
                    if (spilled) {
                        m = (int)((e0 >> 16) & 0xffu);
                        if (e0 & ZF_POOL) {
                            sp = pool + zf[n + rowi + sx];
                        } else {
                            const size_t blk = ((size_t)(pz / chunk) * ny + sy) * ((nx + 63) / 64) + sx / 64;
                            sp = spill + blk * (size_t)(SPILL_ROW_SLICE * chunk) + (e0 & 0xffffu);
                        }
                    }
                    for (int q = 0; __ballot(q < m); ++q) {
                        const bool has = q < m;
                        int v = 0, b = 0;
                        if (has) {
                            const uint32_t w = sp[q];
                            v = (int)(w & ZF_D_MASK);
                            const int dz = (int)((w >> ZF_DZ_SHIFT) & ZF_DZ_MASK) - 512;
                            b = v - (W ? spc.wz : 1) * dz * dz;
                        }
                        disc_push<NDIM, W>(t, nlist, has && b > need && v > fl, v, b, sx, sy, lane);
                    }
                }
                // fronts that did not fit the spill region: every kept centre of the
                // column (within the object's z range) that reaches this slice -- a
                // superset of the front.  The wave walks the offsets dz = -R..R
                // together, four independent loads at a time.
                if (NDIM == 3 && __ballot(rescan)) {
                    const size_t col = (size_t)sy * nx + sx;
                    for (int d0 = -Rz; d0 <= Rz; d0 += 4) {
                        int kv[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int zc = pz + d0 + u;
                            kv[u] = (rescan && d0 + u <= Rz && zc >= z0 && zc < z1) ? kd[col * (size_t)nz + zc] : 0;
                        }
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int dz = d0 + u;
                            const int b = kv[u] - (W ? spc.wz : 1) * dz * dz;
                            disc_push<NDIM, W>(t, nlist, kv[u] > fl && b > 0 && b > need, kv[u], b, sx, sy,
                                               lane);
                        }
                    }
                }
            };
            // labels and plane-0 fronts of a whole source row, loaded together; the
            // next row of the wave is fetched while the current one is processed
            constexpr int MAXC = 3;                       // source rows span <= 64 + 2 * 64 columns
            // Source rows of at most 32 columns (3D, small objects): two rows per wave
            // iteration, 32 lanes each (3D disc entries carry their own source row).  Four
            // rows of 16 lanes for rows of at most 16 columns measured slower.
            const int rs = NDIM == 3 && sx1 - sx0 <= 32 ? 1 : 0;
            const int lx = lane & ((64 >> rs) - 1);       // the lane's column in its row chunk
            const int lrow = lane >> (6 - rs);            // the lane's row within the iteration
            const int rfirst = sy0 + (wid << rs), rstep = nwaves << rs;
            L nlv[MAXC];
            uint32_t nev[MAXC];
            auto fetch_row = [&](int sbn) {
                const int syn = sbn + lrow;
                const size_t ri = ((size_t)pz * ny + syn) * nx;
#pragma unroll
                for (int c = 0; c < MAXC; ++c) {
                    const int sx = sx0 + c * 64 + lx;
                    const bool in = syn < sy1 && sx < sx1;
                    nlv[c] = in ? lab[ri + sx] : L(0);
                    nev[c] = in ? zf[ri + sx] : 0u;
                }
            };
            if constexpr (BAND) {
                // Objects of large reach: the source groups (one source row x 64 columns)
                // in NBANDS bands of value, from the object's largest D down, with the
                // tile's floor (smallest value painted so far over the object's cells in
                // this slice) taken after every band but the last.  A group whose bound
                // does not exceed the floor, and any disc whose value does not, cannot
                // raise a cell and is skipped.
                const uint32_t* bms = bmap + (size_t)pz * ny * ngroups;
                int fl = 0;
                // group bounds of a source row, loaded together BM_CH chunks of 64
                // columns at a time (one round trip for rows up to 384 columns)
                constexpr int BM_CH = 6;
                const int nch = (sx1 - sx0 + 63) >> 6;
                for (int band = 0; band < NBANDS; ++band) {
                    // bands from the object's largest D down: [mdl, inf), then equal steps
                    // of mdl (with three bands [mdl / 2, mdl) and the rest)
                    const int lo_b = band == 0 ? mdl : band == NBANDS - 1 ? INT_MIN
                                                                          : (int)(((long long)mdl * (NBANDS - 1 - band)) / (NBANDS - 1));
                    const int hi_b = band == 0 ? INT_MAX
                                               : (int)(((long long)mdl * (NBANDS - band)) / (NBANDS - 1));
                    // no value of this band, or a later one, exceeds the floor: done
                    if (band > 0 && fl >= hi_b) break;
                    for (int sy = sy0 + wid; sy < sy1; sy += nwaves) {
                        const size_t rowi = ((size_t)pz * ny + sy) * nx;
                        const int ddy = max(max(t.ty0 - sy, sy - (t.ty0 + t.H - 1)), 0);
                        const int rowd = W ? spc.wy * ddy * ddy : ddy * ddy;
                        for (int cb = 0; cb < nch; cb += BM_CH) {
                            int bmr[BM_CH];
#pragma unroll
                            for (int u = 0; u < BM_CH; ++u) {
                                const int sx = sx0 + (cb + u) * 64 + lane;
                                bmr[u] = sx < sx1 ? (int)bms[(size_t)sy * ngroups + (sx >> 6)] : 0;
                            }
                        for (int u = 0; u < BM_CH && cb + u < nch; ++u) {
                            const int c = cb + u;
                            const int sx = sx0 + c * 64 + lane;
                            const bool in = sx < sx1;
                            int bmv = bmr[0];
#pragma unroll
                            for (int q = 1; q < BM_CH; ++q) bmv = u == q ? bmr[q] : bmv;
                            // a group is visited in every band its bound reaches; in 3D each
                            // lane then takes its column in the band of the column's largest
                            // kept D (no smaller than any value its discs carry, no larger than
                            // the group bound of a slice where it has discs), so every column
                            // is painted in one band and only columns reaching it in the first
                            bool go = in && bmv >= lo_b && bmv > fl;
                            if (!__ballot(go)) continue;
                            if (NDIM == 3) {
                                const int cml = go ? colmax[(size_t)sy * nx + sx] : 0;
                                go = go && cml >= lo_b && cml < hi_b && cml > fl;
                                if (!__ballot(go)) continue;
                            } else {
                                go = go && bmv < hi_b;
                                if (!__ballot(go)) continue;
                            }
                            const int ddx = max(max(t.tx0 - sx, sx - (t.tx0 + t.W - 1)), 0);
                            const int need = rowd + (W ? spc.wx * ddx * ddx : ddx * ddx);
                            const L lc = go ? lab[rowi + sx] : L(0);
                            const uint32_t ec = go ? zf[rowi + sx] : 0u;
                            column(lc, ec, sx, sy, rowi, need, fl);
                        }
                        }
                        if (NDIM == 2 && nlist) {             // 2D lists hold one source row
                            disc_flush<NDIM, W>(t, nlist, sy, lane);
                            nlist = 0;
                        }
                    }
                    if (nlist) disc_flush<NDIM, W>(t, nlist, sy0, lane);
                    nlist = 0;
                    if (band < NBANDS - 1) fl = tile_floor(band & 1, pz);
                }
            } else {
                fetch_row(rfirst);
                for (int sb = rfirst; sb < sy1; sb += rstep) {
                    const int sy = sb + lrow;                 // this lane's source row (past sy1: no column)
                    sylast = sb;
                    L lv[MAXC];
                    uint32_t ev[MAXC];
#pragma unroll
                    for (int c = 0; c < MAXC; ++c) {
                        lv[c] = nlv[c];
                        ev[c] = nev[c];
                    }
                    fetch_row(sb + rstep);
                    const size_t rowi = ((size_t)pz * ny + sy) * nx;
                    // a disc of residual b reaches a tile cell only if b exceeds the squared
                    // distance from its centre to the tile: discs below it are not listed
                    const int ddy = max(max(t.ty0 - sy, sy - (t.ty0 + t.H - 1)), 0);
                    const int rowd = W ? spc.wy * ddy * ddy : ddy * ddy;
                    for (int c = 0; c * 64 < sx1 - sx0; ++c) {
                        const int sx = sx0 + c * 64 + lx;
                        const int ddx = max(max(t.tx0 - sx, sx - (t.tx0 + t.W - 1)), 0);
                        const int need = rowd + (W ? spc.wx * ddx * ddx : ddx * ddx);
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
                        column(lc, ec, sx, sy, rowi, need, 0);
                    }
                    if (NDIM == 2 && nlist) {                 // 2D lists hold one source row
                        disc_flush<NDIM, W>(t, nlist, sy, lane);
                        nlist = 0;
                    }
                }
                if (nlist) disc_flush<NDIM, W>(t, nlist, sylast, lane);
            }
            __syncthreads();
            // push-down of the sparse table, one wave per painted row: level k-1 at
            // column c takes the blocks of level k starting at c and c - 2^(k-1); then
            // write the painted cells and clear every level of the row.  Rows no disc
            // reached are still clear and hold no voxel of the object.
            const unsigned long long painted = *t.dirty;
            if (tid == 0) {
                s_dirty[(pz + 1) & 1] = 0ull;             // the next slice's mask
                s_floor[0] = s_floor[1] = INT_MAX;        // read before the last band
            }
            for (int row = wid; row < t.H; row += nwaves) {
                if (!((painted >> row) & 1ull)) continue;
                // levels above floor(log2(min(W, 2R + 1))) are never painted and hold
                // zeros: every level is read and cleared, so the lane mask is the only
                // condition
                uint32_t val[TILE_LEVELS];
#pragma unroll
                for (int k = 0; k < TILE_LEVELS; ++k)
                    val[k] = lane < t.W ? t.M[k * t.lstride + row * TILE_STRIDE + lane] : 0u;
#pragma unroll
                for (int k = TILE_LEVELS - 1; k >= 1; --k) {
                    const uint32_t up = (uint32_t)__builtin_amdgcn_ds_bpermute((int)pd_idx[k], (int)val[k]);
                    val[k - 1] = max(val[k - 1], max(val[k], up));
                }
                if (lane < t.W) {
                    if (val[0]) {
                        const int gy = t.ty0 + row, gx = t.tx0 + lane;
                        const size_t gi = ((size_t)pz * ny + gy) * nx + gx;
                        lt[gi] = (int32_t)val[0];
                        if (ms.vol) {
                            const int v = (int)val[0];
                            const uint64_t q = radius_q23(v);
                            // on the shell exactly when a face neighbour (or the image
                            // border) is not of the object: D = 1 at unit spacing
                            bool shell;
                            if (!W) {
                                shell = Dmap[gi] == 1;
                            } else {
                                const L lo = (L)l;
                                shell = gx == 0 || gx == nx - 1 || gy == 0 || gy == ny - 1 || lab[gi - 1] != lo ||
                                        lab[gi + 1] != lo || lab[gi - nx] != lo || lab[gi + nx] != lo;
                                if (NDIM == 3 && !shell) {
                                    const size_t pl = (size_t)nx * ny;
                                    shell = pz == 0 || pz == nz - 1 || lab[gi - pl] != lo || lab[gi + pl] != lo;
                                }
                            }
                            ++a_n;
                            a_q += q;
                            a_mx = max(a_mx, v);
                            if (shell) {
                                ++a_sn;
                                a_sq += q;
                            }
                        }
                    }
#pragma unroll
                    for (int k = 0; k < TILE_LEVELS; ++k) t.M[k * t.lstride + row * TILE_STRIDE + lane] = 0u;
                }
            }
            __syncthreads();
        }
        if (ms.vol) {                                    // one set of atomics per wave and item
            uint64_t n1 = a_n, n2 = a_sn, q1 = a_q, q2 = a_sq;
            int m1 = a_mx;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                n1 += __shfl_xor((unsigned long long)n1, off, 64);
                n2 += __shfl_xor((unsigned long long)n2, off, 64);
                q1 += __shfl_xor((unsigned long long)q1, off, 64);
                q2 += __shfl_xor((unsigned long long)q2, off, 64);
                m1 = max(m1, __shfl_xor(m1, off, 64));
            }
            if (lane == 0 && n1) {
                atomicAdd((unsigned long long*)&ms.vol[l], (unsigned long long)n1);
                atomicAdd((unsigned long long*)&ms.sq[l], (unsigned long long)q1);
                atomicMax(&ms.mx[l], m1);
                if (n2) {
                    atomicAdd((unsigned long long*)&ms.shc[l], (unsigned long long)n2);
                    atomicAdd((unsigned long long*)&ms.ssq[l], (unsigned long long)q2);
                }
            }
        }
    }
}

// ------------------------------------------------------------------ host side

static inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct ThickLayout {
    size_t bb, maxd, toff, toff_big, ord, counter, zf, kd, spill, colmax, work, pool, bmap, total;
    uint32_t wcap;          // long-list work items: one per (column, chunk) at the smallest chunk
    size_t pool_words;
};

static ThickLayout thick_layout(const Geom& g, uint32_t max_label) {
    const size_t nlab = (size_t)max_label + 1;
    ThickLayout o;
    size_t at = 0;
    o.bb = at;      at += align256(6 * nlab * sizeof(int32_t));
    o.maxd = at;    at += align256(nlab * sizeof(int32_t));
    o.toff = at;    at += align256((nlab + 1) * sizeof(uint32_t));
    o.toff_big = at; at += align256((nlab + 1) * sizeof(uint32_t));
    o.ord = at;     at += align256(nlab * sizeof(uint32_t));
    o.counter = at; at += 256;
    o.zf = at;      at += align256((g.ndim == 3 ? ZF_PLANES : 1) * g.n * sizeof(uint32_t));
    o.kd = at;      at += g.ndim == 3 ? align256(g.n * sizeof(int32_t)) : 0;
    // spill regions of the front pass: one per (row of 64 columns, z chunk); the chunks
    // (32, 64 or 128 slices) all divide 128, so the z extent rounded up to 128 holds them
    o.spill = at;
    at += g.ndim == 3 ? align256((size_t)((g.nx + 63) / 64) * g.ny * ((g.nz + 127) & ~127) * SPILL_ROW_SLICE *
                                 sizeof(uint32_t))
                      : 0;
    o.colmax = at;  at += g.ndim == 3 ? align256((size_t)g.ny * g.nx * sizeof(int32_t)) : 0;
    o.wcap = g.ndim == 3 ? (uint32_t)((size_t)g.ny * g.nx * ((g.nz + 31) / 32)) : 0u;
    o.work = at;    at += align256((size_t)o.wcap * sizeof(uint32_t));
    o.pool_words = g.ndim == 3 ? g.n : 0;
    o.pool = at;    at += align256(o.pool_words * sizeof(uint32_t));
    // bound on the front values per (slice, row, 64-column group): the largest kept D
    // of the group's columns that have a front in the slice
    o.bmap = at;    at += align256((size_t)g.nz * g.ny * ((g.nx + 63) / 64) * sizeof(uint32_t));
    o.total = at;
    return o;
}

size_t thickness_scratch_bytes(const Geom& g, uint32_t max_label) {
    return thick_layout(g, max_label).total;
}

// Dynamic LDS of a paint block: the sparse table for `rows` tile rows plus one disc
// list per wave.
static size_t paint_lds(int rows, int threads) {
    return (size_t)TILE_LEVELS * (rows * TILE_STRIDE + 1) * sizeof(uint32_t) +
           (size_t)(threads / 64) * (4 * DL_CAP + 64) * sizeof(int);
}

// Tile rows of the paint pass: 64 when the device lets one 1024-thread block hold
// the 64-row table (7 levels x 64 x 65 words = 116,480 B) and its wave lists, else 32.
constexpr size_t PAINT_DYN64 = (size_t)TILE_LEVELS * (64 * TILE_STRIDE + 1) * sizeof(uint32_t) +
                               (size_t)(PAINT_THREADS / 64) * (4 * DL_CAP + 64) * sizeof(int);

int paint_tile_rows(lt_ctx* ctx) {
    const size_t dyn64 = PAINT_DYN64;
    static std::once_flag once;
    std::call_once(once, [] {
        const void* fns[] = {(const void*)paint_tiles<3, uint16_t>, (const void*)paint_tiles<3, int32_t>,
                             (const void*)paint_tiles<3, uint32_t>, (const void*)paint_tiles<2, uint16_t>,
                             (const void*)paint_tiles<2, int32_t>, (const void*)paint_tiles<2, uint32_t>,
                             (const void*)paint_tiles<3, uint16_t, true>, (const void*)paint_tiles<3, int32_t, true>,
                             (const void*)paint_tiles<3, uint32_t, true>, (const void*)paint_tiles<2, uint16_t, true>,
                             (const void*)paint_tiles<2, int32_t, true>, (const void*)paint_tiles<2, uint32_t, true>,
                             (const void*)paint_tiles<3, uint16_t, false, true>,
                             (const void*)paint_tiles<3, int32_t, false, true>,
                             (const void*)paint_tiles<3, uint32_t, false, true>,
                             (const void*)paint_tiles<3, uint16_t, true, true>,
                             (const void*)paint_tiles<3, int32_t, true, true>,
                             (const void*)paint_tiles<3, uint32_t, true, true>,
                             (const void*)paint_tiles<2, uint16_t, false, true>,
                             (const void*)paint_tiles<2, int32_t, false, true>,
                             (const void*)paint_tiles<2, uint32_t, false, true>,
                             (const void*)paint_tiles<2, uint16_t, true, true>,
                             (const void*)paint_tiles<2, int32_t, true, true>,
                             (const void*)paint_tiles<2, uint32_t, true, true>};
        for (const void* f : fns)
            (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)PAINT_DYN64);
    });
    // dynamic table and wave lists + static reach table and work-item word
    const bool fits64 = ctx->lds_per_block >= dyn64 + REACH_TAB + 64;
    if (ctx->tune.paint_tile_rows == 32) return 32;
    return fits64 ? 64 : 32;
}

template <typename L>
static lt_status thickness_typed(lt_ctx* ctx, const L* lab, const Geom& g, const int32_t* D,
                                 uint32_t max_label, int32_t* lt, void* scratch, hipStream_t s,
                                 const MeasureSums* sums, int32_t* boxes, const Spacing& sp) {
    const bool w = !sp.unit();
    const int32_t* tabw = nullptr;                    // weighted containment tables
    if (w) {
        lt_status st = prune_tables_weighted(ctx, g.ndim, sp, &tabw);
        if (st) return st;
    }
    const MeasureSums none{nullptr, nullptr, nullptr, nullptr, nullptr};
    const MeasureSums ms = sums ? *sums : none;
    const ThickLayout lay = thick_layout(g, max_label);
    char* base = (char*)scratch;
    int32_t* bb = boxes ? boxes : (int32_t*)(base + lay.bb);
    int32_t* maxd = (int32_t*)(base + lay.maxd);
    uint32_t* toff = (uint32_t*)(base + lay.toff);
    uint32_t* toff_big = (uint32_t*)(base + lay.toff_big);
    uint32_t* ord = (uint32_t*)(base + lay.ord);
    uint32_t* counter = (uint32_t*)(base + lay.counter);
    uint32_t* zf = (uint32_t*)(base + lay.zf);
    int32_t* kd = (int32_t*)(base + lay.kd);
    uint32_t* spill = (uint32_t*)(base + lay.spill);
    int32_t* colmax = (int32_t*)(base + lay.colmax);
    uint32_t* work = (uint32_t*)(base + lay.work);
    uint32_t* bmap = (uint32_t*)(base + lay.bmap);
    // LT_SPILL_CAP (environment, read at every call) caps each block's spill region and
    // the pool at that many words: with 0 every front longer than ZF_PLANES is rescanned
    // by the paint pass (the fallback kept for full spill space), which tests of that
    // path use.  Same results.
    size_t pool_words = lay.pool_words;
    uint32_t region_cap = 0xffffffffu;
    if (const char* e = getenv("LT_SPILL_CAP")) {
        const unsigned long long c = strtoull(e, nullptr, 10);
        pool_words = std::min(pool_words, (size_t)c);
        region_cap = (uint32_t)std::min(c, 0xffffffffull);
    }
    const SpillPool pool{(uint32_t*)(base + lay.pool), (unsigned long long*)(counter + 4), pool_words};
    const size_t ncol = g.ndim == 3 ? (size_t)g.ny * g.nx : 0;
    const int chunk = ctx->tune.front_chunk > 0 ? ctx->tune.front_chunk : 64;
    const uint32_t nlab = max_label + 1;

    {
        ProfScope _p(ctx, s, "init_label_arrays");
        const size_t items = std::max((size_t)nlab, std::min(ncol, (size_t)1 << 20));
        init_label_arrays<<<(unsigned)((items + 255) / 256), 256, 0, s>>>(boxes ? nullptr : bb, maxd, nlab, counter,
                                                                          colmax, ncol);
    }
    if (!boxes) {
        ProfScope _p(ctx, s, "bbox_runs");
        bbox_runs<L><<<dim3(1, (g.ny + BB_ROWS_Y - 1) / BB_ROWS_Y, (g.nz + BB_ROWS_Z - 1) / BB_ROWS_Z), 1024, 0,
                       s>>>(lab, g.nx, g.ny, g.nz, max_label, bb, nlab, ctx->d_err);
    }
    if (g.ndim == 3) {
        {
            ProfScope _p(ctx, s, "prune3d");
            const dim3 grid((g.nx + 63) / 64, (g.ny + PR_TY - 1) / PR_TY, (g.nz + PR_ZB - 1) / PR_ZB);
            if (w)
                prune3d<L, true><<<grid, dim3(64, PR_TY), 0, s>>>(lab, D, g.nx, g.ny, g.nz, max_label, tabw, kd, lt,
                                                                   maxd, colmax, ctx->d_err, sp.wz, sp.wy, sp.wx);
            else
                prune3d<L><<<grid, dim3(64, PR_TY), 0, s>>>(lab, D, g.nx, g.ny, g.nz, max_label, ctx->d_prune3, kd,
                                                             lt, maxd, colmax, ctx->d_err);
        }
        {
            ProfScope _p(ctx, s, "fronts3d");
            const dim3 grid((g.nx + 63) / 64, g.ny, (g.nz + chunk - 1) / chunk);
            if (w)
                fronts3d<true><<<grid, 256, fronts3d_lds(chunk), s>>>(kd, g.nx, g.ny, g.nz, chunk, colmax, zf, spill,
                                                                      work, counter + 2, lay.wcap, pool, bmap, region_cap, sp.wz);
            else
                fronts3d<<<grid, 256, fronts3d_lds(chunk), s>>>(kd, g.nx, g.ny, g.nz, chunk, colmax, zf, spill,
                                                                work, counter + 2, lay.wcap, pool, bmap, region_cap);
        }
        {
            // columns with more listed centres than the front pass holds (objects of
            // large radius); returns at once when there are none
            ProfScope _p(ctx, s, "fronts3d_long");
            const int blocks = ctx->n_cu * 2;
            if (w)
                fronts3d_long<true><<<blocks, 256, fronts3d_long_lds(), s>>>(kd, g.nx, g.ny, g.nz, chunk, colmax, zf,
                                                                            work, counter + 2, lay.wcap, counter + 3,
                                                                            pool, sp.wz);
            else
                fronts3d_long<<<blocks, 256, fronts3d_long_lds(), s>>>(kd, g.nx, g.ny, g.nz, chunk, colmax, zf, work,
                                                                      counter + 2, lay.wcap, counter + 3, pool);
        }
    } else {
        ProfScope _p(ctx, s, "pixels2d");
        if (w)
            pixels2d<L, true><<<dim3((g.nx + 255) / 256, g.ny), dim3(256), 0, s>>>(lab, D, g.nx, g.ny, max_label,
                                                                                  tabw, zf, lt, maxd, bmap, sp.wy, sp.wx);
        else
            pixels2d<L><<<dim3((g.nx + 255) / 256, g.ny), dim3(256), 0, s>>>(lab, D, g.nx, g.ny, max_label,
                                                                            ctx->d_prune2, zf, lt, maxd, bmap);
    }
    const int tile_y = paint_tile_rows(ctx);
    // objects with balls reaching BAND_REACH or more along y or x take the banded launch:
    // largest D above BAND_REACH^2 times the smaller in-plane squared spacing
    const int band_d = BAND_REACH * BAND_REACH * std::min(sp.wy, sp.wx);
    {
        ProfScope _p(ctx, s, "plan_tiles");
        plan_tiles<<<1, 1024, 0, s>>>(bb, maxd, nlab, tile_y, band_d, toff, toff_big, ord, counter);
    }
    // two blocks of 512 threads per CU (32-row tiles) when both fit in the LDS, else one
    // block of 1024 threads: two blocks overlap each other's slice barriers
    const bool two = ctx->tune.paint_blocks_per_cu >= 2 &&
                     2 * (paint_lds(tile_y, PAINT_THREADS / 2) + REACH_TAB + 64) <= ctx->lds_per_block;
    const int threads = two ? PAINT_THREADS / 2 : PAINT_THREADS;
    const size_t lds = paint_lds(tile_y, threads);
    const int blocks = ctx->n_cu * (two ? 2 : 1);
    if (g.ndim == 3) {
        {
            // objects of large reach (returns at once when there are none)
            ProfScope _p(ctx, s, "paint_tiles_banded");
            if (w)
                paint_tiles<3, L, true, true><<<blocks, threads, lds, s>>>(
                    lab, zf, kd, bb, maxd, toff_big, ord, nlab, g.nx, g.ny, g.nz, tile_y, counter + 6, lt, spill,
                    pool.base, bmap, colmax, chunk, ms, D, sp);
            else
                paint_tiles<3, L, false, true><<<blocks, threads, lds, s>>>(
                    lab, zf, kd, bb, maxd, toff_big, ord, nlab, g.nx, g.ny, g.nz, tile_y, counter + 6, lt, spill,
                    pool.base, bmap, colmax, chunk, ms, D);
        }
        ProfScope _p(ctx, s, "paint_tiles");
        if (w)
            paint_tiles<3, L, true><<<blocks, threads, lds, s>>>(lab, zf, kd, bb, maxd, toff, ord, nlab, g.nx, g.ny, g.nz,
                                                                 tile_y, counter, lt, spill, pool.base, bmap, colmax,
                                                                 chunk, ms, D, sp);
        else
            paint_tiles<3, L><<<blocks, threads, lds, s>>>(lab, zf, kd, bb, maxd, toff, ord, nlab, g.nx, g.ny, g.nz,
                                                           tile_y, counter, lt, spill, pool.base, bmap, colmax, chunk,
                                                           ms, D);
    } else {
        {
            ProfScope _p(ctx, s, "paint_tiles_banded");
            if (w)
                paint_tiles<2, L, true, true><<<blocks, threads, lds, s>>>(
                    lab, zf, kd, bb, maxd, toff_big, ord, nlab, g.nx, g.ny, 1, tile_y, counter + 6, lt, spill, pool.base,
                    bmap, nullptr, chunk, ms, D, sp);
            else
                paint_tiles<2, L, false, true><<<blocks, threads, lds, s>>>(
                    lab, zf, kd, bb, maxd, toff_big, ord, nlab, g.nx, g.ny, 1, tile_y, counter + 6, lt, spill, pool.base,
                    bmap, nullptr, chunk, ms, D);
        }
        ProfScope _p(ctx, s, "paint_tiles");
        if (w)
            paint_tiles<2, L, true><<<blocks, threads, lds, s>>>(lab, zf, kd, bb, maxd, toff, ord, nlab, g.nx, g.ny, 1,
                                                                 tile_y, counter, lt, spill, pool.base, bmap, nullptr,
                                                                 chunk, ms, D, sp);
        else
            paint_tiles<2, L><<<blocks, threads, lds, s>>>(lab, zf, kd, bb, maxd, toff, ord, nlab, g.nx, g.ny, 1, tile_y,
                                                           counter, lt, spill, pool.base, bmap, nullptr, chunk, ms,
                                                           D);
    }
    return hip_check(hipGetLastError(), "thickness launch");
}

lt_status launch_thickness(lt_ctx* ctx, const void* labels, lt_dtype dt, const Geom& g,
                           const int32_t* dist_sq, uint32_t max_label, int32_t* lt_sq,
                           void* scratch, hipStream_t s, const MeasureSums* sums, int32_t* boxes,
                           const Spacing* sp) {
    const Spacing unit;
    const Spacing& spc = sp ? *sp : unit;
    switch (dt) {
        case LT_U16:
            return thickness_typed(ctx, (const uint16_t*)labels, g, dist_sq, max_label, lt_sq, scratch, s, sums,
                                   boxes, spc);
        case LT_I32:
            return thickness_typed(ctx, (const int32_t*)labels, g, dist_sq, max_label, lt_sq, scratch, s, sums,
                                   boxes, spc);
        case LT_U32:
            return thickness_typed(ctx, (const uint32_t*)labels, g, dist_sq, max_label, lt_sq, scratch, s, sums,
                                   boxes, spc);
    }
    return set_error(LT_E_DTYPE, "unknown dtype");
}

}  // namespace lt
