// Per-label squared Euclidean distance transform, three separable passes.
//
// For an object voxel p of label l the nearest non-l lattice point (another label,
// background, or any position outside the image) is sought.  Along each line the
// voxels of l form runs; the run's end points act as zero-cost sites and a voxel of
// the same label in another run is never nearer than the non-l voxel between the
// runs, so every run is an independent 1D problem:
//   pass x:  g(p)  = distance along x to the first non-l position (1D transform);
//   pass y:  d2(p) = min over j in the y-run of p of (y_p - y_j)^2 + g(j)^2, and the
//            squared distance to the run's end sites;
//   pass z:  d(p)  = the same along z over d2 (3D only).
// Each pass searches outward from p and stops as soon as k^2 reaches the best value
// found, so the search is exact and costs O(sqrt(D)) loads per voxel.  Lanes of a
// wave hold consecutive x, so every load of a pass is a coalesced row access.
#include <type_traits>

#include "lt_internal.h"

namespace lt {

// Pass x: each wave takes whole rows, one at a time, with no block barrier.  All
// MAXC 64-voxel chunks of a row are loaded at once (their loads in flight
// together); a voxel's left and right neighbours come from the adjacent lanes by
// DPP lane shifts (across a chunk edge by readlane of the neighbouring chunk).
// Ballots give, per chunk, the positions where a run starts (label differs from
// the left neighbour, or x = 0) and ends; these masks are wave-uniform, so the
// nearest start before a chunk and the nearest end after it are scalars carried
// along the row.  A voxel's run [s, e] comes from its own chunk's masks by bit
// scans, else from those scalars, and g = min(x - s + 1, e - x + 1).
// With BOX, the object runs of a row are compacted into the wave's list in LDS
// (label, start, end) and merged with the row's z into the block's label table,
// 64 runs per pass (bounding boxes of the fused pipeline); all waves of a block walk
// slices of one row index y, so the table holds z and x extents only (y is the
// block's), an object's runs meet in few blocks, and the table is flushed to the
// global boxes once per block.  The next row's labels are loaded while a row is
// processed.
constexpr int XBOX_TAB = 128;
constexpr int XW = 4;                                // waves per block of the x pass
constexpr int XRUNS = 64;                            // run list entries per wave

template <typename L, bool BOX, int MAXC>
__global__ void __launch_bounds__(64 * XW)
edt_pass_x(const L* __restrict__ lab, uint16_t* __restrict__ g, int nx, int ny, int nz, uint32_t* err,
           BoxTarget box, int zper) {
    __shared__ uint32_t s_key[BOX ? XBOX_TAB : 1];
    __shared__ int s_bb[4][BOX ? XBOX_TAB : 1];          // zmin, zmax, xmin, xmax
    __shared__ uint32_t s_run[BOX ? XW : 1][BOX ? 3 * XRUNS : 1];
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int chunks = (nx + 63) >> 6;                 // <= MAXC
    const int y = blockIdx.y;
    if (BOX) {
        for (int t = threadIdx.x; t < XBOX_TAB; t += blockDim.x) {
            s_key[t] = 0u;
            s_bb[0][t] = s_bb[2][t] = 0x7fffffff;
            s_bb[1][t] = s_bb[3][t] = -1;
        }
        __syncthreads();
    }
    const int zb = blockIdx.z * zper, ze = min(nz, zb + zper);
    bool bad = false;
    uint32_t* runs = s_run[BOX ? wid : 0];
    // merge the wave's listed runs (n of them, row z) into the block table
    auto merge_runs = [&](int n, int z) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < n) {
            const uint32_t l = runs[3 * lane];
            const int s0 = (int)runs[3 * lane + 1], e0 = (int)runs[3 * lane + 2];
            const int slot = lds_slot<XBOX_TAB>(s_key, l);
            if (slot >= 0) {
                atomicMin(&s_bb[0][slot], z);
                atomicMax(&s_bb[1][slot], z);
                atomicMin(&s_bb[2][slot], s0);
                atomicMax(&s_bb[3][slot], e0);
            } else {
                atomicMin(&box.bb[0 * box.nlab + l], z);
                atomicMax(&box.bb[1 * box.nlab + l], z);
                atomicMin(&box.bb[2 * box.nlab + l], y);
                atomicMax(&box.bb[3 * box.nlab + l], y);
                atomicMin(&box.bb[4 * box.nlab + l], s0);
                atomicMax(&box.bb[5 * box.nlab + l], e0);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    auto load_row = [&](int z, uint32_t (&v)[MAXC]) {
        const L* r = lab + ((size_t)z * ny + y) * nx;
#pragma unroll
        for (int c = 0; c < MAXC; ++c) {
            const int x = c * 64 + lane;
            v[c] = (z < ze && c < chunks && x < nx) ? (uint32_t)r[x] : 0u;
        }
    };
    uint32_t nv[MAXC];
    load_row(zb + wid, nv);
    for (int z = zb + wid; z < ze; z += XW) {
        const size_t row = (size_t)z * ny + y;
        uint32_t v[MAXC];
#pragma unroll
        for (int c = 0; c < MAXC; ++c) v[c] = nv[c];
        load_row(z + XW, nv);
        // run starts and ends per chunk (wave-uniform masks)
        unsigned long long st[MAXC], en[MAXC];
#pragma unroll
        for (int c = 0; c < MAXC; ++c) {
            if (c >= chunks) {
                st[c] = en[c] = 0ull;
                continue;
            }
            const int x = c * 64 + lane;
            // left neighbour: lane - 1, lane 0 takes lane 63 of the previous chunk
            const uint32_t left_edge = c > 0 ? (uint32_t)__builtin_amdgcn_readlane((int)v[c > 0 ? c - 1 : 0], 63) : 0u;
            const uint32_t right_edge =
                c + 1 < chunks ? (uint32_t)__builtin_amdgcn_readlane((int)v[c + 1 < MAXC ? c + 1 : c], 0) : 0u;
            const uint32_t lm = (uint32_t)__builtin_amdgcn_update_dpp((int)left_edge, (int)v[c], 0x138, 0xf, 0xf, false);
            const uint32_t lp = (uint32_t)__builtin_amdgcn_update_dpp((int)right_edge, (int)v[c], 0x130, 0xf, 0xf, false);
            const bool in = x < nx;
            st[c] = __ballot(in && (x == 0 || lm != v[c]));
            en[c] = __ballot(in && (x == nx - 1 || lp != v[c]));
        }
        // nearest end after each chunk, from the right (scalars)
        int next_end[MAXC];
        {
            int ne = nx - 1;
#pragma unroll
            for (int c = MAXC - 1; c >= 0; --c) {
                next_end[c] = ne;
                if (c < chunks && en[c]) ne = c * 64 + __ffsll(en[c]) - 1;
            }
        }
        int prev_start = 0;                             // last start before the chunk
        int nrun = 0;                                   // listed runs of this row (wave-uniform)
#pragma unroll
        for (int c = 0; c < MAXC; ++c) {
            if (c >= chunks) break;
            const int x = c * 64 + lane;
            const uint32_t l = v[c];
            int out = 0;
            bool first = false;
            int s0 = 0, e0 = 0;
            if (x < nx && l != 0u) {
                bad |= label_negative(L(l));
                const unsigned long long below = st[c] & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
                s0 = below ? c * 64 + 63 - __clzll(below) : prev_start;
                const unsigned long long above = en[c] & ~((1ull << lane) - 1ull);
                e0 = above ? c * 64 + __ffsll(above) - 1 : next_end[c];
                out = min(x - s0 + 1, e0 - x + 1);
                if (BOX && x == s0) {                   // first voxel of its run
                    if ((uint64_t)L(l) > box.max_label || label_negative(L(l))) bad = true;
                    else first = true;
                }
            }
            if (x < nx) g[row * nx + x] = (uint16_t)out;
            if (st[c]) prev_start = c * 64 + 63 - __clzll(st[c]);
            if (BOX) {
                const unsigned long long fm = __ballot(first);
                if (fm) {
                    const int k = __popcll(fm);
                    if (nrun + k > XRUNS) {
                        merge_runs(nrun, z);
                        nrun = 0;
                    }
                    if (first) {
                        const int at = nrun + __popcll(fm & ((1ull << lane) - 1ull));
                        runs[3 * at] = l;
                        runs[3 * at + 1] = (uint32_t)s0;
                        runs[3 * at + 2] = (uint32_t)e0;
                    }
                    nrun += k;
                }
            }
        }
        if (BOX && nrun) merge_runs(nrun, z);
    }
    if (__ballot(bad) && lane == 0) atomicOr(err, ERR_LABEL);
    if (BOX) {
        __syncthreads();
        for (int t = threadIdx.x; t < XBOX_TAB; t += blockDim.x) {
            const uint32_t u = s_key[t];
            if (u == 0u) continue;
            atomicMin(&box.bb[0 * box.nlab + u], s_bb[0][t]);
            atomicMax(&box.bb[1 * box.nlab + u], s_bb[1][t]);
            atomicMin(&box.bb[2 * box.nlab + u], y);
            atomicMax(&box.bb[3 * box.nlab + u], y);
            atomicMin(&box.bb[4 * box.nlab + u], s_bb[2][t]);
            atomicMax(&box.bb[5 * box.nlab + u], s_bb[3][t]);
        }
    }
}

__global__ void init_boxes(int32_t* bb, uint32_t nlab) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l < nlab) init_box(bb, nlab, l);
}

// One line pass along y (AXIS = 1, input g, squared here) or z (AXIS = 2, input d2).
// A block owns 64 consecutive x and LINE_T consecutive positions along the pass
// axis; it stages the values of those positions plus LINE_H on each side in LDS
// (coalesced row loads), each packed with two run-boundary bits (derived from the
// labels, staged first in the same words): LINE_BLK_DN when
// the position's label differs from the next one's (a search walking down from
// the next position stops there), LINE_BLK_UP when it differs from the previous
// one's; positions outside the image count as background.  Each voxel's outward
// search then reads one LDS word per step and direction.  A search that runs past
// the staged range continues with global loads (exact either way).  The y pass
// stages its 11-bit input g in both direction forms instead: the low half holds g,
// or 0 below a run end (LINE_BLK_DN), the high half g, or 0 past a run start
// (LINE_BLK_UP), so a step's candidate is a 24-bit square of one half.
// With W (anisotropic spacing) a step k along the axis costs wa k^2 (wa = the
// squared spacing of the axis) and the y pass stages w_x g^2 in the word form of
// the z pass.
constexpr int LINE_T = 64, LINE_H = 24, LINE_ROWS = LINE_T + 2 * LINE_H;
// Staged row r is held by the wave r mod 8 (rows ty + 8 q); the output rows LINE_H + ty
// + 8 j must be the waves' own staged rows (the y pass reads its per-row flags from
// registers), so the halo is a multiple of the wave count.
static_assert(LINE_H % 8 == 0 && LINE_T % 8 == 0, "line-pass rows must stay with their staging wave");
constexpr uint32_t LINE_BLK_DN = 1u << 31, LINE_BLK_UP = 1u << 30, LINE_VAL = LINE_BLK_UP - 1u;

// Value a staged word offers a search walking down (up) to it: its value, or 0 when
// the word carries the boundary bit of that direction (a site of another label).
__device__ __forceinline__ int line_down(uint32_t w) { return (int)(w & LINE_VAL) & ~((int)w >> 31); }
__device__ __forceinline__ int line_up(uint32_t w) {    // w << 1: the up bit becomes the sign
    return (int)((uint32_t)max((int)(w << 1), 0) >> 1);
}

// Smaller of the values offered by the word wl below and wh above the searching position.
template <int AXIS>
__device__ __forceinline__ int line_pair(uint32_t wl, uint32_t wh) {
    if (AXIS == 1) {
        const int a = (int)(wl & 0xffffu), b = (int)(wh >> 16);
        return min(__mul24(a, a), __mul24(b, b));
    }
    return min(line_down(wl), line_up(wh));
}

template <typename L, int AXIS, typename F, bool W = false>
__global__ void __launch_bounds__(512)
edt_pass_line(const L* __restrict__ lab, const F* __restrict__ f, int32_t* __restrict__ out,
              int nx, int ny, int nz, int wa = 1, int wprev = 1) {
    constexpr bool HALF = AXIS == 1 && !W;                 // the y pass's half-word form
    // one LDS word per staged position: first the labels (to derive the boundary
    // bits), then the value with its bits; the values wait in registers meanwhile
    __shared__ uint32_t s_val[LINE_ROWS * 64];
    constexpr int RPT = LINE_ROWS / 8;                     // staged rows per thread
    const int tx = threadIdx.x;                            // 64 x 8: one wave per ty
    const int ty = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int x = blockIdx.x * 64 + tx;
    const int n = AXIS == 1 ? ny : nz;
    const int a0 = (AXIS == 1 ? blockIdx.y : blockIdx.z) * LINE_T;
    const int o = AXIS == 1 ? blockIdx.z : blockIdx.y;     // the other coordinate
    const ptrdiff_t stride = AXIS == 1 ? (ptrdiff_t)nx : (ptrdiff_t)nx * ny;
    const size_t base = AXIS == 1 ? (size_t)o * ny * nx : (size_t)o * nx;   // (a = 0, x = 0)
    const int lo = max(0, a0 - LINE_H), hi = min(n, a0 + LINE_T + LINE_H);
    uint32_t vals[RPT];
    uint32_t obj = 0u;                                     // y pass: bit q, staged row ty + 8q holds g >= 1
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = ty + 8 * q;
        const int a = a0 - LINE_H + r;
        L lv = L(0);
        int fv = 0;
        if (a >= lo && a < hi && x < nx) {
            const size_t i = base + (size_t)a * stride + x;
            lv = lab[i];
            fv = (int)f[i];
            if (W && AXIS == 1) fv = wprev * fv * fv;          // weighted g^2
        }
        s_val[r * 64 + tx] = (uint32_t)lv;
        vals[q] = (uint32_t)fv;
        if (HALF && fv > 0) obj |= 1u << q;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = ty + 8 * q;
        const uint32_t lv = s_val[r * 64 + tx];
        const bool dn = r + 1 >= LINE_ROWS || s_val[(r + 1) * 64 + tx] != lv;
        const bool up = r == 0 || s_val[(r - 1) * 64 + tx] != lv;
        if (HALF)
            vals[q] = (dn ? 0u : vals[q]) | ((up ? 0u : vals[q]) << 16);
        else
            vals[q] |= (dn ? LINE_BLK_DN : 0u) | (up ? LINE_BLK_UP : 0u);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RPT; ++q) s_val[(ty + 8 * q) * 64 + tx] = vals[q];
    __syncthreads();
    if (x >= nx) return;
    for (int r = LINE_H + ty; r < LINE_H + LINE_T; r += 8) {
        const int p = a0 - LINE_H + r;
        if (p >= n) break;
        const size_t i = base + (size_t)p * stride + x;
        const uint32_t w0 = s_val[r * 64 + tx];
        int best;                                          // 0: background, no search
        if (HALF) {
            // g from either half; a run of one position (both halves 0) has D2 = 1
            const int g0 = (int)max(w0 & 0xffffu, w0 >> 16);
            best = g0 ? __mul24(g0, g0) : (int)((obj >> ((r - ty) >> 3)) & 1u);
        } else {
            best = (int)(w0 & LINE_VAL);
        }
        // A position past a label boundary offers k^2 (its run ends there); once that
        // happens best <= k^2 and every later candidate, at least (k + 1)^2, loses, so
        // the search needs no per-direction stop: it ends when k^2 reaches best.
        int k = 1;
        // step cost wa k^2 (k^2 unless W)
        auto cost = [&](int kk) { return W ? wa * kk * kk : kk * kk; };
        // staged range, four steps per round: the eight words are loaded first so
        // that their latencies overlap; the steps are then applied in order.  The
        // wave runs while any lane still searches (a lane already done only takes
        // candidates that cannot lower its best), so the loop needs no exec masks.
        while (__ballot(cost(k) < best) != 0ull && r - k - 3 >= 0 && r + k + 3 < LINE_ROWS) {
            uint32_t wl[4], wh[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                wl[u] = s_val[(r - k - u) * 64 + tx];
                wh[u] = s_val[(r + k + u) * 64 + tx];
            }
            int kk = cost(k);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                best = min(best, kk + line_pair<HALF ? 1 : 2>(wl[u], wh[u]));
                kk += (W ? wa : 1) * (2 * (k + u) + 1);
            }
            k += 4;
        }
        for (; __ballot(cost(k) < best) != 0ull; ++k) {
            if (r - k < 0 || r + k >= LINE_ROWS) break;           // leave the staged range
            const uint32_t wl = s_val[(r - k) * 64 + tx], wh = s_val[(r + k) * 64 + tx];
            best = min(best, cost(k) + line_pair<HALF ? 1 : 2>(wl, wh));
        }
        const L l = cost(k) < best ? lab[i] : L(0);
        for (; cost(k) < best; ++k) {                              // beyond the halo
            const int kk = cost(k);
            int cl = kk, ch = kk;
            if (p - k >= 0 && lab[i - k * stride] == l) {
                const int v = (int)f[i - k * stride];
                cl += AXIS == 1 ? (W ? wprev : 1) * v * v : v;
            }
            if (p + k < n && lab[i + k * stride] == l) {
                const int v = (int)f[i + k * stride];
                ch += AXIS == 1 ? (W ? wprev : 1) * v * v : v;
            }
            best = min(best, min(cl, ch));
        }
        out[i] = best;
    }
}

size_t edt_scratch_bytes(const Geom& g) {
    const size_t gbytes = (g.n * sizeof(uint16_t) + 255) & ~size_t(255);
    return gbytes + (g.ndim == 3 ? g.n * sizeof(int32_t) : 0);
}

template <typename L>
static lt_status edt_typed(lt_ctx* ctx, const L* lab, const Geom& g, int32_t* dist, void* scratch,
                           hipStream_t s, const BoxTarget* box, const Spacing& sp) {
    // scratch: g (uint16) then d2 (int32, 3D only)
    const size_t gbytes = (g.n * sizeof(uint16_t) + 255) & ~size_t(255);
    uint16_t* gx = (uint16_t*)scratch;
    int32_t* d2 = (int32_t*)((char*)scratch + gbytes);
    {
        ProfScope _p(ctx, s, "edt_pass_x");
        const int chunks = (g.nx + 63) / 64;
        // many small blocks (about 32 per compute unit): 0.27 ms at 512^3 against 0.38 with
        // 16 waves and 4 blocks per unit
        const int gz = loop_extent(g.nz, g.ny, ctx, 32);
        const int zper = (g.nz + gz - 1) / gz;
        const int nzb = (g.nz + zper - 1) / zper;
        const dim3 grid(1, g.ny, nzb);
        const BoxTarget nobox{nullptr, 0, 0};
        auto launch = [&](auto maxc) {
            constexpr int MC = decltype(maxc)::value;
            if (box)
                edt_pass_x<L, true, MC><<<grid, 64 * XW, 0, s>>>(lab, gx, g.nx, g.ny, g.nz, ctx->d_err, *box, zper);
            else
                edt_pass_x<L, false, MC><<<grid, 64 * XW, 0, s>>>(lab, gx, g.nx, g.ny, g.nz, ctx->d_err, nobox, zper);
        };
        if (chunks <= 4) launch(std::integral_constant<int, 4>());
        else if (chunks <= 8) launch(std::integral_constant<int, 8>());
        else if (chunks <= 16) launch(std::integral_constant<int, 16>());
        else launch(std::integral_constant<int, 32>());
    }
    const dim3 lblock(64, 8);
    const int bx = (g.nx + 63) / 64;
    const dim3 gy(bx, (g.ny + LINE_T - 1) / LINE_T, g.nz);
    const dim3 gz(bx, g.ny, (g.nz + LINE_T - 1) / LINE_T);
    const bool w = !sp.unit();
    int32_t* ydst = g.ndim == 2 ? dist : d2;
    {
        ProfScope _p(ctx, s, "edt_pass_y");
        if (w)
            edt_pass_line<L, 1, uint16_t, true><<<gy, lblock, 0, s>>>(lab, gx, ydst, g.nx, g.ny, g.nz, sp.wy, sp.wx);
        else
            edt_pass_line<L, 1, uint16_t><<<gy, lblock, 0, s>>>(lab, gx, ydst, g.nx, g.ny, g.nz);
    }
    if (g.ndim == 3) {
        ProfScope _p(ctx, s, "edt_pass_z");
        if (w)
            edt_pass_line<L, 2, int32_t, true><<<gz, lblock, 0, s>>>(lab, d2, dist, g.nx, g.ny, g.nz, sp.wz, 1);
        else
            edt_pass_line<L, 2, int32_t><<<gz, lblock, 0, s>>>(lab, d2, dist, g.nx, g.ny, g.nz);
    }
    return hip_check(hipGetLastError(), "edt launch");
}

lt_status launch_edt(lt_ctx* ctx, const void* labels, lt_dtype dt, const Geom& g, int32_t* dist_sq,
                     void* scratch, hipStream_t s, const BoxTarget* box, const Spacing* sp) {
    const Spacing unit;
    const Spacing& spc = sp ? *sp : unit;
    switch (dt) {
        case LT_U16: return edt_typed(ctx, (const uint16_t*)labels, g, dist_sq, scratch, s, box, spc);
        case LT_I32: return edt_typed(ctx, (const int32_t*)labels, g, dist_sq, scratch, s, box, spc);
        case LT_U32: return edt_typed(ctx, (const uint32_t*)labels, g, dist_sq, scratch, s, box, spc);
    }
    return set_error(LT_E_DTYPE, "unknown dtype");
}

lt_status launch_init_boxes(lt_ctx* ctx, int32_t* bb, uint32_t nlab, hipStream_t s) {
    ProfScope _p(ctx, s, "init_boxes");
    init_boxes<<<(nlab + 255) / 256, 256, 0, s>>>(bb, nlab);
    return hip_check(hipGetLastError(), "box init launch");
}

}  // namespace lt
