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
#include "lt_internal.h"

namespace lt {

// Pass x: one block per row.  A wave takes 64 consecutive voxels; ballots give the
// positions where a run starts (label differs from the left neighbour, or x = 0)
// and ends.  A voxel's run [s, e] is found from the nearest start at or before it
// and the nearest end at or after it -- in its own chunk via bit scans, otherwise
// from the per-chunk extremes kept in LDS -- and g = min(x - s + 1, e - x + 1).
// With BOX, the first voxel of every object run also merges (z, y, run) into the
// block's label table in LDS (bounding boxes of the fused pipeline); a block walks
// consecutive slices of one row index y, so an object's runs meet in few blocks,
// and the table is flushed to the global boxes once per block.
constexpr int XBOX_TAB = 128;
constexpr int XR = 8;                // slices per round of the x pass

template <typename L, bool BOX>
__global__ void __launch_bounds__(1024)
edt_pass_x(const L* __restrict__ lab, uint16_t* __restrict__ g, int nx, int ny, int nz, uint32_t* err,
           BoxTarget box, int zper) {
    __shared__ unsigned long long s_start[XR][ROW_MAX_CHUNKS], s_end[XR][ROW_MAX_CHUNKS];
    __shared__ uint32_t s_key[BOX ? XBOX_TAB : 1];
    __shared__ int s_bb[6][BOX ? XBOX_TAB : 1];
    const int lane = threadIdx.x & 63, wid = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int nw = blockDim.x >> 6;
    const int chunks = (nx + 63) >> 6;
    const int y = blockIdx.y;
    if (BOX) {
        for (int t = threadIdx.x; t < XBOX_TAB; t += blockDim.x) {
            s_key[t] = 0u;
            s_bb[0][t] = s_bb[2][t] = s_bb[4][t] = 0x7fffffff;
            s_bb[1][t] = s_bb[3][t] = s_bb[5][t] = -1;
        }
        __syncthreads();
    }
    const int zb = blockIdx.z * zper, ze = min(nz, zb + zper);
  // XR slices per round: their loads are in flight together and they share the
  // round's two barriers
  for (int z0 = zb; z0 < ze; z0 += XR) {
    for (int c = wid; c < chunks; c += nw) {
        const int x = c * 64 + lane;
        L lv[XR], lm[XR], lp[XR];
#pragma unroll
        for (int q = 0; q < XR; ++q) {
            const bool ok = z0 + q < ze && x < nx;
            const L* r = lab + ((size_t)(z0 + q) * ny + y) * nx;
            lv[q] = ok ? r[x] : L(0);
            lm[q] = ok && x > 0 ? r[x - 1] : L(0);
            lp[q] = ok && x + 1 < nx ? r[x + 1] : L(0);
        }
#pragma unroll
        for (int q = 0; q < XR; ++q) {
            const bool ok = z0 + q < ze && x < nx;
            bool st = false, en = false;
            if (ok) {
                if (label_negative(lv[q])) atomicOr(err, ERR_LABEL);
                st = x == 0 || lm[q] != lv[q];
                en = x == nx - 1 || lp[q] != lv[q];
            }
            const unsigned long long ms = __ballot(st), me = __ballot(en);
            if (lane == 0) {
                s_start[q][c] = ms;
                s_end[q][c] = me;
            }
        }
    }
    __syncthreads();
    for (int c = wid; c < chunks; c += nw) {
        const int x = c * 64 + lane;
        if (x >= nx) continue;
#pragma unroll
        for (int q = 0; q < XR; ++q) {
            const int z = z0 + q;
            if (z >= ze) break;
            const size_t row = (size_t)z * ny + y;
            const L l = lab[row * nx + x];
            int out = 0;
            if (l != 0) {
                const unsigned long long below = s_start[q][c] & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
                int s0;
                if (below) {
                    s0 = c * 64 + 63 - __clzll(below);
                } else {
                    int cc = c - 1;
                    while (s_start[q][cc] == 0ull) --cc;       // chunk 0 always has a start at x = 0
                    s0 = cc * 64 + 63 - __clzll(s_start[q][cc]);
                }
                const unsigned long long above = s_end[q][c] & ~((1ull << lane) - 1ull);
                int e0;
                if (above) {
                    e0 = c * 64 + __ffsll(above) - 1;
                } else {
                    int cc = c + 1;
                    while (s_end[q][cc] == 0ull) ++cc;         // the last chunk ends at x = nx - 1
                    e0 = cc * 64 + __ffsll(s_end[q][cc]) - 1;
                }
                out = min(x - s0 + 1, e0 - x + 1);
                if (BOX && x == s0) {                          // first voxel of its run
                    if ((uint64_t)l > box.max_label) {
                        atomicOr(err, ERR_LABEL);
                    } else if (!label_negative(l)) {
                        const uint32_t u = (uint32_t)l;
                        const int slot = lds_slot<XBOX_TAB>(s_key, u);
                        if (slot >= 0) {
                            atomicMin(&s_bb[0][slot], z);
                            atomicMax(&s_bb[1][slot], z);
                            atomicMin(&s_bb[2][slot], y);
                            atomicMax(&s_bb[3][slot], y);
                            atomicMin(&s_bb[4][slot], s0);
                            atomicMax(&s_bb[5][slot], e0);
                        } else {
                            atomicMin(&box.bb[0 * box.nlab + u], z);
                            atomicMax(&box.bb[1 * box.nlab + u], z);
                            atomicMin(&box.bb[2 * box.nlab + u], y);
                            atomicMax(&box.bb[3 * box.nlab + u], y);
                            atomicMin(&box.bb[4 * box.nlab + u], s0);
                            atomicMax(&box.bb[5 * box.nlab + u], e0);
                        }
                    }
                }
            }
            g[row * nx + x] = (uint16_t)out;
        }
    }
    __syncthreads();                                     // the masks are reused by the next round
  }
    if (BOX) {
        for (int t = threadIdx.x; t < XBOX_TAB; t += blockDim.x) {
            const uint32_t u = s_key[t];
            if (u == 0u) continue;
            atomicMin(&box.bb[0 * box.nlab + u], s_bb[0][t]);
            atomicMax(&box.bb[1 * box.nlab + u], s_bb[1][t]);
            atomicMin(&box.bb[2 * box.nlab + u], s_bb[2][t]);
            atomicMax(&box.bb[3 * box.nlab + u], s_bb[3][t]);
            atomicMin(&box.bb[4 * box.nlab + u], s_bb[4][t]);
            atomicMax(&box.bb[5 * box.nlab + u], s_bb[5][t]);
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
constexpr int LINE_T = 64, LINE_H = 32, LINE_ROWS = LINE_T + 2 * LINE_H;
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
        const int threads = min(1024, ((g.nx + 63) / 64) * 64);
        const int gz = loop_extent(g.nz, g.ny, ctx);
        const int zper = (g.nz + gz - 1) / gz;
        const int nzb = (g.nz + zper - 1) / zper;
        if (box)
            edt_pass_x<L, true><<<dim3(1, g.ny, nzb), threads, 0, s>>>(lab, gx, g.nx, g.ny, g.nz, ctx->d_err, *box,
                                                                     zper);
        else
            edt_pass_x<L, false><<<dim3(1, g.ny, nzb), threads, 0, s>>>(lab, gx, g.nx, g.ny, g.nz, ctx->d_err,
                                                                      BoxTarget{nullptr, 0, 0}, zper);
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
