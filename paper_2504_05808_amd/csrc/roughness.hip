// Roughness-filtered roundness and the 0-1 remap of roundness.
//
// Discussion (applicability of the roundness approximation): the contour / surface
// roundness responds to surface roughness, and that influence can be controlled by
// filtering.  The filter used here acts on the shell values before they are
// averaged: a shell voxel's local thickness is replaced by the largest shell local
// thickness found within half-width w along x, then along y, then along z (2D: x,
// then y), each step taking only positions that carry the voxel's own label.  A
// bump narrower than w loses its small inscribed balls to the larger values around
// it; w = 0 gives the plain roundness (Method, Roundness).
//   F_0(p) = LT_sq(p) if p is a shell voxel (D(p) = 1: a face neighbour is of
//            another label or outside the image), else 0;
//   F_a(p) = max{ F_{a-1}(p + o e_a) : |o| <= w, label(p + o e_a) = label(p) }.
// Filtered roundness of object l = mean over its shell voxels of sqrt(F_last) over
// sqrt(max LT_sq of l).
// Results, performance on the 2D charts: roundness can be mapped onto the usual
// 0-1 range through the smallest observed value m: R' = (R - m) / (1 - m).
//
// Each pass stages a tile and its +-w halo (labels and values) in LDS; the last
// pass reduces per label (per-lane running totals merged into a block label table
// in LDS when the label changes, Q.23 radius sums in uint64) instead of writing its
// field.
#include <math.h>

#include <algorithm>

#include "lt_internal.h"

namespace lt {

constexpr int RF_MAXW = 16;          // largest half-width
constexpr int RF_T = 32;             // line positions per block (y and z passes)
constexpr int RF_TAB = 64;           // labels per block table

// x pass: one wave per row segment of RF_XSEG voxels, staged with its halo.
constexpr int RF_XSEG = 256;

template <typename L>
__global__ void __launch_bounds__(256)
rough_x(const L* __restrict__ lab, const int32_t* __restrict__ D, const int32_t* __restrict__ lt, int nx,
        int nrows, int w, int32_t* __restrict__ out) {
    __shared__ uint32_t s_l[4][RF_XSEG + 2 * RF_MAXW];
    __shared__ int32_t s_f[4][RF_XSEG + 2 * RF_MAXW];
    const int lane = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int row = blockIdx.y * 4 + wv;
    if (row >= nrows) return;                          // wave-uniform; no block barrier below
    const int x0 = blockIdx.x * RF_XSEG;
    const int seg = min(RF_XSEG, nx - x0);
    const size_t rb = (size_t)row * nx;
    // the segment's labels first, then D and LT of its object voxels, all loads of a
    // stage in flight together
    constexpr int KX = (RF_XSEG + 2 * RF_MAXW + 63) / 64;
    uint32_t lv[KX];
#pragma unroll
    for (int q = 0; q < KX; ++q) {
        const int k = lane + 64 * q, x = x0 - w + k;
        lv[q] = (k < seg + 2 * w && x >= 0 && x < nx) ? (uint32_t)lab[rb + x] : 0u;
    }
    int32_t dv[KX], tv[KX];
#pragma unroll
    for (int q = 0; q < KX; ++q) {
        const int x = x0 - w + lane + 64 * q;
        dv[q] = lv[q] != 0u ? D[rb + x] : 0;
        tv[q] = lv[q] != 0u ? lt[rb + x] : 0;
    }
#pragma unroll
    for (int q = 0; q < KX; ++q) {
        const int k = lane + 64 * q;
        if (k < seg + 2 * w) {
            s_l[wv][k] = lv[q];
            s_f[wv][k] = dv[q] == 1 ? tv[q] : 0;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int c = lane; c < seg; c += 64) {
        const uint32_t me = s_l[wv][c + w];
        int32_t best = 0;
        if (me != 0u)
            for (int o = 0; o <= 2 * w; ++o)
                if (s_l[wv][c + o] == me) best = max(best, s_f[wv][c + o]);
        out[rb + x0 + c] = best;
    }
}

struct RoughSums {
    uint64_t* shc;      // shell voxels
    uint64_t* ssq;      // sum of round(sqrt(F) * 2^23) over the shell
    int32_t* mx;        // largest LT_sq of the object
};

// Running totals of one label in one lane.
struct RoughRun {
    uint32_t l;
    uint64_t shc, ssq;
    int mx;
};

__device__ __forceinline__ void rough_merge(uint32_t* s_key, unsigned long long* s_shc, unsigned long long* s_ssq,
                                            int* s_mx, const RoughSums& sums, const RoughRun& r) {
    if (r.l == 0u) return;
    const int slot = lds_slot<RF_TAB>(s_key, r.l);
    if (slot >= 0) {
        atomicMax(&s_mx[slot], r.mx);
        if (r.shc) {
            atomicAdd(&s_shc[slot], (unsigned long long)r.shc);
            atomicAdd(&s_ssq[slot], (unsigned long long)r.ssq);
        }
    } else {
        atomicMax(&sums.mx[r.l], r.mx);
        if (r.shc) {
            atomicAdd((unsigned long long*)&sums.shc[r.l], (unsigned long long)r.shc);
            atomicAdd((unsigned long long*)&sums.ssq[r.l], (unsigned long long)r.ssq);
        }
    }
}

// y / z pass (AXIS 1 / 2): block = 64 x-columns x 4 waves over RF_T consecutive line
// positions; the tile and its +-w halo along the line are staged in LDS.  With
// FINAL the pass reduces per label instead of writing its field.
template <int AXIS, bool FINAL, typename L>
__global__ void __launch_bounds__(256)
rough_line(const L* __restrict__ lab, const int32_t* __restrict__ fin, const int32_t* __restrict__ D,
           const int32_t* __restrict__ lt, int nx, int ny, int nz, int w, uint32_t max_label,
           int32_t* __restrict__ out, RoughSums sums, uint32_t* err) {
    // dynamic LDS: labels then values, (RF_T + 2 w) rows of 64 each
    extern __shared__ uint32_t s_dyn[];
    uint32_t (*s_l)[64] = (uint32_t (*)[64])s_dyn;
    int32_t (*s_f)[64] = (int32_t (*)[64])(s_dyn + (RF_T + 2 * w) * 64);
    __shared__ uint32_t s_key[RF_TAB];
    __shared__ unsigned long long s_shc[RF_TAB], s_ssq[RF_TAB];
    __shared__ int s_mx[RF_TAB];
    const int lane = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int tid = wv * 64 + lane;
    if (FINAL && tid < RF_TAB) {
        s_key[tid] = 0u;
        s_shc[tid] = s_ssq[tid] = 0ull;
        s_mx[tid] = 0;
    }
    const int x = blockIdx.x * 64 + lane;
    const int n_line = AXIS == 1 ? ny : nz;
    const int t0 = blockIdx.y * RF_T;
    const int other = blockIdx.z;                      // z for the y pass, y for the z pass
    const size_t stride = AXIS == 1 ? (size_t)nx : (size_t)nx * ny;
    const size_t base = AXIS == 1 ? (size_t)other * ny * nx + x : (size_t)other * nx + x;
    const bool xin = x < nx;
    RoughRun run{0u, 0ull, 0ull, 0};
#pragma unroll 4
    for (int k = wv; k < RF_T + 2 * w; k += 4) {
        const int t = t0 - w + k;
        uint32_t l = 0u;
        int32_t f = 0;
        if (xin && t >= 0 && t < n_line) {
            const size_t i = base + (size_t)t * stride;
            l = (uint32_t)lab[i];
            f = fin[i];
        }
        s_l[k][lane] = l;
        s_f[k][lane] = f;
    }
    __syncthreads();
    // final pass: D and LT of this wave's positions, fetched before the reduction
    constexpr int KF = RF_T / 4;
    int32_t dfin[KF], tfin[KF];
    if (FINAL) {
#pragma unroll
        for (int q = 0; q < KF; ++q) {
            const int k = wv + 4 * q, t = t0 + k;
            const bool in = xin && t < n_line && s_l[k + w][lane] != 0u;
            const size_t i = base + (size_t)t * stride;
            dfin[q] = in ? D[i] : 0;
            tfin[q] = in ? lt[i] : 0;
        }
    }
#pragma unroll
    for (int q = 0; q < KF; ++q) {
        const int k = wv + 4 * q;
        const int t = t0 + k;
        const bool in = xin && t < n_line;
        const uint32_t me = in ? s_l[k + w][lane] : 0u;
        int32_t best = 0;
        if (me != 0u)
            for (int o = 0; o <= 2 * w; ++o)
                if (s_l[k + o][lane] == me) best = max(best, s_f[k + o][lane]);
        if (!FINAL) {
            if (in) out[base + (size_t)t * stride] = best;
            continue;
        }
        // final pass: per-label shell count, Q.23 sum of sqrt(F) and largest LT, as
        // per-lane running totals of one label (labels change rarely along a line)
        if (me == 0u) continue;
        if ((uint64_t)me > max_label) {
            atomicOr(err, ERR_LABEL);
            continue;
        }
        if (me != run.l) {
            rough_merge(s_key, s_shc, s_ssq, s_mx, sums, run);
            run = RoughRun{me, 0ull, 0ull, 0};
        }
        run.mx = max(run.mx, tfin[q]);
        if (dfin[q] == 1) {
            ++run.shc;
            run.ssq += radius_q23(best);
        }
    }
    if (FINAL) {
        rough_merge(s_key, s_shc, s_ssq, s_mx, sums, run);
        __syncthreads();
        if (tid < RF_TAB && s_key[tid] != 0u) {
            const uint32_t L0 = s_key[tid];
            atomicMax(&sums.mx[L0], s_mx[tid]);
            if (s_shc[tid]) {
                atomicAdd((unsigned long long*)&sums.shc[L0], s_shc[tid]);
                atomicAdd((unsigned long long*)&sums.ssq[L0], s_ssq[tid]);
            }
        }
    }
}

__global__ void rough_zero(RoughSums s, uint32_t nlab) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlab) return;
    s.shc[l] = 0;
    s.ssq[l] = 0;
    s.mx[l] = 0;
}

// roundness_w = (ssq / 2^23 / shc) / sqrt(mx); NaN without shell voxels.
__global__ void rough_finish(RoughSums s, uint32_t nlab, float* __restrict__ roundness) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlab) return;
    const uint64_t n = s.shc[l];
    double r = __builtin_nan("");
    if (n > 0 && s.mx[l] > 0) r = ((double)s.ssq[l] / SUM_SCALE / (double)n) / sqrt((double)s.mx[l]);
    roundness[l] = (float)r;
}

size_t rough_scratch_bytes(const Geom& g, uint32_t max_label) {
    const size_t field = (g.n * sizeof(int32_t) + 255) & ~size_t(255);
    const size_t nl = (size_t)max_label + 1;
    return 2 * field + 2 * ((nl * 8 + 255) & ~size_t(255)) + ((nl * 4 + 255) & ~size_t(255));
}

template <typename L>
static lt_status rough_typed(lt_ctx* ctx, const L* lab, const Geom& g, const int32_t* D, const int32_t* lt,
                             uint32_t max_label, int w, int32_t* fa, int32_t* fb, RoughSums sums,
                             hipStream_t s) {
    const int nrows = g.nz * g.ny;
    {
        ProfScope p(ctx, s, "rough_x");
        rough_x<L><<<dim3((g.nx + RF_XSEG - 1) / RF_XSEG, (nrows + 3) / 4), dim3(64, 4), 0, s>>>(lab, D, lt, g.nx,
                                                                                          nrows, w, fa);
    }
    lt_status st = hip_check(hipGetLastError(), "rough_x launch");
    if (st) return st;
    const dim3 blk(64, 4);
    const size_t lds = (size_t)(RF_T + 2 * w) * 64 * 8;
    if (g.ndim == 2) {
        ProfScope p(ctx, s, "rough_y_final");
        rough_line<1, true, L><<<dim3((g.nx + 63) / 64, (g.ny + RF_T - 1) / RF_T, 1), blk, lds, s>>>(
            lab, fa, D, lt, g.nx, g.ny, 1, w, max_label, nullptr, sums, ctx->d_err);
        return hip_check(hipGetLastError(), "rough_y launch");
    }
    {
        ProfScope p(ctx, s, "rough_y");
        rough_line<1, false, L><<<dim3((g.nx + 63) / 64, (g.ny + RF_T - 1) / RF_T, g.nz), blk, lds, s>>>(
            lab, fa, D, lt, g.nx, g.ny, g.nz, w, max_label, fb, sums, ctx->d_err);
    }
    if ((st = hip_check(hipGetLastError(), "rough_y launch"))) return st;
    {
        ProfScope p(ctx, s, "rough_z_final");
        rough_line<2, true, L><<<dim3((g.nx + 63) / 64, (g.nz + RF_T - 1) / RF_T, g.ny), blk, lds, s>>>(
            lab, fb, D, lt, g.nx, g.ny, g.nz, w, max_label, nullptr, sums, ctx->d_err);
    }
    return hip_check(hipGetLastError(), "rough_z launch");
}

lt_status launch_filtered_roundness(lt_ctx* ctx, const void* labels, lt_dtype dt, const Geom& g,
                                    const int32_t* D, const int32_t* lt, uint32_t max_label, int w,
                                    float* roundness, void* scratch, hipStream_t s) {
    const size_t field = (g.n * sizeof(int32_t) + 255) & ~size_t(255);
    const size_t nl = (size_t)max_label + 1;
    char* p = (char*)scratch;
    int32_t* fa = (int32_t*)p;
    int32_t* fb = (int32_t*)(p + field);
    RoughSums sums;
    sums.shc = (uint64_t*)(p + 2 * field);
    sums.ssq = (uint64_t*)(p + 2 * field + ((nl * 8 + 255) & ~size_t(255)));
    sums.mx = (int32_t*)(p + 2 * field + 2 * ((nl * 8 + 255) & ~size_t(255)));
    const uint32_t nlab = max_label + 1;
    {
        ProfScope pz(ctx, s, "rough_zero");
        rough_zero<<<(nlab + 255) / 256, 256, 0, s>>>(sums, nlab);
    }
    lt_status st = hip_check(hipGetLastError(), "rough_zero launch");
    if (st) return st;
    if (g.n > 0) {
        switch (dt) {
            case LT_U16: st = rough_typed(ctx, (const uint16_t*)labels, g, D, lt, max_label, w, fa, fb, sums, s); break;
            case LT_I32: st = rough_typed(ctx, (const int32_t*)labels, g, D, lt, max_label, w, fa, fb, sums, s); break;
            case LT_U32: st = rough_typed(ctx, (const uint32_t*)labels, g, D, lt, max_label, w, fa, fb, sums, s); break;
        }
        if (st) return st;
    }
    {
        ProfScope pf(ctx, s, "rough_finish");
        rough_finish<<<(nlab + 255) / 256, 256, 0, s>>>(sums, nlab, roundness);
    }
    return hip_check(hipGetLastError(), "rough_finish launch");
}

// ---------------------------------------------------------------- 0-1 remap

// Order-preserving key of a float (smaller value, smaller key) and back.
__device__ __forceinline__ uint32_t fkey(float v) {
    const uint32_t b = __float_as_uint(v);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float fkey_inv(uint32_t k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

// Smallest finite value, as a key; the word starts at the key of +inf.
__global__ void remap_min(const float* __restrict__ r, uint32_t n, uint32_t* __restrict__ mkey) {
    uint32_t best = 0xff800000u;                        // fkey(+inf)
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const float v = r[i];
        if (isfinite(v)) best = min(best, fkey(v));
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) best = min(best, (uint32_t)__shfl_xor((int)best, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMin(mkey, best);
}

__global__ void remap_init(uint32_t* mkey, float r_min) {
    *mkey = isnan(r_min) ? 0xff800000u : fkey(r_min);
}

// R' = (R - m) / (1 - m); every finite R maps to 1 when m >= 1; NaN stays NaN.
__global__ void remap_apply(const float* __restrict__ r, uint32_t n, const uint32_t* __restrict__ mkey,
                            float* __restrict__ out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float m = fkey_inv(*mkey);
    const float v = r[i];
    float o = v;
    if (isfinite(v)) o = m >= 1.0f ? 1.0f : (v - m) / (1.0f - m);
    out[i] = o;
}

lt_status launch_remap(lt_ctx* ctx, const float* r, uint32_t n, float r_min, float* out, void* scratch,
                       hipStream_t s) {
    uint32_t* mkey = (uint32_t*)scratch;
    {
        ProfScope p(ctx, s, "remap_init");
        remap_init<<<1, 1, 0, s>>>(mkey, r_min);
    }
    lt_status st = hip_check(hipGetLastError(), "remap_init launch");
    if (st) return st;
    if (isnan(r_min)) {
        const uint32_t blocks = std::min<uint32_t>((n + 255) / 256, (uint32_t)ctx->n_cu * 4);
        ProfScope p(ctx, s, "remap_min");
        remap_min<<<blocks, 256, 0, s>>>(r, n, mkey);
        if ((st = hip_check(hipGetLastError(), "remap_min launch"))) return st;
    }
    {
        ProfScope p(ctx, s, "remap_apply");
        remap_apply<<<(n + 255) / 256, 256, 0, s>>>(r, n, mkey, out);
    }
    return hip_check(hipGetLastError(), "remap_apply launch");
}

}  // namespace lt
