// Shell extraction, per-object reductions and closed forms.
//
// Method, Roundness: contour / surface voxels are object voxels with a background
// neighbour in the 4-neighbourhood (2D) or the corresponding 6 face neighbours
// (3D); here outside the image and other labels count as background.  Roundness is
// the mean local thickness over those voxels divided by the object's largest local
// thickness, the radius of the maximal inscribed circle/sphere.
// Method, Sphericity: a spheroid (3D) or ellipse (2D) with semi-axis a = mean local
// thickness and the object's volume / area replaces the measured surface /
// perimeter in Wadell's sphericity (Background, Eq. 1) or the perimeter
// sphericity P_c / P_o.
//
// Sums of radii are accumulated in Q.23 fixed point in uint64, so results do not
// depend on atomic order.  A wave reduces each run of equal labels among its 64
// lanes (consecutive x); blocks merge the runs of a 64 x 16 x 8 brick per label in
// LDS before one set of global atomics per label and block.
#include <math.h>

#include "lt_internal.h"

namespace lt {

// Wave totals by inclusive DPP scans (row_shr 1, 2, 4, 8 within rows of 16 lanes,
// then row_bcast:15 and row_bcast:31; lanes without a source take the identity 0),
// read from lane 63: VALU only, no LDS permutes.  Every lane of the wave must be active.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_add_u64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)v, CTRL, ROWS, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)(uint32_t)(v >> 32), CTRL, ROWS, 0xf, false);
    return v + (((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
    v = dpp_add_u64<0x111, 0xf>(v);       // row_shr:1
    v = dpp_add_u64<0x112, 0xf>(v);       // row_shr:2
    v = dpp_add_u64<0x114, 0xf>(v);       // row_shr:4
    v = dpp_add_u64<0x118, 0xf>(v);       // row_shr:8
    v = dpp_add_u64<0x142, 0xa>(v);       // row_bcast:15
    v = dpp_add_u64<0x143, 0xc>(v);       // row_bcast:31
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return ((uint64_t)hi << 32) | lo;
}

// Wave maximum of non-negative values (identity 0).
__device__ __forceinline__ int wave_max_i32(int v) {
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false));
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false));
    return __builtin_amdgcn_readlane(v, 63);
}

__global__ void zero_measure_arrays(uint64_t* vol, uint64_t* shc, int32_t* mx, uint64_t* sq,
                                    uint64_t* ssq, uint32_t nlab) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlab) return;
    vol[l] = 0;
    shc[l] = 0;
    mx[l] = 0;
    sq[l] = 0;
    ssq[l] = 0;
}

constexpr int SUM_TAB = 64;                  // labels per block table
constexpr int SUM_BY = 16, SUM_BZ = 8;       // block brick: 64 (x) x SUM_BY (y) x SUM_BZ (z)

// Label table slot (open addressing, linear probing, key 0 = empty); -1 if full.
__device__ __forceinline__ int sum_slot(uint32_t* keys, uint32_t l) {
    int h = (int)((l * 2654435761u) >> 7) & (SUM_TAB - 1);
    for (int probe = 0; probe < SUM_TAB; ++probe) {
        const uint32_t k = atomicCAS(&keys[h], 0u, l);
        if (k == 0u || k == l) return h;
        h = (h + 1) & (SUM_TAB - 1);
    }
    return -1;
}

// One block per 64 x 16 x 8 brick.  Per slice, each wave (one 64-voxel row segment)
// reduces every run of equal labels among its lanes; the run's lead lane merges the
// totals into the block's label table with LDS atomics (global atomics if the table
// is full); the table is flushed to global memory once per block.
template <int NDIM, typename L>
__global__ void __launch_bounds__(1024)
object_sums(const L* __restrict__ lab, const int32_t* __restrict__ lt, int nx, int ny, int nz,
            uint32_t max_label, uint64_t* __restrict__ vol, uint64_t* __restrict__ shc,
            int32_t* __restrict__ mx, uint64_t* __restrict__ sq, uint64_t* __restrict__ ssq,
            uint32_t* err) {
    __shared__ uint32_t s_key[SUM_TAB];
    __shared__ unsigned long long s_vol[SUM_TAB], s_shc[SUM_TAB], s_sq[SUM_TAB], s_ssq[SUM_TAB];
    __shared__ int s_mx[SUM_TAB];
    const int wy = __builtin_amdgcn_readfirstlane((int)threadIdx.y);   // one wave per row of the brick
    const int tid = wy * 64 + threadIdx.x;
    if (tid < SUM_TAB) {
        s_key[tid] = 0u;
        s_vol[tid] = s_shc[tid] = s_sq[tid] = s_ssq[tid] = 0ull;
        s_mx[tid] = 0;
    }
    __syncthreads();
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * SUM_BY + wy;
    const size_t plane = (size_t)ny * nx;
    const int z0 = blockIdx.z * SUM_BZ, z1 = min(nz, z0 + SUM_BZ);
    for (int z = z0; z < z1; ++z) {
        const size_t i = (size_t)z * plane + (size_t)y * nx + x;
        uint32_t l = 0;
        int v = 0;
        bool shell = false;
        uint64_t q = 0;
        if (x < nx && y < ny) {
            const L raw = lab[i];
            if (raw != 0) {
                if (label_negative(raw) || (uint64_t)raw > max_label) {
                    atomicOr(err, ERR_LABEL);
                } else {
                    l = (uint32_t)raw;
                    v = lt[i];
                    q = radius_q23(v);
                    shell = x == 0 || x == nx - 1 || y == 0 || y == ny - 1 ||
                            lab[i - 1] != raw || lab[i + 1] != raw || lab[i - nx] != raw ||
                            lab[i + nx] != raw;
                    if (NDIM == 3 && !shell)
                        shell = z == 0 || z == nz - 1 || lab[i - plane] != raw || lab[i + plane] != raw;
                }
            }
        }
        uint64_t active = __ballot(l != 0);
        while (active) {
            const int lead = __ffsll((unsigned long long)active) - 1;
            const uint32_t L0 = (uint32_t)__builtin_amdgcn_readlane((int)l, lead);
            const bool in = (l == L0);
            const uint64_t m = __ballot(in);
            const uint64_t sm = __ballot(in && shell);
            const uint64_t s1 = wave_sum_u64(in ? q : 0);
            const uint64_t s2 = wave_sum_u64(in && shell ? q : 0);
            const int m1 = wave_max_i32(in ? v : 0);
            if ((int)threadIdx.x == lead) {
                const int slot = sum_slot(s_key, L0);
                if (slot >= 0) {
                    atomicAdd(&s_vol[slot], (unsigned long long)__popcll(m));
                    atomicAdd(&s_sq[slot], (unsigned long long)s1);
                    atomicMax(&s_mx[slot], m1);
                    if (sm) {
                        atomicAdd(&s_shc[slot], (unsigned long long)__popcll(sm));
                        atomicAdd(&s_ssq[slot], (unsigned long long)s2);
                    }
                } else {
                    atomicAdd((unsigned long long*)&vol[L0], (unsigned long long)__popcll(m));
                    atomicAdd((unsigned long long*)&sq[L0], (unsigned long long)s1);
                    atomicMax(&mx[L0], m1);
                    if (sm) {
                        atomicAdd((unsigned long long*)&shc[L0], (unsigned long long)__popcll(sm));
                        atomicAdd((unsigned long long*)&ssq[L0], (unsigned long long)s2);
                    }
                }
            }
            active &= ~m;
        }
    }
    __syncthreads();
    if (tid < SUM_TAB && s_key[tid] != 0u) {
        const uint32_t L0 = s_key[tid];
        atomicAdd((unsigned long long*)&vol[L0], s_vol[tid]);
        atomicAdd((unsigned long long*)&sq[L0], s_sq[tid]);
        atomicMax(&mx[L0], s_mx[tid]);
        if (s_shc[tid]) {
            atomicAdd((unsigned long long*)&shc[L0], s_shc[tid]);
            atomicAdd((unsigned long long*)&ssq[L0], s_ssq[tid]);
        }
    }
}

// Local-thickness histogram (32 bins of sqrt(LT_sq) / R, R^2 = the object's max):
// bin k (1..32) is the smallest k with 1024 * LT_sq <= k^2 * R^2, decided in integers.
template <typename L>
__global__ void __launch_bounds__(256)
lt_histogram(const L* __restrict__ lab, const int32_t* __restrict__ lt, size_t n,
             uint32_t max_label, const int32_t* __restrict__ mx, uint32_t* __restrict__ hist) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const L raw = lab[i];
    if (raw == 0 || label_negative(raw) || (uint64_t)raw > max_label) return;
    const uint32_t l = (uint32_t)raw;
    const int64_t num = 1024 * (int64_t)lt[i];
    const int64_t r2 = mx[l];
    if (r2 <= 0) return;
    int k = (int)ceil(32.0 * sqrt((double)lt[i] / (double)r2));
    k = min(max(k, 1), 32);
    while (k < 32 && (int64_t)k * k * r2 < num) ++k;
    while (k > 1 && (int64_t)(k - 1) * (k - 1) * r2 >= num) --k;
    atomicAdd(&hist[(size_t)l * 32 + (k - 1)], 1u);
}

// Surface of the spheroid with equal semi-axes a and third semi-axis c, in FP32
// with forms that stay accurate near the sphere and for extreme elongation:
// with q = min(a, c) / max(a, c), e^2 = (1 - q)(1 + q);
//   oblate  (c < a): S = 2 pi a^2 (1 + q^2 artanh(e) / e),  artanh(e) = log((1 + e) / q);
//   prolate (c > a): S = 2 pi a^2 (1 + asin(e) / (q e)),     asin(e)   = atan2(e, q);
// and Taylor series of artanh(e)/e and asin(e)/e in e^2 when e^2 < 2^-7.
__device__ float spheroid_surface_f32(float a, float c) {
    const float two_pi_a2 = 6.2831853f * a * a;
    if (c == a) return 2.0f * two_pi_a2;
    const bool oblate = c < a;
    const float q = oblate ? c / a : a / c;
    const float e2 = (1.0f - q) * (1.0f + q);
    float ratio;                                  // artanh(e)/e or asin(e)/e
    if (e2 < 0.0078125f) {
        if (oblate)
            ratio = 1.0f + e2 * (1.0f / 3.0f + e2 * (1.0f / 5.0f + e2 * (1.0f / 7.0f + e2 * (1.0f / 9.0f))));
        else
            ratio = 1.0f + e2 * (1.0f / 6.0f + e2 * (3.0f / 40.0f + e2 * (5.0f / 112.0f + e2 * (35.0f / 1152.0f))));
    } else {
        const float e = sqrtf(e2);
        ratio = oblate ? logf((1.0f + e) / q) / e : atan2f(e, q) / e;
    }
    return oblate ? two_pi_a2 * (1.0f + q * q * ratio) : two_pi_a2 * (1.0f + ratio / q);
}

__global__ void closed_forms_kernel(const uint64_t* __restrict__ vol, const uint64_t* __restrict__ sq,
                                    const int32_t* __restrict__ mx, const uint64_t* __restrict__ shc,
                                    const uint64_t* __restrict__ ssq, uint32_t nlab, int ndim,
                                    float* __restrict__ mean_lt, float* __restrict__ shell_mean,
                                    float* __restrict__ sph, float* __restrict__ rnd,
                                    const uint32_t* __restrict__ hist, float* __restrict__ hist_out,
                                    float vsize) {
    const uint32_t l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= nlab) return;
    const float nan = __int_as_float(0x7fc00000);
    const uint64_t V = vol[l];
    if (V == 0) {
        mean_lt[l] = shell_mean[l] = sph[l] = rnd[l] = nan;
        if (hist_out)
            for (int k = 0; k < 32; ++k) hist_out[(size_t)l * 32 + k] = nan;
        return;
    }
    const float a = (float)((double)sq[l] / SUM_SCALE / (double)V);
    const float Vf = (float)V * vsize;            // physical volume (area): voxels x voxel size
    const float R = sqrtf((float)mx[l]);
    mean_lt[l] = a;
    const uint64_t ns = shc[l];
    if (ns) {
        const float sm = (float)((double)ssq[l] / SUM_SCALE / (double)ns);
        shell_mean[l] = sm;
        rnd[l] = sm / R;
    } else {
        shell_mean[l] = rnd[l] = nan;
    }
    const float pi = 3.14159265f;
    if (ndim == 3) {
        const float c = 3.0f * Vf / (4.0f * pi * a * a);
        const float S = spheroid_surface_f32(a, c);
        const float k6 = cbrtf(6.0f * Vf);
        sph[l] = 1.46459189f * k6 * k6 / S;      // pi^(1/3) (6V)^(2/3) / S
    } else {
        const float b = Vf / (pi * a);
        const float po = pi * (3.0f * (a + b) - sqrtf((3.0f * a + b) * (a + 3.0f * b)));
        sph[l] = 2.0f * sqrtf(pi * Vf) / po;
    }
    if (hist_out) {
        const float inv = 1.0f / (float)V;
        for (int k = 0; k < 32; ++k) hist_out[(size_t)l * 32 + k] = (float)hist[(size_t)l * 32 + k] * inv;
    }
}

static inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

size_t measures_scratch_bytes(uint32_t max_label) {
    const size_t nlab = (size_t)max_label + 1;
    return 2 * align256(nlab * sizeof(uint64_t)) + align256(nlab * 32 * sizeof(uint32_t));
}

__global__ void fill_u32(uint32_t* p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

// Per-object accumulators in the caller's scratch: Q.23 radius sums of all and of
// shell voxels, then the histogram counts.
struct MeasureScratch {
    uint64_t *sq, *ssq;
    uint32_t* hist;
};

static MeasureScratch measure_scratch(void* scratch, size_t nlab) {
    char* base = (char*)scratch;
    MeasureScratch m;
    m.sq = (uint64_t*)base;
    m.ssq = (uint64_t*)(base + align256(nlab * sizeof(uint64_t)));
    m.hist = (uint32_t*)(base + 2 * align256(nlab * sizeof(uint64_t)));
    return m;
}

lt_status launch_measures_zero(lt_ctx* ctx, uint32_t max_label, const lt_measures* out, void* scratch,
                               hipStream_t s, MeasureSums* sums) {
    const size_t nlab = (size_t)max_label + 1;
    const MeasureScratch m = measure_scratch(scratch, nlab);
    {
        ProfScope _p(ctx, s, "zero_measure_arrays");
        zero_measure_arrays<<<(unsigned)((nlab + 255) / 256), 256, 0, s>>>(out->volume, out->shell_count,
                                                                          out->max_lt_sq, m.sq, m.ssq,
                                                                          (uint32_t)nlab);
    }
    if (sums) *sums = MeasureSums{out->volume, out->shell_count, out->max_lt_sq, m.sq, m.ssq};
    return hip_check(hipGetLastError(), "measures launch");
}

template <typename L>
static lt_status measures_finish_typed(lt_ctx* ctx, const L* lab, const Geom& g, const int32_t* lt,
                                       uint32_t max_label, const lt_measures* out, void* scratch,
                                       hipStream_t s, float vsize) {
    const size_t nlab = (size_t)max_label + 1;
    const MeasureScratch m = measure_scratch(scratch, nlab);
    if (out->hist32) {
        {
            ProfScope _p(ctx, s, "fill_u32");
            fill_u32<<<(unsigned)min((size_t)4096, (nlab * 32 + 255) / 256), 256, 0, s>>>(m.hist, nlab * 32);
        }
        if (g.n > 0) {
            ProfScope _p(ctx, s, "lt_histogram");
            lt_histogram<L><<<(unsigned)((g.n + 255) / 256), 256, 0, s>>>(lab, lt, g.n, max_label,
                                                                         out->max_lt_sq, m.hist);
        }
    }
    {
        ProfScope _p(ctx, s, "closed_forms");
        closed_forms_kernel<<<(unsigned)((nlab + 255) / 256), 256, 0, s>>>(
            out->volume, m.sq, out->max_lt_sq, out->shell_count, m.ssq, (uint32_t)nlab, g.ndim, out->mean_lt,
            out->shell_mean_lt, out->sphericity, out->roundness, m.hist, out->hist32, vsize);
    }
    return hip_check(hipGetLastError(), "measures launch");
}

template <typename L>
static lt_status measures_typed(lt_ctx* ctx, const L* lab, const Geom& g, const int32_t* lt,
                                uint32_t max_label, const lt_measures* out, void* scratch,
                                hipStream_t s, float vsize) {
    MeasureSums sums;
    lt_status st = launch_measures_zero(ctx, max_label, out, scratch, s, &sums);
    if (st) return st;
    if (g.n > 0) {
        ProfScope _p(ctx, s, "object_sums");
        const dim3 grid((g.nx + 63) / 64, (g.ny + SUM_BY - 1) / SUM_BY, (g.nz + SUM_BZ - 1) / SUM_BZ),
            blk(64, SUM_BY);
        if (g.ndim == 3)
            object_sums<3, L><<<grid, blk, 0, s>>>(lab, lt, g.nx, g.ny, g.nz, max_label, sums.vol, sums.shc,
                                                   sums.mx, sums.sq, sums.ssq, ctx->d_err);
        else
            object_sums<2, L><<<grid, blk, 0, s>>>(lab, lt, g.nx, g.ny, 1, max_label, sums.vol, sums.shc,
                                                   sums.mx, sums.sq, sums.ssq, ctx->d_err);
    }
    return measures_finish_typed(ctx, lab, g, lt, max_label, out, scratch, s, vsize);
}

lt_status launch_measures(lt_ctx* ctx, const void* labels, lt_dtype dt, const Geom& g,
                          const int32_t* lt_sq, uint32_t max_label, const lt_measures* out,
                          void* scratch, hipStream_t s, float vsize) {
    switch (dt) {
        case LT_U16:
            return measures_typed(ctx, (const uint16_t*)labels, g, lt_sq, max_label, out, scratch, s, vsize);
        case LT_I32:
            return measures_typed(ctx, (const int32_t*)labels, g, lt_sq, max_label, out, scratch, s, vsize);
        case LT_U32:
            return measures_typed(ctx, (const uint32_t*)labels, g, lt_sq, max_label, out, scratch, s, vsize);
    }
    return set_error(LT_E_DTYPE, "unknown dtype");
}

lt_status launch_measures_finish(lt_ctx* ctx, const void* labels, lt_dtype dt, const Geom& g,
                                 const int32_t* lt_sq, uint32_t max_label, const lt_measures* out,
                                 void* scratch, hipStream_t s, float vsize) {
    switch (dt) {
        case LT_U16:
            return measures_finish_typed(ctx, (const uint16_t*)labels, g, lt_sq, max_label, out, scratch, s, vsize);
        case LT_I32:
            return measures_finish_typed(ctx, (const int32_t*)labels, g, lt_sq, max_label, out, scratch, s, vsize);
        case LT_U32:
            return measures_finish_typed(ctx, (const uint32_t*)labels, g, lt_sq, max_label, out, scratch, s, vsize);
    }
    return set_error(LT_E_DTYPE, "unknown dtype");
}

lt_status launch_closed_forms(const uint64_t* volume, const uint64_t* sum_lt_q, const int32_t* max_lt_sq,
                              const uint64_t* shell_count, const uint64_t* shell_sum_q, uint32_t n,
                              int ndim, float* mean_lt, float* shell_mean_lt, float* sphericity,
                              float* roundness, hipStream_t s) {
    closed_forms_kernel<<<(n + 255) / 256, 256, 0, s>>>(volume, sum_lt_q, max_lt_sq, shell_count,
                                                        shell_sum_q, n, ndim, mean_lt, shell_mean_lt,
                                                        sphericity, roundness, nullptr, nullptr, 1.0f);
    return hip_check(hipGetLastError(), "closed forms launch");
}

}  // namespace lt
