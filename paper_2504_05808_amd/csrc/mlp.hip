// Learned sphericity correction: a 34 -> 64 -> 64 -> 64 -> 1 SiLU MLP trained and run
// with BF16 MFMA products accumulated in FP32.
//
// Inputs per object: the 32-bin local-thickness histogram, log V and
// mean LT / V^(1/3), standardised with the training set's mean and spread.  The
// network predicts the standardised difference between a mesh-based sphericity and
// the spheroid closed form; lt_mlp_correct adds it back to the closed form and keeps
// the closed form wherever the guard rejects the prediction (a feature outside the
// training range, a non-finite output, or a correction larger than any seen in
// training).
//
// A training step is two launches: a fused forward + backward per chunk of rows
// (weights and activations in LDS, v_mfma_f32_16x16x16_bf16 tiles) writing partial
// gradients, and a fixed-order reduction of the partials fused with AdamW; so a
// step is deterministic.  Inference is one fused launch.  Master weights and AdamW
// moments are FP32; the BF16 copies used by the products are refreshed after every
// update.  mfma_gemm (one wave per 16x16 output tile) serves lt_bf16_gemm.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <random>
#include <vector>

#include "lt_internal.h"

namespace lt {

constexpr int MLP_IN = 34, MLP_INP = 48, MLP_H = 64, MLP_OUTP = 16;
// parameter layout (FP32 master and BF16 copy share offsets)
constexpr int OFF_W1 = 0;                              // [64][48]
constexpr int OFF_B1 = OFF_W1 + MLP_H * MLP_INP;       // [64]
constexpr int OFF_W2 = OFF_B1 + MLP_H;                 // [64][64]
constexpr int OFF_B2 = OFF_W2 + MLP_H * MLP_H;
constexpr int OFF_W3 = OFF_B2 + MLP_H;
constexpr int OFF_B3 = OFF_W3 + MLP_H * MLP_H;
constexpr int OFF_W4 = OFF_B3 + MLP_H;                 // [16][64], row 0 used
constexpr int OFF_B4 = OFF_W4 + MLP_OUTP * MLP_H;      // [16], entry 0 used
constexpr int N_PARAM = OFF_B4 + MLP_OUTP;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {           // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// C[M x N] = A[M x K] * B[K x N]; A(i, k) = A[i*lda + k] (ta = 0) or A[k*lda + i]
// (ta = 1); B(k, j) = B[k*ldb + j] (tb = 0) or B[j*ldb + k] (tb = 1).  M, N, K are
// multiples of 16.  One wave per 16x16 tile of C: lane l supplies A(i, k..k+3) with
// i = l % 16, k = 4 (l / 16), and B(k..k+3, j) with j = l % 16; it receives
// C(4 (l / 16) + r, l % 16), r = 0..3.
__global__ void __launch_bounds__(256)
mfma_gemm(int M, int N, int K, const uint16_t* __restrict__ A, int lda, int ta,
          const uint16_t* __restrict__ B, int ldb, int tb, float* __restrict__ C, int ldc) {
    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int tiles_n = N / 16;
    if (tile >= (M / 16) * tiles_n) return;
    const int m0 = (tile / tiles_n) * 16, n0 = (tile % tiles_n) * 16;
    const int r16 = lane & 15, kq = (lane >> 4) * 4;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x4 a, b;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = k0 + kq + j;
            const int i = m0 + r16, n = n0 + r16;
            a[j] = (short)(ta ? A[(size_t)k * lda + i] : A[(size_t)i * lda + k]);
            b[j] = (short)(tb ? B[(size_t)n * ldb + k] : B[(size_t)k * ldb + n]);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) C[(size_t)(m0 + kq + r) * ldc + n0 + r16] = acc[r];
}

__global__ void mlp_to_bf16(const float* __restrict__ w, uint16_t* __restrict__ wb, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = f2bf(w[i]);
}

// Features of lt_object_measures outputs: hist (32), log V, mean LT / V^(1/3).
__global__ void mlp_features(const float* __restrict__ hist, const uint64_t* __restrict__ vol,
                             const float* __restrict__ mean_lt, uint32_t n, float* __restrict__ x) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const float V = (float)vol[r];
    for (int k = 0; k < 32; ++k) x[(size_t)r * MLP_IN + k] = hist[(size_t)r * 32 + k];
    x[(size_t)r * MLP_IN + 32] = logf(V);
    x[(size_t)r * MLP_IN + 33] = mean_lt[r] / cbrtf(V);
}

__global__ void mlp_guard(const float* __restrict__ x, const float* __restrict__ s_lt,
                          const float* __restrict__ delta, int n, const float* __restrict__ fmin,
                          const float* __restrict__ fmax, float max_abs_delta, float* __restrict__ s_corr,
                          uint32_t* __restrict__ n_fallback) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    bool ok = isfinite(delta[r]) && fabsf(delta[r]) <= max_abs_delta && isfinite(s_lt[r]);
    for (int k = 0; k < MLP_IN && ok; ++k) {
        const float f = x[(size_t)r * MLP_IN + k];
        ok = f >= fmin[k] && f <= fmax[k];
    }
    s_corr[r] = ok ? s_lt[r] + delta[r] : s_lt[r];
    if (!ok) atomicAdd(n_fallback, 1u);
}

// ------------------------------------------------------------------ fused step
//
// A training step runs as two kernels.  mlp_fused_fwd_bwd: one workgroup per chunk
// of FB_ROWS rows keeps the BF16 weights, its activations and their gradients in
// LDS; forward (standardisation, three bias + SiLU layers, output), loss gradient
// and backward through every layer run back to back, and the chunk writes its
// partial weight and bias gradients (and its sum of squared errors).  Rows past the
// batch get a zero loss gradient, so they add nothing.  mlp_reduce_adamw sums the
// chunks' partials in chunk order (deterministic) into the gradient, then applies
// AdamW and refreshes the BF16 copy.  The BF16 rounding points are those of the
// unfused layers: inputs, hidden activations, output gradient and hidden
// pre-activation gradients enter the products as BF16; bias gradients sum the FP32
// pre-activation gradients.
constexpr int FB_ROWS = 32;                            // rows per workgroup
constexpr int FB_THREADS = 256;

// One 16 x 16 tile of C = A B from LDS operands with element strides:
// A(i, k) = A[i * ai + k * ak], B(k, j) = B[k * bk + j * bj].  Lane l supplies
// A(m0 + l % 16, k0 + 4 (l / 16) + q) and B(k0 + 4 (l / 16) + q, n0 + l % 16) and
// holds C(m0 + 4 (l / 16) + r, n0 + l % 16) in acc[r].
__device__ __forceinline__ f32x4 lds_tile(const uint16_t* A, int ai, int ak, const uint16_t* B, int bk, int bj,
                                          int m0, int n0, int K, int lane) {
    const int r16 = lane & 15, kq = (lane >> 4) * 4;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf16x4 a, b;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = k0 + kq + q;
            a[q] = (short)A[(m0 + r16) * ai + k * ak];
            b[q] = (short)B[k * bk + (n0 + r16) * bj];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    return acc;
}

struct FusedLds {
    uint16_t *w1, *w2, *w3, *w4;       // BF16 weights [64][48], [64][64], [64][64], [16][64]
    float* b;                          // b1 b2 b3 [64 each], b4 [16]
    uint16_t* xb;                      // [R][48]
    uint16_t *h1, *h2, *h3;            // [R][64]
    float *z1, *z2, *z3;               // [R][64] pre-activations
    float* o;                          // [R][16]
    uint16_t* dob;                     // [R][16]
    float* d;                          // [R][64] FP32 gradient of the current layer
    uint16_t* db;                      // [R][64] its BF16 copy
};

__host__ __device__ constexpr size_t fused_lds_bytes(bool train) {
    return (size_t)(MLP_H * MLP_INP + 2 * MLP_H * MLP_H + MLP_OUTP * MLP_H) * 2 + (3 * MLP_H + MLP_OUTP) * 4 +
           (size_t)FB_ROWS * MLP_INP * 2 + 3 * (size_t)FB_ROWS * MLP_H * 2 +
           (train ? 3 * (size_t)FB_ROWS * MLP_H * 4 : 0) + (size_t)FB_ROWS * MLP_OUTP * 4 +
           (train ? (size_t)FB_ROWS * MLP_OUTP * 2 + (size_t)FB_ROWS * MLP_H * 6 : 0) + 64;
}

__device__ FusedLds fused_layout(char* base, bool train) {
    FusedLds L;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        char* p = base + at;
        at += (bytes + 7) & ~size_t(7);
        return p;
    };
    L.w1 = (uint16_t*)take(MLP_H * MLP_INP * 2);
    L.w2 = (uint16_t*)take(MLP_H * MLP_H * 2);
    L.w3 = (uint16_t*)take(MLP_H * MLP_H * 2);
    L.w4 = (uint16_t*)take(MLP_OUTP * MLP_H * 2);
    L.b = (float*)take((3 * MLP_H + MLP_OUTP) * 4);
    L.xb = (uint16_t*)take(FB_ROWS * MLP_INP * 2);
    L.h1 = (uint16_t*)take(FB_ROWS * MLP_H * 2);
    L.h2 = (uint16_t*)take(FB_ROWS * MLP_H * 2);
    L.h3 = (uint16_t*)take(FB_ROWS * MLP_H * 2);
    L.z1 = train ? (float*)take(FB_ROWS * MLP_H * 4) : nullptr;
    L.z2 = train ? (float*)take(FB_ROWS * MLP_H * 4) : nullptr;
    L.z3 = train ? (float*)take(FB_ROWS * MLP_H * 4) : nullptr;
    L.o = (float*)take(FB_ROWS * MLP_OUTP * 4);
    L.dob = train ? (uint16_t*)take(FB_ROWS * MLP_OUTP * 2) : nullptr;
    L.d = train ? (float*)take(FB_ROWS * MLP_H * 4) : nullptr;
    L.db = train ? (uint16_t*)take(FB_ROWS * MLP_H * 2) : nullptr;
    return L;
}

// Weights, biases and the chunk's standardised BF16 inputs into LDS.
__device__ void fused_load(const FusedLds& L, const uint16_t* __restrict__ wb, const float* __restrict__ w,
                           const float* __restrict__ x, int B, int r0, const float* __restrict__ mean,
                           const float* __restrict__ inv_std, int tid) {
    for (int i = tid; i < MLP_H * MLP_INP; i += FB_THREADS) L.w1[i] = wb[OFF_W1 + i];
    for (int i = tid; i < MLP_H * MLP_H; i += FB_THREADS) {
        L.w2[i] = wb[OFF_W2 + i];
        L.w3[i] = wb[OFF_W3 + i];
    }
    for (int i = tid; i < MLP_OUTP * MLP_H; i += FB_THREADS) L.w4[i] = wb[OFF_W4 + i];
    for (int i = tid; i < MLP_H; i += FB_THREADS) {
        L.b[i] = w[OFF_B1 + i];
        L.b[MLP_H + i] = w[OFF_B2 + i];
        L.b[2 * MLP_H + i] = w[OFF_B3 + i];
    }
    if (tid < MLP_OUTP) L.b[3 * MLP_H + tid] = w[OFF_B4 + tid];
    for (int i = tid; i < FB_ROWS * MLP_INP; i += FB_THREADS) {
        const int r = i / MLP_INP, c = i % MLP_INP;
        float v = 0.f;
        if (c < MLP_IN && r0 + r < B) {
            v = (x[(size_t)(r0 + r) * MLP_IN + c] - mean[c]) * inv_std[c];
            if (!isfinite(v)) v = 0.f;
        }
        L.xb[i] = f2bf(v);
    }
}

// Forward of the chunk: z = h_prev W^T + b (kept with TRAIN), h = bf16(silu(z)); o =
// h3 W4^T (without b4).  Each wave takes tiles round-robin.
template <bool TRAIN>
__device__ void fused_forward(const FusedLds& L, int wid, int lane) {
    const uint16_t* hin[3] = {L.xb, L.h1, L.h2};
    uint16_t* hout[3] = {L.h1, L.h2, L.h3};
    float* zout[3] = {L.z1, L.z2, L.z3};
    const uint16_t* wt[3] = {L.w1, L.w2, L.w3};
    const int kin[3] = {MLP_INP, MLP_H, MLP_H};
    const int r16 = lane & 15, kq = (lane >> 4) * 4;
    for (int layer = 0; layer < 3; ++layer) {
        const int K = kin[layer];
        for (int t = wid; t < (FB_ROWS / 16) * (MLP_H / 16); t += FB_THREADS / 64) {
            const int m0 = (t / (MLP_H / 16)) * 16, n0 = (t % (MLP_H / 16)) * 16;
            const f32x4 acc = lds_tile(hin[layer], K, 1, wt[layer], 1, K, m0, n0, K, lane);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + kq + r, col = n0 + r16;
                const float v = acc[r] + L.b[layer * MLP_H + col];
                if (TRAIN) zout[layer][row * MLP_H + col] = v;
                hout[layer][row * MLP_H + col] = f2bf(v / (1.f + expf(-v)));
            }
        }
        __syncthreads();
    }
    for (int t = wid; t < FB_ROWS / 16; t += FB_THREADS / 64) {
        const int m0 = t * 16;
        const f32x4 acc = lds_tile(L.h3, MLP_H, 1, L.w4, 1, MLP_H, m0, 0, MLP_H, lane);
#pragma unroll
        for (int r = 0; r < 4; ++r) L.o[(m0 + kq + r) * MLP_OUTP + r16] = acc[r];
    }
    __syncthreads();
}

// Training: forward, loss gradient and backward of one chunk; partial gradients to
// part[chunk][N_PARAM] and the chunk's sum of squared errors to sse[chunk].
__global__ void __launch_bounds__(FB_THREADS)
mlp_fused_fwd_bwd(const float* __restrict__ x, const float* __restrict__ y, int B,
                  const float* __restrict__ consts, const float* __restrict__ w, const uint16_t* __restrict__ wb,
                  float* __restrict__ part, float* __restrict__ sse) {
    extern __shared__ __align__(16) char lds[];
    const FusedLds L = fused_layout(lds, true);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int chunk = blockIdx.x, r0 = chunk * FB_ROWS;
    fused_load(L, wb, w, x, B, r0, consts, consts + MLP_IN, tid);
    __syncthreads();
    fused_forward<true>(L, wid, lane);
    float* P = part + (size_t)chunk * N_PARAM;
    const int r16 = lane & 15, kq = (lane >> 4) * 4;
    // loss gradient: d = 2 (p - y) / B in output column 0 (rows past B: 0)
    if (tid < FB_ROWS) {
        const int r = tid;
        float d = 0.f;
        if (r0 + r < B) d = 2.f * (L.o[r * MLP_OUTP] + L.b[3 * MLP_H] - y[r0 + r]) / (float)B;
        for (int c = 0; c < MLP_OUTP; ++c) L.dob[r * MLP_OUTP + c] = c == 0 ? f2bf(d) : (uint16_t)0;
        L.d[r] = d;                                        // column 0 of d, for db4
    }
    __syncthreads();
    if (tid == 0) {                                        // db4 and the squared errors, in row order
        float db4 = 0.f, sq = 0.f;
        for (int r = 0; r < FB_ROWS && r0 + r < B; ++r) {
            db4 += L.d[r];
            const float e = L.o[r * MLP_OUTP] + L.b[3 * MLP_H] - y[r0 + r];
            sq += e * e;
        }
        P[OFF_B4] = db4;
        sse[chunk] = sq;
    }
    if (tid > 0 && tid < MLP_OUTP) P[OFF_B4 + tid] = 0.f;
    // dW4 [16][64] = dob^T h3; dh3 [R][64] = dob W4
    for (int t = wid; t < MLP_H / 16; t += FB_THREADS / 64) {
        const f32x4 acc = lds_tile(L.dob, 1, MLP_OUTP, L.h3, MLP_H, 1, 0, t * 16, FB_ROWS, lane);
#pragma unroll
        for (int r = 0; r < 4; ++r) P[OFF_W4 + (kq + r) * MLP_H + t * 16 + r16] = acc[r];
    }
    __syncthreads();                                       // L.d (column 0) is read above
    for (int t = wid; t < (FB_ROWS / 16) * (MLP_H / 16); t += FB_THREADS / 64) {
        const int m0 = (t / (MLP_H / 16)) * 16, n0 = (t % (MLP_H / 16)) * 16;
        const f32x4 acc = lds_tile(L.dob, MLP_OUTP, 1, L.w4, MLP_H, 1, m0, n0, MLP_OUTP, lane);
#pragma unroll
        for (int r = 0; r < 4; ++r) L.d[(m0 + kq + r) * MLP_H + n0 + r16] = acc[r];
    }
    __syncthreads();
    const float* zs[3] = {L.z1, L.z2, L.z3};
    const uint16_t* hprev[3] = {L.xb, L.h1, L.h2};
    const uint16_t* wt[3] = {L.w1, L.w2, L.w3};
    const int kin[3] = {MLP_INP, MLP_H, MLP_H};
    const int offw[3] = {OFF_W1, OFF_W2, OFF_W3}, offb[3] = {OFF_B1, OFF_B2, OFF_B3};
    for (int layer = 2; layer >= 0; --layer) {
        // dz = dh * silu'(z) (FP32 and BF16)
        for (int i = tid; i < FB_ROWS * MLP_H; i += FB_THREADS) {
            const float v = zs[layer][i];
            const float sg = 1.f / (1.f + expf(-v));
            const float g = L.d[i] * sg * (1.f + v * (1.f - sg));
            L.d[i] = g;
            L.db[i] = f2bf(g);
        }
        __syncthreads();
        // db = column sums of dz in row order
        if (tid < MLP_H) {
            float sb = 0.f;
            for (int r = 0; r < FB_ROWS; ++r) sb += L.d[r * MLP_H + tid];
            P[offb[layer] + tid] = sb;
        }
        // dW [64][K] = dz^T h_prev
        const int K = kin[layer];
        for (int t = wid; t < (MLP_H / 16) * (K / 16); t += FB_THREADS / 64) {
            const int m0 = (t / (K / 16)) * 16, n0 = (t % (K / 16)) * 16;
            const f32x4 acc = lds_tile(L.db, 1, MLP_H, hprev[layer], K, 1, m0, n0, FB_ROWS, lane);
#pragma unroll
            for (int r = 0; r < 4; ++r) P[offw[layer] + (m0 + kq + r) * K + n0 + r16] = acc[r];
        }
        if (layer == 0) break;
        __syncthreads();                                   // every lane has read L.d for db
        // dh_prev [R][64] = dz W (layer's weights [64][K], K = 64 here)
        for (int t = wid; t < (FB_ROWS / 16) * (MLP_H / 16); t += FB_THREADS / 64) {
            const int m0 = (t / (MLP_H / 16)) * 16, n0 = (t % (MLP_H / 16)) * 16;
            const f32x4 acc = lds_tile(L.db, MLP_H, 1, wt[layer], K, 1, m0, n0, MLP_H, lane);
#pragma unroll
            for (int r = 0; r < 4; ++r) L.d[(m0 + kq + r) * MLP_H + n0 + r16] = acc[r];
        }
        __syncthreads();
    }
}

// Gradient = chunk partials summed in chunk order; with lr > 0 AdamW on the FP32
// master weights (bias-corrected moments, decoupled weight decay on matrices) and
// the BF16 refresh.  Thread 0 also sums the chunks' squared errors into sse_out.
__global__ void mlp_reduce_adamw(const float* __restrict__ part, int nchunk, const float* __restrict__ sse,
                                 float* __restrict__ sse_out, float* __restrict__ w, float* __restrict__ g,
                                 float* __restrict__ m, float* __restrict__ v, uint16_t* __restrict__ wb, float lr,
                                 float wd, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && sse_out) {
        float sq = 0.f;
        for (int c = 0; c < nchunk; ++c) sq += sse[c];
        *sse_out = sq;
    }
    if (i >= N_PARAM) return;
    float gi = 0.f;
    for (int c = 0; c < nchunk; ++c) gi += part[(size_t)c * N_PARAM + i];
    g[i] = gi;
    if (!(lr > 0.f)) return;
    const bool is_bias = (i >= OFF_B1 && i < OFF_W2) || (i >= OFF_B2 && i < OFF_W3) ||
                         (i >= OFF_B3 && i < OFF_W4) || i >= OFF_B4;
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float wi = w[i];
    if (!is_bias) wi -= lr * wd * wi;
    wi -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    wb[i] = f2bf(wi);
}

// Inference: forward of a chunk and the de-standardised output (b4 added).
__global__ void __launch_bounds__(FB_THREADS)
mlp_fused_infer(const float* __restrict__ x, int B, const float* __restrict__ consts,
                const float* __restrict__ w, const uint16_t* __restrict__ wb, float scale, float shift,
                float* __restrict__ out) {
    extern __shared__ __align__(16) char lds[];
    const FusedLds L = fused_layout(lds, false);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int r0 = blockIdx.x * FB_ROWS;
    fused_load(L, wb, w, x, B, r0, consts, consts + MLP_IN, tid);
    __syncthreads();
    fused_forward<false>(L, wid, lane);
    if (tid < FB_ROWS && r0 + tid < B) out[r0 + tid] = (L.o[tid * MLP_OUTP] + L.b[3 * MLP_H]) * scale + shift;
}

}  // namespace lt

struct lt_mlp {
    lt_ctx* ctx = nullptr;
    int cap = 0;                 // batch capacity of the activation buffers
    uint64_t step = 0;
    // host copies of the normalisation and guard
    float mean[lt::MLP_IN], inv_std[lt::MLP_IN], fmin[lt::MLP_IN], fmax[lt::MLP_IN];
    float t_shift = 0.f, t_scale = 1.f, max_abs_delta = 1e30f;
    // device
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    uint16_t* wb = nullptr;
    float* consts = nullptr;     // mean[34], inv_std[34], fmin[34], fmax[34]
    float* part = nullptr;       // per-chunk gradient partials and squared errors for `cap` rows
};

namespace lt {

static inline unsigned nb(size_t n) { return (unsigned)((n + 255) / 256); }

static void gemm(int M, int N, int K, const uint16_t* A, int lda, int ta, const uint16_t* B, int ldb, int tb,
                 float* C, int ldc, hipStream_t s, lt_ctx* ctx = nullptr) {
    ProfScope _p(ctx, s, "mfma_gemm");
    const int tiles = (M / 16) * (N / 16);
    mfma_gemm<<<(tiles + 3) / 4, 256, 0, s>>>(M, N, K, A, lda, ta, B, ldb, tb, C, ldc);
}

static size_t part_floats(int cap) {
    const size_t nchunk = (size_t)(cap + FB_ROWS - 1) / FB_ROWS;
    return nchunk * N_PARAM + nchunk;
}

static lt_status ensure_cap(lt_mlp* p, int B) {
    if (B <= p->cap) return LT_OK;
    if (p->part) (void)hipFree(p->part), p->part = nullptr;
    const int cap = (B + 255) & ~255;
    lt_status st = device_alloc((void**)&p->part, part_floats(cap) * sizeof(float), "hipMalloc(mlp partials)");
    if (!st) p->cap = cap;
    return st;
}

// Dynamic LDS limits of the fused kernels (above the 64 KiB default), set once.
static void fused_attributes() {
    static std::once_flag once;
    std::call_once(once, [] {
        (void)hipFuncSetAttribute((const void*)mlp_fused_fwd_bwd, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)fused_lds_bytes(true));
        (void)hipFuncSetAttribute((const void*)mlp_fused_infer, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)fused_lds_bytes(false));
    });
}

static lt_status upload_consts(lt_mlp* p) {
    float h[4 * MLP_IN];
    memcpy(h, p->mean, sizeof(p->mean));
    memcpy(h + MLP_IN, p->inv_std, sizeof(p->inv_std));
    memcpy(h + 2 * MLP_IN, p->fmin, sizeof(p->fmin));
    memcpy(h + 3 * MLP_IN, p->fmax, sizeof(p->fmax));
    return hip_check(hipMemcpy(p->consts, h, sizeof(h), hipMemcpyHostToDevice), "copy mlp constants");
}

}  // namespace lt

using namespace lt;

extern "C" {

lt_status lt_mlp_create(lt_ctx* ctx, uint64_t seed, lt_mlp** out) {
    lt::CallScope call_scope_("lt_mlp_create");
    if (!ctx || !out) return set_error(LT_E_ARG, "ctx or out is NULL");
    *out = nullptr;
    lt_status st = hip_check(hipSetDevice(ctx->device), "hipSetDevice");
    if (st) return st;
    lt_mlp* p = new (std::nothrow) lt_mlp();
    if (!p) return set_error(LT_E_ALLOC, "host allocation failed");
    p->ctx = ctx;
    for (int k = 0; k < MLP_IN; ++k) {
        p->mean[k] = 0.f;
        p->inv_std[k] = 1.f;
        p->fmin[k] = -1e30f;
        p->fmax[k] = 1e30f;
    }
    const size_t pb = N_PARAM * sizeof(float);
    if ((st = device_alloc((void**)&p->w, 4 * pb, "hipMalloc(mlp params)")) ||
        (st = device_alloc((void**)&p->wb, N_PARAM * sizeof(uint16_t), "hipMalloc(mlp bf16)")) ||
        (st = device_alloc((void**)&p->consts, 4 * MLP_IN * sizeof(float), "hipMalloc(mlp consts)"))) {
        lt_mlp_destroy(p);
        return st;
    }
    p->g = p->w + N_PARAM;
    p->m = p->g + N_PARAM;
    p->v = p->m + N_PARAM;
    // He-uniform initialisation of the used weights (fixed seed); zero biases and pads
    std::vector<float> h(4 * (size_t)N_PARAM, 0.f);
    std::mt19937_64 rng(seed);
    auto init = [&](int off, int rows, int cols, int fan_in, int used_rows, int used_cols) {
        const float lim = sqrtf(6.f / (float)fan_in);
        std::uniform_real_distribution<float> u(-lim, lim);
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < cols; ++c)
                h[off + r * cols + c] = (r < used_rows && c < used_cols) ? u(rng) : 0.f;
    };
    init(OFF_W1, MLP_H, MLP_INP, MLP_IN, MLP_H, MLP_IN);
    init(OFF_W2, MLP_H, MLP_H, MLP_H, MLP_H, MLP_H);
    init(OFF_W3, MLP_H, MLP_H, MLP_H, MLP_H, MLP_H);
    init(OFF_W4, MLP_OUTP, MLP_H, MLP_H, 1, MLP_H);
    if ((st = hip_check(hipMemcpy(p->w, h.data(), 4 * pb, hipMemcpyHostToDevice), "copy mlp params")) ||
        (st = upload_consts(p))) {
        lt_mlp_destroy(p);
        return st;
    }
    mlp_to_bf16<<<nb(N_PARAM), 256>>>(p->w, p->wb, N_PARAM);
    if ((st = hip_check(hipDeviceSynchronize(), "mlp init"))) {
        lt_mlp_destroy(p);
        return st;
    }
    *out = p;
    return LT_OK;
}

lt_status lt_mlp_destroy(lt_mlp* p) {
    lt::CallScope call_scope_("lt_mlp_destroy");
    if (!p) return LT_OK;
    (void)hipSetDevice(p->ctx->device);
    (void)hipDeviceSynchronize();
    if (p->w) (void)hipFree(p->w);
    if (p->wb) (void)hipFree(p->wb);
    if (p->consts) (void)hipFree(p->consts);
    if (p->part) (void)hipFree(p->part);
    delete p;
    return LT_OK;
}

lt_status lt_mlp_set_normalization(lt_mlp* p, const float* mean, const float* stdev, float target_shift,
                                   float target_scale) {
    lt::CallScope call_scope_("lt_mlp_set_normalization");
    if (!p || !mean || !stdev) return set_error(LT_E_ARG, "NULL argument");
    if (!(target_scale > 0.f)) return set_error(LT_E_ARG, "target_scale must be positive");
    for (int k = 0; k < MLP_IN; ++k) {
        p->mean[k] = mean[k];
        p->inv_std[k] = stdev[k] > 0.f ? 1.f / stdev[k] : 1.f;
    }
    p->t_shift = target_shift;
    p->t_scale = target_scale;
    return upload_consts(p);
}

lt_status lt_mlp_set_guard(lt_mlp* p, const float* fmin, const float* fmax, float max_abs_delta) {
    lt::CallScope call_scope_("lt_mlp_set_guard");
    if (!p || !fmin || !fmax) return set_error(LT_E_ARG, "NULL argument");
    memcpy(p->fmin, fmin, sizeof(p->fmin));
    memcpy(p->fmax, fmax, sizeof(p->fmax));
    p->max_abs_delta = max_abs_delta;
    return upload_consts(p);
}

lt_status lt_mlp_train_step(lt_mlp* p, const float* x, const float* y, int B, float lr, float weight_decay,
                            float* loss_out, void* stream) {
    lt::CallScope call_scope_("lt_mlp_train_step");
    if (!p || !x || !y) return set_error(LT_E_ARG, "NULL argument");
    if (B <= 0 || B % 16) return set_error(LT_E_ARG, "batch size must be a positive multiple of 16");
    lt_status st = hip_check(hipSetDevice(p->ctx->device), "hipSetDevice");
    if (st || (st = ensure_cap(p, B))) return st;
    fused_attributes();
    hipStream_t s = (hipStream_t)stream;
    const int nchunk = (B + FB_ROWS - 1) / FB_ROWS;
    float* sse = p->part + (size_t)nchunk * N_PARAM;
    {
        ProfScope _p(p->ctx, s, "mlp_fused_fwd_bwd");
        mlp_fused_fwd_bwd<<<nchunk, FB_THREADS, fused_lds_bytes(true), s>>>(x, y, B, p->consts, p->w, p->wb, p->part,
                                                                          sse);
    }
    float c1 = 1.f, c2 = 1.f;
    const float b1 = 0.9f, b2 = 0.999f;
    if (lr > 0.f) {
        p->step += 1;
        c1 = 1.f - powf(b1, (float)p->step);
        c2 = 1.f - powf(b2, (float)p->step);
    }
    {
        ProfScope _p(p->ctx, s, "mlp_reduce_adamw");
        mlp_reduce_adamw<<<nb(N_PARAM), 256, 0, s>>>(p->part, nchunk, sse, loss_out, p->w, p->g, p->m, p->v, p->wb,
                                                     lr, weight_decay, b1, b2, 1e-8f, c1, c2);
    }
    return hip_check(hipGetLastError(), "mlp train step");
}

lt_status lt_mlp_infer(lt_mlp* p, const float* x, int B, float* delta, void* stream) {
    lt::CallScope call_scope_("lt_mlp_infer");
    if (!p || (B > 0 && (!x || !delta))) return set_error(LT_E_ARG, "NULL argument");
    if (B <= 0) return LT_OK;
    lt_status st = hip_check(hipSetDevice(p->ctx->device), "hipSetDevice");
    if (st) return st;
    fused_attributes();
    hipStream_t s = (hipStream_t)stream;
    {
        ProfScope _p(p->ctx, s, "mlp_fused_infer");
        mlp_fused_infer<<<(B + FB_ROWS - 1) / FB_ROWS, FB_THREADS, fused_lds_bytes(false), s>>>(
            x, B, p->consts, p->w, p->wb, p->t_scale, p->t_shift, delta);
    }
    return hip_check(hipGetLastError(), "mlp infer");
}

lt_status lt_mlp_features(lt_ctx* ctx, const float* hist32, const uint64_t* volume, const float* mean_lt,
                          uint32_t n, float* x, void* stream) {
    lt::CallScope call_scope_("lt_mlp_features");
    if (!ctx || (n > 0 && (!hist32 || !volume || !mean_lt || !x))) return set_error(LT_E_ARG, "NULL argument");
    if (n == 0) return LT_OK;
    lt_status st = hip_check(hipSetDevice(ctx->device), "hipSetDevice");
    if (st) return st;
    mlp_features<<<nb(n), 256, 0, (hipStream_t)stream>>>(hist32, volume, mean_lt, n, x);
    return hip_check(hipGetLastError(), "mlp features");
}

lt_status lt_mlp_correct(lt_mlp* p, const float* x, const float* s_lt, int n, float* delta_scratch,
                         float* s_corr, uint32_t* n_fallback, void* stream) {
    lt::CallScope call_scope_("lt_mlp_correct");
    if (!p || (n > 0 && (!x || !s_lt || !delta_scratch || !s_corr || !n_fallback)))
        return set_error(LT_E_ARG, "NULL argument");
    if (n <= 0) return LT_OK;
    lt_status st = lt_mlp_infer(p, x, n, delta_scratch, stream);
    if (st) return st;
    mlp_guard<<<nb(n), 256, 0, (hipStream_t)stream>>>(x, s_lt, delta_scratch, n, p->consts + 2 * MLP_IN,
                                                       p->consts + 3 * MLP_IN, p->max_abs_delta,
                                                       s_corr, n_fallback);
    return hip_check(hipGetLastError(), "mlp guard");
}

// Parameters (FP32 master weights, AdamW moments, step) and the normalisation /
// guard constants, as one host blob: N_PARAM * 3 floats, then 4 * 34 + 3 floats,
// then the step as two 32-bit words.
size_t lt_mlp_state_size(void) { return (3 * (size_t)N_PARAM + 4 * MLP_IN + 3 + 2) * sizeof(float); }

lt_status lt_mlp_get_state(lt_mlp* p, void* blob, size_t bytes) {
    lt::CallScope call_scope_("lt_mlp_get_state");
    if (!p || !blob || bytes < lt_mlp_state_size()) return set_error(LT_E_WORKSPACE, "state buffer too small");
    float* f = (float*)blob;
    lt_status st = hip_check(hipSetDevice(p->ctx->device), "hipSetDevice");
    if (st) return st;
    if ((st = hip_check(hipDeviceSynchronize(), "sync"))) return st;
    if ((st = hip_check(hipMemcpy(f, p->w, N_PARAM * 4, hipMemcpyDeviceToHost), "copy w")) ||
        (st = hip_check(hipMemcpy(f + N_PARAM, p->m, 2 * (size_t)N_PARAM * 4, hipMemcpyDeviceToHost), "copy m v")))
        return st;
    float* c = f + 3 * (size_t)N_PARAM;
    for (int k = 0; k < MLP_IN; ++k) {
        c[k] = p->mean[k];
        c[MLP_IN + k] = p->inv_std[k];
        c[2 * MLP_IN + k] = p->fmin[k];
        c[3 * MLP_IN + k] = p->fmax[k];
    }
    c[4 * MLP_IN] = p->t_shift;
    c[4 * MLP_IN + 1] = p->t_scale;
    c[4 * MLP_IN + 2] = p->max_abs_delta;
    uint32_t* sw = (uint32_t*)(c + 4 * MLP_IN + 3);
    sw[0] = (uint32_t)(p->step & 0xffffffffu);
    sw[1] = (uint32_t)(p->step >> 32);
    return LT_OK;
}

lt_status lt_mlp_set_state(lt_mlp* p, const void* blob, size_t bytes) {
    lt::CallScope call_scope_("lt_mlp_set_state");
    if (!p || !blob || bytes < lt_mlp_state_size()) return set_error(LT_E_WORKSPACE, "state buffer too small");
    const float* f = (const float*)blob;
    lt_status st = hip_check(hipSetDevice(p->ctx->device), "hipSetDevice");
    if (st) return st;
    if ((st = hip_check(hipMemcpy(p->w, f, N_PARAM * 4, hipMemcpyHostToDevice), "copy w")) ||
        (st = hip_check(hipMemcpy(p->m, f + N_PARAM, 2 * (size_t)N_PARAM * 4, hipMemcpyHostToDevice), "copy m v")))
        return st;
    const float* c = f + 3 * (size_t)N_PARAM;
    for (int k = 0; k < MLP_IN; ++k) {
        p->mean[k] = c[k];
        p->inv_std[k] = c[MLP_IN + k];
        p->fmin[k] = c[2 * MLP_IN + k];
        p->fmax[k] = c[3 * MLP_IN + k];
    }
    p->t_shift = c[4 * MLP_IN];
    p->t_scale = c[4 * MLP_IN + 1];
    p->max_abs_delta = c[4 * MLP_IN + 2];
    const uint32_t* sw = (const uint32_t*)(c + 4 * MLP_IN + 3);
    p->step = (uint64_t)sw[0] | ((uint64_t)sw[1] << 32);
    if ((st = upload_consts(p))) return st;
    mlp_to_bf16<<<nb(N_PARAM), 256>>>(p->w, p->wb, N_PARAM);
    return hip_check(hipDeviceSynchronize(), "mlp state");
}

lt_status lt_bf16_gemm(int M, int N, int K, const uint16_t* A, int lda, int trans_a, const uint16_t* B,
                       int ldb, int trans_b, float* C, int ldc, void* stream) {
    lt::CallScope call_scope_("lt_bf16_gemm");
    if (M < 0 || N < 0 || K < 0 || M % 16 || N % 16 || K % 16)
        return set_error(LT_E_SHAPE, "M, N and K must be non-negative multiples of 16");
    if (M == 0 || N == 0) return LT_OK;
    if (!A || !B || !C) return set_error(LT_E_ARG, "NULL matrix");
    gemm(M, N, K, A, lda, trans_a ? 1 : 0, B, ldb, trans_b ? 1 : 0, C, ldc, (hipStream_t)stream);
    return hip_check(hipGetLastError(), "bf16 gemm");
}

// Device pointers to the FP32 master weights and gradients (N_PARAM floats each) and
// the parameter count.
lt_status lt_mlp_buffers(lt_mlp* p, float** weights, float** grads, int* n_param) {
    lt::CallScope call_scope_("lt_mlp_buffers");
    if (!p) return set_error(LT_E_ARG, "mlp is NULL");
    if (weights) *weights = p->w;
    if (grads) *grads = p->g;
    if (n_param) *n_param = N_PARAM;
    return LT_OK;
}

lt_status lt_mlp_read(lt_mlp* p, int which, float* host, size_t n) {
    lt::CallScope call_scope_("lt_mlp_read");
    if (!p || !host) return set_error(LT_E_ARG, "NULL argument");
    if (which < 0 || which > 3) return set_error(LT_E_ARG, "which must be 0..3");
    if (n < (size_t)N_PARAM) return set_error(LT_E_WORKSPACE, "host buffer holds fewer than n_param floats");
    const float* src[4] = {p->w, p->g, p->m, p->v};
    lt_status st = hip_check(hipSetDevice(p->ctx->device), "hipSetDevice");
    if (st || (st = hip_check(hipDeviceSynchronize(), "sync"))) return st;
    return hip_check(hipMemcpy(host, src[which], N_PARAM * sizeof(float), hipMemcpyDeviceToHost), "copy mlp array");
}

}  // extern "C"
