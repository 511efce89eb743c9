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
// Every matrix product goes through mfma_gemm (one wave per 16x16 output tile,
// v_mfma_f32_16x16x16_bf16, K stepped by 16).  Weight gradients are full reductions
// over the batch inside one GEMM and bias gradients are fixed-order column sums, so
// a training step is deterministic.  Master weights and AdamW moments are FP32; the
// BF16 copies used by the products are refreshed after every update.
#include <math.h>
#include <stdio.h>
#include <string.h>

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

// x (B x 34 FP32 features) -> standardised BF16 rows of 48 (zero pad); rows
// B .. Bp-1 (padding up to a multiple of 16) are zero.
__global__ void mlp_prep_input(const float* __restrict__ x, int B, int Bp, const float* __restrict__ mean,
                               const float* __restrict__ inv_std, uint16_t* __restrict__ xb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Bp * MLP_INP) return;
    const int r = i / MLP_INP, c = i % MLP_INP;
    float v = 0.f;
    if (c < MLP_IN && r < B) {
        v = (x[(size_t)r * MLP_IN + c] - mean[c]) * inv_std[c];
        if (!isfinite(v)) v = 0.f;
    }
    xb[i] = f2bf(v);
}

// z += bias (in place, kept for the backward pass); h = bf16(silu(z)).
__global__ void mlp_bias_silu(float* __restrict__ z, const float* __restrict__ bias, int B,
                              uint16_t* __restrict__ h) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * MLP_H) return;
    const float v = z[i] + bias[i % MLP_H];
    z[i] = v;
    h[i] = f2bf(v / (1.f + expf(-v)));
}

// prediction p = o[:, 0] + b4; d o = 2 (p - y) / B in column 0 (BF16), loss terms.
__global__ void mlp_loss_grad(const float* __restrict__ o, const float* __restrict__ b4,
                              const float* __restrict__ y, int B, uint16_t* __restrict__ dob,
                              float* __restrict__ dcol0, float* __restrict__ sq) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= B) return;
    const float p = o[(size_t)r * MLP_OUTP] + b4[0];
    const float d = 2.f * (p - y[r]) / (float)B;
    for (int c = 0; c < MLP_OUTP; ++c) dob[(size_t)r * MLP_OUTP + c] = c == 0 ? f2bf(d) : (uint16_t)0;
    dcol0[r] = d;
    sq[r] = (p - y[r]) * (p - y[r]);
}

// dz = dh * silu'(z) -> BF16.
__global__ void mlp_silu_back(const float* __restrict__ dh, const float* __restrict__ z, int B,
                              uint16_t* __restrict__ dzb, float* __restrict__ dz) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * MLP_H) return;
    const float v = z[i];
    const float s = 1.f / (1.f + expf(-v));
    const float g = dh[i] * s * (1.f + v * (1.f - s));
    dz[i] = g;
    dzb[i] = f2bf(g);
}

// out[c] = sum over rows r of m[r * ld + c] in row order (one thread per column).
__global__ void mlp_colsum(const float* __restrict__ m, int rows, int cols, int ld, float* __restrict__ out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int r = 0; r < rows; ++r) s += m[(size_t)r * ld + c];
    out[c] = s;
}

// AdamW on the FP32 master weights (bias-corrected moments, decoupled weight
// decay on matrices only), then refresh the BF16 copy.
__global__ void mlp_adamw(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                          float* __restrict__ v, uint16_t* __restrict__ wb, int n, float lr, float wd,
                          float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool is_bias = (i >= OFF_B1 && i < OFF_W2) || (i >= OFF_B2 && i < OFF_W3) ||
                         (i >= OFF_B3 && i < OFF_W4) || i >= OFF_B4;
    const float gi = g[i];
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

__global__ void mlp_to_bf16(const float* __restrict__ w, uint16_t* __restrict__ wb, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = f2bf(w[i]);
}

__global__ void mlp_output(const float* __restrict__ o, const float* __restrict__ b4, int B, float scale,
                           float shift, float* __restrict__ out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < B) out[r] = (o[(size_t)r * MLP_OUTP] + b4[0]) * scale + shift;
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
    char* act = nullptr;         // activations for `cap` rows
};

namespace lt {

struct Act {
    uint16_t *xb, *h1, *h2, *h3, *dob, *dz3b, *dz2b, *dz1b;
    float *z1, *z2, *z3, *o, *dh, *dz, *dcol0, *sq, *pred;
};

static size_t act_bytes(int cap) {
    const size_t c = (size_t)cap;
    return c * (MLP_INP + 3 * MLP_H + MLP_OUTP + 3 * MLP_H) * 2 +
           c * (3 * MLP_H + MLP_OUTP + 2 * MLP_H + 3) * 4 + 32 * 256;   // + per-array alignment slack
}

static Act act_layout(char* base, int cap) {
    Act a;
    size_t at = 0;
    auto take = [&](size_t bytes) {
        char* p = base + at;
        at += (bytes + 255) & ~size_t(255);
        return p;
    };
    const size_t c = (size_t)cap;
    a.xb = (uint16_t*)take(c * MLP_INP * 2);
    a.h1 = (uint16_t*)take(c * MLP_H * 2);
    a.h2 = (uint16_t*)take(c * MLP_H * 2);
    a.h3 = (uint16_t*)take(c * MLP_H * 2);
    a.dob = (uint16_t*)take(c * MLP_OUTP * 2);
    a.dz3b = (uint16_t*)take(c * MLP_H * 2);
    a.dz2b = (uint16_t*)take(c * MLP_H * 2);
    a.dz1b = (uint16_t*)take(c * MLP_H * 2);
    a.z1 = (float*)take(c * MLP_H * 4);
    a.z2 = (float*)take(c * MLP_H * 4);
    a.z3 = (float*)take(c * MLP_H * 4);
    a.o = (float*)take(c * MLP_OUTP * 4);
    a.dh = (float*)take(c * MLP_H * 4);
    a.dz = (float*)take(c * MLP_H * 4);
    a.dcol0 = (float*)take(c * 4);
    a.sq = (float*)take(c * 4);
    a.pred = (float*)take(c * 4);
    return a;
}

static inline unsigned nb(size_t n) { return (unsigned)((n + 255) / 256); }

static void gemm(int M, int N, int K, const uint16_t* A, int lda, int ta, const uint16_t* B, int ldb, int tb,
                 float* C, int ldc, hipStream_t s, lt_ctx* ctx = nullptr) {
    ProfScope _p(ctx, s, "mfma_gemm");
    const int tiles = (M / 16) * (N / 16);
    mfma_gemm<<<(tiles + 3) / 4, 256, 0, s>>>(M, N, K, A, lda, ta, B, ldb, tb, C, ldc);
}

static lt_status ensure_cap(lt_mlp* p, int B) {
    if (B <= p->cap) return LT_OK;
    if (p->act) (void)hipFree(p->act), p->act = nullptr;
    const int cap = (B + 255) & ~255;
    lt_status st = device_alloc((void**)&p->act, act_bytes(cap), "hipMalloc(mlp activations)");
    if (!st) p->cap = cap;
    return st;
}

static lt_status upload_consts(lt_mlp* p) {
    float h[4 * MLP_IN];
    memcpy(h, p->mean, sizeof(p->mean));
    memcpy(h + MLP_IN, p->inv_std, sizeof(p->inv_std));
    memcpy(h + 2 * MLP_IN, p->fmin, sizeof(p->fmin));
    memcpy(h + 3 * MLP_IN, p->fmax, sizeof(p->fmax));
    return hip_check(hipMemcpy(p->consts, h, sizeof(h), hipMemcpyHostToDevice), "copy mlp constants");
}

// Forward pass of the B rows of x (B x 34 FP32), computed on Bp >= B rows (a
// multiple of 16 within capacity; the extra rows are zero inputs).
static void forward(lt_mlp* p, const float* x, int Bvalid, int B, const Act& a, hipStream_t s) {
    const float* mean = p->consts;
    const float* inv_std = p->consts + MLP_IN;
    mlp_prep_input<<<nb((size_t)B * MLP_INP), 256, 0, s>>>(x, Bvalid, B, mean, inv_std, a.xb);
    gemm(B, MLP_H, MLP_INP, a.xb, MLP_INP, 0, p->wb + OFF_W1, MLP_INP, 1, a.z1, MLP_H, s, p->ctx);
    mlp_bias_silu<<<nb((size_t)B * MLP_H), 256, 0, s>>>(a.z1, p->w + OFF_B1, B, a.h1);
    gemm(B, MLP_H, MLP_H, a.h1, MLP_H, 0, p->wb + OFF_W2, MLP_H, 1, a.z2, MLP_H, s, p->ctx);
    mlp_bias_silu<<<nb((size_t)B * MLP_H), 256, 0, s>>>(a.z2, p->w + OFF_B2, B, a.h2);
    gemm(B, MLP_H, MLP_H, a.h2, MLP_H, 0, p->wb + OFF_W3, MLP_H, 1, a.z3, MLP_H, s, p->ctx);
    mlp_bias_silu<<<nb((size_t)B * MLP_H), 256, 0, s>>>(a.z3, p->w + OFF_B3, B, a.h3);
    gemm(B, MLP_OUTP, MLP_H, a.h3, MLP_H, 0, p->wb + OFF_W4, MLP_H, 1, a.o, MLP_OUTP, s, p->ctx);
}

}  // namespace lt

using namespace lt;

extern "C" {

lt_status lt_mlp_create(lt_ctx* ctx, uint64_t seed, lt_mlp** out) {
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
    if (!p) return LT_OK;
    (void)hipSetDevice(p->ctx->device);
    (void)hipDeviceSynchronize();
    if (p->w) (void)hipFree(p->w);
    if (p->wb) (void)hipFree(p->wb);
    if (p->consts) (void)hipFree(p->consts);
    if (p->act) (void)hipFree(p->act);
    delete p;
    return LT_OK;
}

lt_status lt_mlp_set_normalization(lt_mlp* p, const float* mean, const float* stdev, float target_shift,
                                   float target_scale) {
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
    if (!p || !fmin || !fmax) return set_error(LT_E_ARG, "NULL argument");
    memcpy(p->fmin, fmin, sizeof(p->fmin));
    memcpy(p->fmax, fmax, sizeof(p->fmax));
    p->max_abs_delta = max_abs_delta;
    return upload_consts(p);
}

lt_status lt_mlp_train_step(lt_mlp* p, const float* x, const float* y, int B, float lr, float weight_decay,
                            float* loss_out, void* stream) {
    if (!p || !x || !y) return set_error(LT_E_ARG, "NULL argument");
    if (B <= 0 || B % 16) return set_error(LT_E_ARG, "batch size must be a positive multiple of 16");
    lt_status st = hip_check(hipSetDevice(p->ctx->device), "hipSetDevice");
    if (st || (st = ensure_cap(p, B))) return st;
    hipStream_t s = (hipStream_t)stream;
    const Act a = act_layout(p->act, p->cap);
    forward(p, x, B, B, a, s);
    mlp_loss_grad<<<nb(B), 256, 0, s>>>(a.o, p->w + OFF_B4, y, B, a.dob, a.dcol0, a.sq);
    float* g = p->g;
    mlp_colsum<<<1, 64, 0, s>>>(a.dcol0, B, 1, 1, g + OFF_B4);                          // db4
    gemm(MLP_OUTP, MLP_H, B, a.dob, MLP_OUTP, 1, a.h3, MLP_H, 0, g + OFF_W4, MLP_H, s, p->ctx);   // dW4
    gemm(B, MLP_H, MLP_OUTP, a.dob, MLP_OUTP, 0, p->wb + OFF_W4, MLP_H, 0, a.dh, MLP_H, s, p->ctx);  // dH3
    mlp_silu_back<<<nb((size_t)B * MLP_H), 256, 0, s>>>(a.dh, a.z3, B, a.dz3b, a.dz);
    mlp_colsum<<<1, 64, 0, s>>>(a.dz, B, MLP_H, MLP_H, g + OFF_B3);
    gemm(MLP_H, MLP_H, B, a.dz3b, MLP_H, 1, a.h2, MLP_H, 0, g + OFF_W3, MLP_H, s, p->ctx);        // dW3
    gemm(B, MLP_H, MLP_H, a.dz3b, MLP_H, 0, p->wb + OFF_W3, MLP_H, 0, a.dh, MLP_H, s, p->ctx);   // dH2
    mlp_silu_back<<<nb((size_t)B * MLP_H), 256, 0, s>>>(a.dh, a.z2, B, a.dz2b, a.dz);
    mlp_colsum<<<1, 64, 0, s>>>(a.dz, B, MLP_H, MLP_H, g + OFF_B2);
    gemm(MLP_H, MLP_H, B, a.dz2b, MLP_H, 1, a.h1, MLP_H, 0, g + OFF_W2, MLP_H, s, p->ctx);        // dW2
    gemm(B, MLP_H, MLP_H, a.dz2b, MLP_H, 0, p->wb + OFF_W2, MLP_H, 0, a.dh, MLP_H, s, p->ctx);   // dH1
    mlp_silu_back<<<nb((size_t)B * MLP_H), 256, 0, s>>>(a.dh, a.z1, B, a.dz1b, a.dz);
    mlp_colsum<<<1, 64, 0, s>>>(a.dz, B, MLP_H, MLP_H, g + OFF_B1);
    gemm(MLP_H, MLP_INP, B, a.dz1b, MLP_H, 1, a.xb, MLP_INP, 0, g + OFF_W1, MLP_INP, s, p->ctx);  // dW1
    if (lr > 0.f) {
        p->step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.f - powf(b1, (float)p->step), c2 = 1.f - powf(b2, (float)p->step);
        mlp_adamw<<<nb(N_PARAM), 256, 0, s>>>(p->w, g, p->m, p->v, p->wb, N_PARAM, lr, weight_decay, b1,
                                              b2, 1e-8f, c1, c2);
    }
    if (loss_out) mlp_colsum<<<1, 64, 0, s>>>(a.sq, B, 1, 1, loss_out);                   // sum of squares
    return hip_check(hipGetLastError(), "mlp train step");
}

lt_status lt_mlp_infer(lt_mlp* p, const float* x, int B, float* delta, void* stream) {
    if (!p || (B > 0 && (!x || !delta))) return set_error(LT_E_ARG, "NULL argument");
    if (B <= 0) return LT_OK;
    lt_status st = hip_check(hipSetDevice(p->ctx->device), "hipSetDevice");
    const int Bp = (B + 15) & ~15;
    if (st || (st = ensure_cap(p, Bp))) return st;
    hipStream_t s = (hipStream_t)stream;
    const Act a = act_layout(p->act, p->cap);
    forward(p, x, B, Bp, a, s);
    mlp_output<<<nb(B), 256, 0, s>>>(a.o, p->w + OFF_B4, B, p->t_scale, p->t_shift, delta);
    return hip_check(hipGetLastError(), "mlp infer");
}

lt_status lt_mlp_features(lt_ctx* ctx, const float* hist32, const uint64_t* volume, const float* mean_lt,
                          uint32_t n, float* x, void* stream) {
    if (!ctx || (n > 0 && (!hist32 || !volume || !mean_lt || !x))) return set_error(LT_E_ARG, "NULL argument");
    if (n == 0) return LT_OK;
    lt_status st = hip_check(hipSetDevice(ctx->device), "hipSetDevice");
    if (st) return st;
    mlp_features<<<nb(n), 256, 0, (hipStream_t)stream>>>(hist32, volume, mean_lt, n, x);
    return hip_check(hipGetLastError(), "mlp features");
}

lt_status lt_mlp_correct(lt_mlp* p, const float* x, const float* s_lt, int n, float* delta_scratch,
                         float* s_corr, uint32_t* n_fallback, void* stream) {
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
    if (!p) return set_error(LT_E_ARG, "mlp is NULL");
    if (weights) *weights = p->w;
    if (grads) *grads = p->g;
    if (n_param) *n_param = N_PARAM;
    return LT_OK;
}

lt_status lt_mlp_read(lt_mlp* p, int which, float* host, size_t n) {
    if (!p || !host) return set_error(LT_E_ARG, "NULL argument");
    if (which < 0 || which > 3) return set_error(LT_E_ARG, "which must be 0..3");
    if (n < (size_t)N_PARAM) return set_error(LT_E_WORKSPACE, "host buffer holds fewer than n_param floats");
    const float* src[4] = {p->w, p->g, p->m, p->v};
    lt_status st = hip_check(hipSetDevice(p->ctx->device), "hipSetDevice");
    if (st || (st = hip_check(hipDeviceSynchronize(), "sync"))) return st;
    return hip_check(hipMemcpy(host, src[which], N_PARAM * sizeof(float), hipMemcpyDeviceToHost), "copy mlp array");
}

}  // extern "C"
