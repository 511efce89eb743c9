// Drives liblt's host code for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host side only (the device code is built as
// usual).  Mode "host" needs no GPU: status strings, argument checks before any
// device use, the mesh cell tables, scratch sizing and the injected allocation
// failure.  Mode "device" also runs, on device 0, every entry-point family on small
// inputs: contexts, the three calls and the fused call in 2D and 3D, the static
// form, anisotropic spacing, mesh measures, filtered roundness and remap, a batch
// with its per-volume status, and the correction network (create, train, infer,
// state round trip).  Prints "lib sanitizer run ok (<mode>)" when done.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../include/lt.h"

#define CHECK(x)                                                                         \
    do {                                                                                 \
        const lt_status s_ = (x);                                                        \
        if (s_ != LT_OK) {                                                               \
            printf("%s:%d %s -> %d (%s)\n", __FILE__, __LINE__, #x, (int)s_, lt_last_error()); \
            return 1;                                                                    \
        }                                                                                \
    } while (0)
#define EXPECT(x, code)                                                                  \
    do {                                                                                 \
        const lt_status s_ = (x);                                                        \
        if (s_ != (code)) {                                                              \
            printf("%s:%d %s -> %d, expected %d\n", __FILE__, __LINE__, #x, (int)s_, (int)(code)); \
            return 1;                                                                    \
        }                                                                                \
    } while (0)

static int host_mode() {
    for (int s = 0; s < 12; ++s)
        if (!lt_status_str((lt_status)s)) return 1;
    if (!strstr(lt_version(), "gfx950")) return 1;
    double cube[256], sq[16];
    CHECK(lt_mesh_table(3, cube));
    CHECK(lt_mesh_table(2, sq));
    EXPECT(lt_mesh_table(4, cube), LT_E_SHAPE);
    const int64_t shape3[3] = {16, 20, 24}, bad[3] = {16, -1, 24}, big[3] = {1025, 8, 8};
    if (lt_pipeline_static_bytes(3, shape3, 10) == 0 || lt_pipeline_static_bytes(3, bad, 10) != 0) return 1;
    char fake[64] = {0};
    lt_ctx* ctx = (lt_ctx*)fake;                 // never dereferenced on these paths
    int32_t* p = (int32_t*)fake;
    EXPECT(lt_edt(ctx, p, (lt_dtype)9, 3, shape3, p, nullptr), LT_E_DTYPE);
    EXPECT(lt_edt(ctx, p, LT_U16, 4, shape3, p, nullptr), LT_E_SHAPE);
    EXPECT(lt_edt(ctx, p, LT_U16, 3, bad, p, nullptr), LT_E_SHAPE);
    EXPECT(lt_edt(ctx, p, LT_U16, 3, big, p, nullptr), LT_E_SHAPE);
    EXPECT(lt_edt(nullptr, p, LT_U16, 3, shape3, p, nullptr), LT_E_ARG);
    EXPECT(lt_filtered_roundness(ctx, p, LT_U16, 3, shape3, p, p, 5, 17, (float*)p, nullptr), LT_E_ARG);
    EXPECT(lt_remap_roundness(ctx, nullptr, 4, 0.5f, (float*)p, nullptr), LT_E_ARG);
    EXPECT(lt_closed_forms(nullptr, nullptr, nullptr, nullptr, nullptr, 4, 3, nullptr, nullptr, nullptr, nullptr,
                           nullptr), LT_E_ARG);
    setenv("LT_FAULT_INJECT", "alloc", 1);
    lt_ctx* c = (lt_ctx*)fake;
    EXPECT(lt_ctx_create(&c, 0), LT_E_ALLOC);
    if (c) return 1;
    unsetenv("LT_FAULT_INJECT");
    return 0;
}

template <typename T>
static T* dalloc(size_t n) {
    void* p = nullptr;
    if (hipMalloc(&p, n * sizeof(T) + 16) != hipSuccess) return nullptr;
    (void)hipMemset(p, 0, n * sizeof(T) + 16);
    return (T*)p;
}

struct Outs {
    std::vector<void*> owned;
    lt_measures m{};
    explicit Outs(uint32_t n) {
        m.volume = dalloc<uint64_t>(n);
        m.shell_count = dalloc<uint64_t>(n);
        m.max_lt_sq = dalloc<int32_t>(n);
        m.mean_lt = dalloc<float>(n);
        m.shell_mean_lt = dalloc<float>(n);
        m.sphericity = dalloc<float>(n);
        m.roundness = dalloc<float>(n);
        m.hist32 = dalloc<float>((size_t)n * 32);
        owned = {m.volume, m.shell_count, m.max_lt_sq, m.mean_lt, m.shell_mean_lt, m.sphericity, m.roundness,
                 m.hist32};
    }
    ~Outs() {
        for (void* p : owned) (void)hipFree(p);
    }
};

static int device_mode() {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
        printf("no device\n");
        return 1;
    }
    lt_ctx* ctx = nullptr;
    CHECK(lt_ctx_create(&ctx, 0));
    const uint32_t L = 6;
    // a 3D and a 2D image of blocky labels with background
    for (int nd = 2; nd <= 3; ++nd) {
        const int64_t shape[3] = {nd == 3 ? 24 : 70, nd == 3 ? 33 : 90, nd == 3 ? 70 : 1};
        const size_t n = nd == 3 ? (size_t)24 * 33 * 70 : (size_t)70 * 90;
        std::vector<uint16_t> h(n);
        for (size_t i = 0; i < n; ++i) h[i] = (uint16_t)(((i / 7) + (i / 500)) % L);
        uint16_t* lab = dalloc<uint16_t>(n);
        int32_t* d = dalloc<int32_t>(n);
        int32_t* t = dalloc<int32_t>(n);
        if (!lab || !d || !t) return 1;
        (void)hipMemcpy(lab, h.data(), n * 2, hipMemcpyHostToDevice);
        {
            Outs o(L);
            CHECK(lt_edt(ctx, lab, LT_U16, nd, shape, d, nullptr));
            CHECK(lt_thickness(ctx, lab, LT_U16, nd, shape, d, L - 1, t, nullptr));
            CHECK(lt_object_measures(ctx, lab, LT_U16, nd, shape, t, L - 1, &o.m, nullptr));
            CHECK(lt_pipeline(ctx, lab, LT_U16, nd, shape, L - 1, d, t, &o.m, nullptr));
            CHECK(lt_pipeline_static(ctx, lab, LT_U16, nd, shape, L - 1, d, t, &o.m, nullptr));
            const int32_t w3[3] = {4, 1, 2}, w2[2] = {1, 9};
            CHECK(lt_pipeline_aniso(ctx, lab, LT_U16, nd, shape, nd == 3 ? w3 : w2, L - 1, d, t, &o.m, nullptr));
            CHECK(lt_mesh_measures(ctx, lab, LT_U16, nd, shape, L - 1, o.m.volume, o.m.mean_lt, o.m.sphericity,
                                   nullptr));
            CHECK(lt_pipeline(ctx, lab, LT_U16, nd, shape, L - 1, d, t, &o.m, nullptr));
            CHECK(lt_filtered_roundness(ctx, lab, LT_U16, nd, shape, d, t, L - 1, 3, o.m.roundness, nullptr));
            CHECK(lt_remap_roundness(ctx, o.m.roundness, L, __builtin_nanf(""), o.m.roundness, nullptr));
            CHECK(lt_sync_status(ctx, nullptr));
            lt_volume v{};
            v.labels = lab;
            v.ndim = nd;
            for (int a = 0; a < nd; ++a) v.shape[a] = shape[a];
            v.max_label = L - 1;
            v.dist_sq = d;
            v.lt_sq = t;
            v.measures = o.m;
            lt_volume vols[2] = {v, v};
            lt_batch* b = nullptr;
            CHECK(lt_batch_create(ctx, vols, 1, LT_U16, &b));
            CHECK(lt_batch_run(b, nullptr));
            int32_t st[1] = {-1};
            CHECK(lt_batch_status(b, nullptr, st));
            if (st[0] != 0) return 1;
            CHECK(lt_batch_destroy(b));
            (void)vols[1];
        }
        (void)hipFree(lab);
        (void)hipFree(d);
        (void)hipFree(t);
    }
    // correction network
    lt_mlp* net = nullptr;
    CHECK(lt_mlp_create(ctx, 7, &net));
    const int B = 64;
    float* x = dalloc<float>((size_t)B * 34);
    float* y = dalloc<float>(B);
    float* delta = dalloc<float>(B);
    std::vector<float> hx((size_t)B * 34), hy(B);
    for (int i = 0; i < B * 34; ++i) hx[i] = (float)((i * 37) % 101) / 101.0f;
    for (int i = 0; i < B; ++i) hy[i] = (float)(i % 7) / 7.0f;
    (void)hipMemcpy(x, hx.data(), hx.size() * 4, hipMemcpyHostToDevice);
    (void)hipMemcpy(y, hy.data(), hy.size() * 4, hipMemcpyHostToDevice);
    for (int it = 0; it < 3; ++it) CHECK(lt_mlp_train_step(net, x, y, B, 1e-3f, 1e-4f, nullptr, nullptr));
    CHECK(lt_mlp_infer(net, x, B, delta, nullptr));
    std::vector<unsigned char> blob(lt_mlp_state_size());
    CHECK(lt_mlp_get_state(net, blob.data(), blob.size()));
    CHECK(lt_mlp_set_state(net, blob.data(), blob.size()));
    EXPECT(lt_mlp_set_state(net, blob.data(), blob.size() - 1), LT_E_WORKSPACE);
    (void)hipDeviceSynchronize();
    CHECK(lt_mlp_destroy(net));
    (void)hipFree(x);
    (void)hipFree(y);
    (void)hipFree(delta);
    CHECK(lt_ctx_destroy(ctx));
    return 0;
}

int main(int argc, char** argv) {
    const bool dev = argc > 1 && strcmp(argv[1], "device") == 0;
    if (host_mode()) return 1;
    if (dev && device_mode()) return 1;
    printf("lib sanitizer run ok (%s)\n", dev ? "device" : "host");
    return 0;
}
