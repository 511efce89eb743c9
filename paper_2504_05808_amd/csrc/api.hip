// C-ABI entry points of liblt: context, argument checks, dispatch, error text.
#include <math.h>
#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "lt_internal.h"

namespace lt {

static thread_local char g_err[512] = "";
static thread_local const char* g_call = nullptr;    // the exported call running on this thread

// LT_LOG (environment): unset or 0, silent; 1, one line on stderr per error status (the
// call it came from, the status and its message); 2, also one line per exported call
// that takes a volume (its name, shape, label type and label bound).  Read at every
// use (host work only), so a process may change it between calls.
static int log_level() {
    const char* e = getenv("LT_LOG");
    return e ? atoi(e) : 0;
}

CallScope::CallScope(const char* fn, int ndim, const int64_t* shape, int dtype, long long max_label)
    : prev(g_call) {
    g_call = fn;
    if ((!shape && dtype < 0) || log_level() < 2) return;
    char buf[256];
    int k = snprintf(buf, sizeof(buf), "[lt] %s", fn);
    if (shape && ndim >= 1 && ndim <= 3) {
        k += snprintf(buf + k, sizeof(buf) - k, " shape=");
        for (int i = 0; i < ndim && k < (int)sizeof(buf); ++i)
            k += snprintf(buf + k, sizeof(buf) - k, i ? "x%lld" : "%lld", (long long)shape[i]);
    }
    static const char* const names[] = {"u16", "i32", "u32"};    // LT_U16, LT_I32, LT_U32
    if (dtype >= 0 && k < (int)sizeof(buf))
        k += dtype >= LT_U16 && dtype <= LT_U32 ? snprintf(buf + k, sizeof(buf) - k, " dtype=%s", names[dtype - 1])
                                                : snprintf(buf + k, sizeof(buf) - k, " dtype=%d", dtype);
    if (max_label >= 0 && k < (int)sizeof(buf)) snprintf(buf + k, sizeof(buf) - k, " max_label=%lld", max_label);
    fprintf(stderr, "%s\n", buf);
}

CallScope::~CallScope() { g_call = prev; }

lt_status set_error(lt_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    if (log_level() >= 1) fprintf(stderr, "[lt] %s: %s: %s\n", g_call ? g_call : "liblt", lt_status_str(s), g_err);
    return s;
}

lt_status hip_check(hipError_t e, const char* what) {
    if (e == hipSuccess) return LT_OK;
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return set_error(LT_E_ALLOC, "%s: %s", what, hipGetErrorString(e));
    return set_error(LT_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Allocation fault injection (tests of the failure paths): LT_FAULT_INJECT=alloc makes
// every device allocation of the library fail with LT_E_ALLOC; alloc:N lets N more
// allocations succeed first (counted from when that value was first seen).
static std::mutex g_fault_mu;
static std::string g_fault_seen;
static long g_fault_left = -1;                  // allocations still allowed; -1: no injection

static bool fault_alloc_next(bool consume) {
    std::lock_guard<std::mutex> lock(g_fault_mu);
    const char* e = getenv("LT_FAULT_INJECT");
    const std::string v = e ? e : "";
    if (v != g_fault_seen) {
        g_fault_seen = v;
        g_fault_left = -1;
        if (v == "alloc") g_fault_left = 0;
        else if (v.rfind("alloc:", 0) == 0) g_fault_left = strtol(v.c_str() + 6, nullptr, 10);
    }
    if (g_fault_left < 0) return false;
    if (g_fault_left == 0) return true;
    if (consume) --g_fault_left;
    return false;
}

lt_status device_alloc(void** p, size_t bytes, const char* what) {
    *p = nullptr;
    if (fault_alloc_next(true)) return set_error(LT_E_ALLOC, "%s: injected allocation failure (LT_FAULT_INJECT)", what);
    return hip_check(hipMalloc(p, bytes), what);
}

lt_status ensure_scratch(lt_ctx* ctx, size_t bytes) {
    if (bytes <= ctx->scratch.bytes) return LT_OK;
    if (ctx->scratch.ptr) {
        lt_status st = hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
        if (st) return st;
        (void)hipFree(ctx->scratch.ptr);
        ctx->scratch.ptr = nullptr;
        ctx->scratch.bytes = 0;
    }
    size_t want = bytes + bytes / 8 + (1u << 20);
    void* p = nullptr;
    lt_status st = device_alloc(&p, want, "hipMalloc(scratch)");
    if (st) return st;
    ctx->scratch.ptr = p;
    ctx->scratch.bytes = want;
    return LT_OK;
}

size_t pipeline_measures_offset(const Geom& g, uint32_t max_label) {
    return (thickness_scratch_bytes(g, max_label) + 255) & ~size_t(255);
}

// Fused pipeline scratch: [EDT | thickness + measures] overlapping from offset 0
// (EDT finishes before thickness starts), then the bounding boxes, which the EDT x
// pass writes and the thickness pass reads.
static size_t pipeline_boxes_offset(const Geom& g, uint32_t max_label) {
    size_t b = edt_scratch_bytes(g);
    b = std::max(b, pipeline_measures_offset(g, max_label) + measures_scratch_bytes(max_label));
    return (b + 255) & ~size_t(255);
}

size_t pipeline_scratch_bytes(const Geom& g, uint32_t max_label) {
    const size_t boxes = 6 * ((size_t)max_label + 1) * sizeof(int32_t);
    return pipeline_boxes_offset(g, max_label) + ((boxes + 255) & ~size_t(255));
}

lt_status launch_pipeline(lt_ctx* ctx, const void* labels, lt_dtype dt, const Geom& g, uint32_t max_label,
                          int32_t* dist_sq, int32_t* lt_sq, const lt_measures* out, void* scratch,
                          hipStream_t s, const Spacing* sp) {
    void* mscr = (char*)scratch + pipeline_measures_offset(g, max_label);
    int32_t* bb = (int32_t*)((char*)scratch + pipeline_boxes_offset(g, max_label));
    const BoxTarget box{bb, max_label + 1, max_label};
    lt_status st = LT_OK;
    if (g.n > 0 && !(st = launch_init_boxes(ctx, bb, max_label + 1, s)))
        st = launch_edt(ctx, labels, dt, g, dist_sq, scratch, s, &box, sp);
    MeasureSums sums;
    if (!st) st = launch_measures_zero(ctx, max_label, out, mscr, s, &sums);
    if (!st && g.n > 0)
        st = launch_thickness(ctx, labels, dt, g, dist_sq, max_label, lt_sq, scratch, s, &sums, bb, sp);
    if (!st) st = launch_measures_finish(ctx, labels, dt, g, lt_sq, max_label, out, mscr, s, sp ? sp->vsize : 1.0f);
    return st;
}

lt_status geom_from(int ndim, const int64_t* shape, Geom* g) {
    if (!shape) return set_error(LT_E_ARG, "shape is NULL");
    if (ndim != 2 && ndim != 3) return set_error(LT_E_SHAPE, "ndim must be 2 or 3 (got %d)", ndim);
    const int64_t lim = ndim == 3 ? 1024 : 2048;
    for (int i = 0; i < ndim; ++i) {
        if (shape[i] < 0) return set_error(LT_E_SHAPE, "negative extent %lld", (long long)shape[i]);
        if (shape[i] > lim)
            return set_error(LT_E_SHAPE, "extent %lld exceeds %lld", (long long)shape[i], (long long)lim);
    }
    g->ndim = ndim;
    g->nz = ndim == 3 ? (int)shape[0] : 1;
    g->ny = (int)shape[ndim - 2];
    g->nx = (int)shape[ndim - 1];
    g->n = (size_t)g->nz * g->ny * g->nx;
    return LT_OK;
}

// Containment tables for the exact centre prune: for a neighbour offset o and
// squared radius d, T[d] = max{ |q - o|^2 : q in Z^n, |q|^2 < d }.  A ball of
// squared radius d centred at x lies inside the open ball of x + o iff
// D(x + o) > T[d].  By lattice symmetry T depends only on |o|^2.
static void build_prune_tables(int n, std::vector<int32_t>& out) {
    const int dcap = PRUNE_DCAP;
    const int r = 129;                          // r*r > dcap
    const int nk = n;                           // |o|^2 = 1 .. n
    std::vector<int32_t> best((size_t)nk * (dcap + 1), -1);
    const int rz = n == 3 ? r : 0;
    for (int qz = -rz; qz <= rz; ++qz)
        for (int qy = -r; qy <= r; ++qy)
            for (int qx = -r; qx <= r; ++qx) {
                int m = qz * qz + qy * qy + qx * qx;
                if (m > dcap) continue;
                for (int k = 1; k <= nk; ++k) {
                    // o_k = (1, 0, 0), (1, 1, 0), (1, 1, 1) in (x, y, z) order
                    int ox = 1, oy = k >= 2 ? 1 : 0, oz = k >= 3 ? 1 : 0;
                    int dx = qx - ox, dy = qy - oy, dz = qz - oz;
                    int v = dx * dx + dy * dy + dz * dz;
                    int32_t& b = best[(size_t)(k - 1) * (dcap + 1) + m];
                    if (v > b) b = v;
                }
            }
    out.assign((size_t)nk * (dcap + 1), -1);
    for (int k = 0; k < nk; ++k) {
        int32_t run = -1;                        // max over |q|^2 < d
        for (int d = 0; d <= dcap; ++d) {
            out[(size_t)k * (dcap + 1) + d] = run;
            int32_t b = best[(size_t)k * (dcap + 1) + d];
            if (b > run) run = b;
        }
    }
}

// Weighted containment tables: for the offset classes c (which axes the neighbour
// offset o_c moves along: bit 2 z, bit 1 y, bit 0 x; c = bits - 1) and d <= PRUNE_DCAP,
// T_c[d] = max{ |q - o_c|_w^2 : |q|_w^2 < d } with |q|_w^2 = wz qz^2 + wy qy^2 + wx qx^2.
// A ball of squared radius d centred at x lies in the open ball of x + o (for any o
// of class c: the lattice ball is symmetric under sign flips of each axis) iff
// D(x + o) > T_c[d].  2D: classes over (y, x) only.
static void build_prune_tables_weighted(int ndim, const Spacing& sp, std::vector<int32_t>& out) {
    const int dcap = PRUNE_DCAP;
    const int nc = ndim == 3 ? 7 : 3;
    std::vector<int32_t> best((size_t)nc * (dcap + 1), -1);
    auto reach = [&](int w) {                    // largest r with w r^2 < dcap
        int r = 0;
        while (w * (r + 1) * (r + 1) < dcap) ++r;
        return r;
    };
    const int rz = ndim == 3 ? reach(sp.wz) : 0, ry = reach(sp.wy), rx = reach(sp.wx);
    for (int qz = -rz; qz <= rz; ++qz)
        for (int qy = -ry; qy <= ry; ++qy)
            for (int qx = -rx; qx <= rx; ++qx) {
                const int m = sp.wz * qz * qz + sp.wy * qy * qy + sp.wx * qx * qx;
                if (m >= dcap) continue;
                for (int c = 0; c < nc; ++c) {
                    const int bits = c + 1;
                    const int oz = ndim == 3 ? (bits >> 2) & 1 : 0, oy = (bits >> 1) & 1, ox = bits & 1;
                    const int v = sp.wz * (qz - oz) * (qz - oz) + sp.wy * (qy - oy) * (qy - oy) +
                                  sp.wx * (qx - ox) * (qx - ox);
                    int32_t& b = best[(size_t)c * (dcap + 1) + m];
                    if (v > b) b = v;
                }
            }
    out.assign((size_t)nc * (dcap + 1), -1);
    for (int c = 0; c < nc; ++c) {
        int32_t run = -1;                        // max over |q|_w^2 < d
        for (int d = 0; d <= dcap; ++d) {
            out[(size_t)c * (dcap + 1) + d] = run;
            const int32_t b = best[(size_t)c * (dcap + 1) + d];
            if (b > run) run = b;
        }
    }
}

lt_status prune_tables_weighted(lt_ctx* ctx, int ndim, const Spacing& sp, const int32_t** out) {
    const std::array<int, 4> key{ndim, ndim == 3 ? sp.wz : 1, sp.wy, sp.wx};
    for (const auto& e : ctx->prune_w)
        if (e.first == key) {
            *out = e.second;
            return LT_OK;
        }
    std::vector<int32_t> tab;
    build_prune_tables_weighted(ndim, sp, tab);
    int32_t* d = nullptr;
    const size_t bytes = tab.size() * sizeof(int32_t);
    lt_status st = device_alloc((void**)&d, bytes, "hipMalloc(weighted prune tables)");
    if (st) return st;
    if ((st = hip_check(hipMemcpy(d, tab.data(), bytes, hipMemcpyHostToDevice), "copy weighted prune tables"))) {
        (void)hipFree(d);
        return st;
    }
    ctx->prune_w.push_back({key, d});
    *out = d;
    return LT_OK;
}

// Squared spacings from the caller: ndim integers in 1..LT_MAX_SQ_SPACING along
// (z, y, x) or (y, x).  Every squared distance of the image is at most
// min_a w_a ((n_a + 1) / 2)^2 (the border is that close along each axis); the
// weighted kernels need it below 2^19 in 3D (packed front entries) and 2^24 in 2D.
static lt_status spacing_from(int ndim, const Geom& g, const int32_t* sq, Spacing* sp) {
    if (!sq) return set_error(LT_E_ARG, "sq_spacing is NULL");
    int w[3] = {1, 1, 1};
    for (int i = 0; i < ndim; ++i) {
        if (sq[i] < 1 || sq[i] > LT_MAX_SQ_SPACING)
            return set_error(LT_E_ARG, "squared spacing %d outside 1..%d", (int)sq[i], LT_MAX_SQ_SPACING);
        w[3 - ndim + i] = sq[i];
    }
    sp->wz = w[0];
    sp->wy = w[1];
    sp->wx = w[2];
    sp->vsize = (float)sqrt((double)w[0] * w[1] * w[2]);
    const int n[3] = {g.nz, g.ny, g.nx};
    int64_t bound = INT64_MAX;
    for (int a = 3 - ndim; a < 3; ++a) {
        const int64_t h = (n[a] + 1) / 2;
        bound = std::min(bound, (int64_t)w[a] * h * h);
    }
    const int64_t lim = ndim == 3 ? (int64_t)ZF_D_MASK : (int64_t)1 << 24;
    if (bound > lim)
        return set_error(LT_E_ARG, "squared distances up to %lld exceed %lld for this shape and spacing",
                         (long long)bound, (long long)lim);
    return LT_OK;
}

static std::once_flag g_tab_once;
static std::vector<int32_t> g_tab3, g_tab2;

// Fixed scratch of lt_pipeline_static: one copy per device, held until the process
// ends.  Host code never passes `scratch` itself (in host code the name is a
// host-side stand-in, not a device address): lt_ctx_create looks up each device's
// address once with hipGetSymbolAddress and keeps it in g_static_scratch.
constexpr size_t STATIC_SCRATCH_BYTES = (size_t)LT_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_static_mu;
static void* g_static_scratch[MAX_DEVICES] = {};

// Device address of `scratch` on the current device `device`, looked up once.
static lt_status static_scratch_lookup(int device, void** out) {
    if (device < 0 || device >= MAX_DEVICES) return set_error(LT_E_ARG, "device %d out of range", device);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_scratch[device]) {
        void* ptr = nullptr;
        lt_status st = hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (st) return st;
        if (!ptr) return set_error(LT_E_HIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_static_scratch[device] = ptr;
    }
    *out = g_static_scratch[device];
    return LT_OK;
}

}  // namespace lt

using namespace lt;

extern "C" {

const char* lt_version(void) { return "liblt 0.1 (gfx950)"; }

const char* lt_last_error(void) { return g_err; }

const char* lt_status_str(lt_status s) {
    switch (s) {
        case LT_OK: return "ok";
        case LT_E_ARG: return "invalid argument";
        case LT_E_DTYPE: return "invalid label dtype";
        case LT_E_SHAPE: return "invalid shape";
        case LT_E_ALLOC: return "device allocation failed";
        case LT_E_HIP: return "HIP runtime error";
        case LT_E_LABEL_RANGE: return "label out of range";
        case LT_E_OVERFLOW: return "range overflow";
        case LT_E_WORKSPACE: return "workspace too small";
        case LT_E_NOT_READY: return "not ready";
    }
    return "unknown status";
}

lt_status lt_ctx_create(lt_ctx** out, int device) {
    lt::CallScope call_scope_("lt_ctx_create");
    if (!out) return set_error(LT_E_ARG, "out is NULL");
    *out = nullptr;
    // a context needs device memory: with allocations failing by injection it fails
    // before touching the device
    if (fault_alloc_next(false))
        return set_error(LT_E_ALLOC, "lt_ctx_create: injected allocation failure (LT_FAULT_INJECT)");
    int count = 0;
    lt_status st = hip_check(hipGetDeviceCount(&count), "hipGetDeviceCount");
    if (st) return st;
    if (device < 0 || device >= count)
        return set_error(LT_E_ARG, "device %d not present (%d devices)", device, count);
    st = hip_check(hipSetDevice(device), "hipSetDevice");
    if (st) return st;
    lt_ctx* c = new (std::nothrow) lt_ctx();
    if (!c) return set_error(LT_E_ALLOC, "host allocation failed");
    c->device = device;
    hipDeviceProp_t prop;
    if ((st = hip_check(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties"))) {
        delete c;
        return st;
    }
    c->n_cu = prop.multiProcessorCount;
    c->lds_per_block = prop.sharedMemPerBlock;
    std::call_once(g_tab_once, [] {
        build_prune_tables(3, g_tab3);
        build_prune_tables(2, g_tab2);
    });
    // the 3D tables go to the device interleaved, {T_1[d], T_2[d], T_3[d], 0} per d, so
    // that the prune reads a centre's three thresholds with one 16-byte load
    std::vector<int32_t> tab3i((size_t)4 * (PRUNE_DCAP + 1), 0);
    for (int d = 0; d <= PRUNE_DCAP; ++d)
        for (int k = 0; k < 3; ++k) tab3i[(size_t)4 * d + k] = g_tab3[(size_t)k * (PRUNE_DCAP + 1) + d];
    size_t b3 = tab3i.size() * sizeof(int32_t), b2 = g_tab2.size() * sizeof(int32_t);
    if ((st = device_alloc((void**)&c->d_err, sizeof(uint32_t), "hipMalloc(err)")) ||
        (st = device_alloc((void**)&c->d_prune3, b3, "hipMalloc(tab3)")) ||
        (st = device_alloc((void**)&c->d_prune2, b2, "hipMalloc(tab2)")) ||
        (st = hip_check(hipMemcpy(c->d_prune3, tab3i.data(), b3, hipMemcpyHostToDevice), "copy tab3")) ||
        (st = hip_check(hipMemcpy(c->d_prune2, g_tab2.data(), b2, hipMemcpyHostToDevice), "copy tab2")) ||
        (st = hip_check(hipMemset(c->d_err, 0, sizeof(uint32_t)), "clear err")) ||
        (st = static_scratch_lookup(device, &c->static_scratch))) {
        lt_ctx_destroy(c);
        return st;
    }
    *out = c;
    return LT_OK;
}

lt_status lt_ctx_destroy(lt_ctx* ctx) {
    lt::CallScope call_scope_("lt_ctx_destroy");
    if (!ctx) return LT_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->scratch.ptr) (void)hipFree(ctx->scratch.ptr);
    if (ctx->d_err) (void)hipFree(ctx->d_err);
    if (ctx->d_prune3) (void)hipFree(ctx->d_prune3);
    if (ctx->d_prune2) (void)hipFree(ctx->d_prune2);
    for (auto& e : ctx->prune_w) (void)hipFree(e.second);
    delete ctx;
    return LT_OK;
}

static lt_status common_checks(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim,
                               const int64_t* shape, Geom* g) {
    if (!ctx) return set_error(LT_E_ARG, "ctx is NULL");
    if (dtype != LT_U16 && dtype != LT_I32 && dtype != LT_U32)
        return set_error(LT_E_DTYPE, "unknown label dtype %d", (int)dtype);
    lt_status st = geom_from(ndim, shape, g);
    if (st) return st;
    if (g->n > 0 && !labels) return set_error(LT_E_ARG, "labels is NULL");
    return hip_check(hipSetDevice(ctx->device), "hipSetDevice");
}

lt_status lt_edt(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim, const int64_t* shape,
                 int32_t* dist_sq, void* stream) {
    lt::CallScope call_scope_("lt_edt", ndim, shape, (int)dtype, -1);
    Geom g;
    lt_status st = common_checks(ctx, labels, dtype, ndim, shape, &g);
    if (st) return st;
    if (g.n == 0) return LT_OK;
    if (!dist_sq) return set_error(LT_E_ARG, "dist_sq is NULL");
    if ((st = ensure_scratch(ctx, edt_scratch_bytes(g)))) return st;
    return launch_edt(ctx, labels, dtype, g, dist_sq, ctx->scratch.ptr, (hipStream_t)stream);
}

lt_status lt_thickness(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim,
                       const int64_t* shape, const int32_t* dist_sq, uint32_t max_label,
                       int32_t* lt_sq, void* stream) {
    lt::CallScope call_scope_("lt_thickness", ndim, shape, (int)dtype, (long long)max_label);
    Geom g;
    lt_status st = common_checks(ctx, labels, dtype, ndim, shape, &g);
    if (st) return st;
    if (g.n == 0) return LT_OK;
    if (!dist_sq || !lt_sq) return set_error(LT_E_ARG, "dist_sq or lt_sq is NULL");
    if (max_label > (1u << 28)) return set_error(LT_E_ARG, "max_label %u exceeds 2^28", max_label);
    if ((st = ensure_scratch(ctx, thickness_scratch_bytes(g, max_label)))) return st;
    return launch_thickness(ctx, labels, dtype, g, dist_sq, max_label, lt_sq, ctx->scratch.ptr,
                            (hipStream_t)stream);
}

lt_status lt_object_measures(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim,
                             const int64_t* shape, const int32_t* lt_sq, uint32_t max_label,
                             const lt_measures* out, void* stream) {
    lt::CallScope call_scope_("lt_object_measures", ndim, shape, (int)dtype, (long long)max_label);
    Geom g;
    lt_status st = common_checks(ctx, labels, dtype, ndim, shape, &g);
    if (st) return st;
    if (!out || !out->volume || !out->shell_count || !out->max_lt_sq || !out->mean_lt ||
        !out->shell_mean_lt || !out->sphericity || !out->roundness)
        return set_error(LT_E_ARG, "an output array of lt_measures is NULL");
    if (g.n > 0 && !lt_sq) return set_error(LT_E_ARG, "lt_sq is NULL");
    if (max_label > (1u << 28)) return set_error(LT_E_ARG, "max_label %u exceeds 2^28", max_label);
    if ((st = ensure_scratch(ctx, measures_scratch_bytes(max_label)))) return st;
    return launch_measures(ctx, labels, dtype, g, lt_sq, max_label, out, ctx->scratch.ptr,
                           (hipStream_t)stream);
}

lt_status lt_pipeline(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim, const int64_t* shape,
                      uint32_t max_label, int32_t* dist_sq, int32_t* lt_sq, const lt_measures* out,
                      void* stream) {
    lt::CallScope call_scope_("lt_pipeline", ndim, shape, (int)dtype, (long long)max_label);
    Geom g;
    lt_status st = common_checks(ctx, labels, dtype, ndim, shape, &g);
    if (st) return st;
    if (!out || !out->volume || !out->shell_count || !out->max_lt_sq || !out->mean_lt ||
        !out->shell_mean_lt || !out->sphericity || !out->roundness)
        return set_error(LT_E_ARG, "an output array of lt_measures is NULL");
    if (g.n > 0 && (!dist_sq || !lt_sq)) return set_error(LT_E_ARG, "dist_sq or lt_sq is NULL");
    if (max_label > (1u << 28)) return set_error(LT_E_ARG, "max_label %u exceeds 2^28", max_label);
    if ((st = ensure_scratch(ctx, pipeline_scratch_bytes(g, max_label)))) return st;
    return launch_pipeline(ctx, labels, dtype, g, max_label, dist_sq, lt_sq, out, ctx->scratch.ptr,
                           (hipStream_t)stream);
}

lt_status lt_mesh_measures(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim, const int64_t* shape,
                           uint32_t max_label, uint64_t* volume, float* area, float* sphericity, void* stream) {
    lt::CallScope call_scope_("lt_mesh_measures", ndim, shape, (int)dtype, (long long)max_label);
    Geom g;
    lt_status st = common_checks(ctx, labels, dtype, ndim, shape, &g);
    if (st) return st;
    if (!volume && !area && !sphericity) return set_error(LT_E_ARG, "volume, area and sphericity are all NULL");
    if (max_label > (1u << 28)) return set_error(LT_E_ARG, "max_label %u exceeds 2^28", max_label);
    if ((st = ensure_scratch(ctx, mesh_scratch_bytes(max_label)))) return st;
    return launch_mesh(ctx, labels, dtype, g, max_label, volume, area, sphericity, ctx->scratch.ptr,
                       (hipStream_t)stream);
}

lt_status lt_edt_aniso(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim, const int64_t* shape,
                       const int32_t* sq_spacing, int32_t* dist_sq, void* stream) {
    lt::CallScope call_scope_("lt_edt_aniso", ndim, shape, (int)dtype, -1);
    Geom g;
    Spacing sp;
    lt_status st = common_checks(ctx, labels, dtype, ndim, shape, &g);
    if (st || (st = spacing_from(ndim, g, sq_spacing, &sp))) return st;
    if (g.n == 0) return LT_OK;
    if (!dist_sq) return set_error(LT_E_ARG, "dist_sq is NULL");
    if ((st = ensure_scratch(ctx, edt_scratch_bytes(g)))) return st;
    return launch_edt(ctx, labels, dtype, g, dist_sq, ctx->scratch.ptr, (hipStream_t)stream, nullptr, &sp);
}

lt_status lt_thickness_aniso(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim, const int64_t* shape,
                             const int32_t* sq_spacing, const int32_t* dist_sq, uint32_t max_label, int32_t* lt_sq,
                             void* stream) {
    lt::CallScope call_scope_("lt_thickness_aniso", ndim, shape, (int)dtype, (long long)max_label);
    Geom g;
    Spacing sp;
    lt_status st = common_checks(ctx, labels, dtype, ndim, shape, &g);
    if (st || (st = spacing_from(ndim, g, sq_spacing, &sp))) return st;
    if (g.n == 0) return LT_OK;
    if (!dist_sq || !lt_sq) return set_error(LT_E_ARG, "dist_sq or lt_sq is NULL");
    if (max_label > (1u << 28)) return set_error(LT_E_ARG, "max_label %u exceeds 2^28", max_label);
    if ((st = ensure_scratch(ctx, thickness_scratch_bytes(g, max_label)))) return st;
    return launch_thickness(ctx, labels, dtype, g, dist_sq, max_label, lt_sq, ctx->scratch.ptr, (hipStream_t)stream,
                            nullptr, nullptr, &sp);
}

lt_status lt_object_measures_aniso(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim, const int64_t* shape,
                                   const int32_t* sq_spacing, const int32_t* lt_sq, uint32_t max_label,
                                   const lt_measures* out, void* stream) {
    lt::CallScope call_scope_("lt_object_measures_aniso", ndim, shape, (int)dtype, (long long)max_label);
    Geom g;
    Spacing sp;
    lt_status st = common_checks(ctx, labels, dtype, ndim, shape, &g);
    if (st || (st = spacing_from(ndim, g, sq_spacing, &sp))) return st;
    if (!out || !out->volume || !out->shell_count || !out->max_lt_sq || !out->mean_lt ||
        !out->shell_mean_lt || !out->sphericity || !out->roundness)
        return set_error(LT_E_ARG, "an output array of lt_measures is NULL");
    if (g.n > 0 && !lt_sq) return set_error(LT_E_ARG, "lt_sq is NULL");
    if (max_label > (1u << 28)) return set_error(LT_E_ARG, "max_label %u exceeds 2^28", max_label);
    if ((st = ensure_scratch(ctx, measures_scratch_bytes(max_label)))) return st;
    return launch_measures(ctx, labels, dtype, g, lt_sq, max_label, out, ctx->scratch.ptr, (hipStream_t)stream,
                           sp.vsize);
}

lt_status lt_pipeline_aniso(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim, const int64_t* shape,
                            const int32_t* sq_spacing, uint32_t max_label, int32_t* dist_sq, int32_t* lt_sq,
                            const lt_measures* out, void* stream) {
    lt::CallScope call_scope_("lt_pipeline_aniso", ndim, shape, (int)dtype, (long long)max_label);
    Geom g;
    Spacing sp;
    lt_status st = common_checks(ctx, labels, dtype, ndim, shape, &g);
    if (st || (st = spacing_from(ndim, g, sq_spacing, &sp))) return st;
    if (!out || !out->volume || !out->shell_count || !out->max_lt_sq || !out->mean_lt ||
        !out->shell_mean_lt || !out->sphericity || !out->roundness)
        return set_error(LT_E_ARG, "an output array of lt_measures is NULL");
    if (g.n > 0 && (!dist_sq || !lt_sq)) return set_error(LT_E_ARG, "dist_sq or lt_sq is NULL");
    if (max_label > (1u << 28)) return set_error(LT_E_ARG, "max_label %u exceeds 2^28", max_label);
    if ((st = ensure_scratch(ctx, pipeline_scratch_bytes(g, max_label)))) return st;
    return launch_pipeline(ctx, labels, dtype, g, max_label, dist_sq, lt_sq, out, ctx->scratch.ptr,
                           (hipStream_t)stream, &sp);
}

lt_status lt_filtered_roundness(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim, const int64_t* shape,
                                const int32_t* dist_sq, const int32_t* lt_sq, uint32_t max_label, int half_width,
                                float* roundness, void* stream) {
    lt::CallScope call_scope_("lt_filtered_roundness", ndim, shape, (int)dtype, (long long)max_label);
    if (half_width < 0 || half_width > LT_ROUGH_MAX_HALF_WIDTH)
        return set_error(LT_E_ARG, "half_width %d outside 0..%d", half_width, LT_ROUGH_MAX_HALF_WIDTH);
    if (max_label > (1u << 28)) return set_error(LT_E_ARG, "max_label %u exceeds 2^28", max_label);
    if (!roundness) return set_error(LT_E_ARG, "roundness is NULL");
    Geom g;
    lt_status st = common_checks(ctx, labels, dtype, ndim, shape, &g);
    if (st) return st;
    if (g.n > 0 && (!dist_sq || !lt_sq)) return set_error(LT_E_ARG, "dist_sq or lt_sq is NULL");
    if ((st = ensure_scratch(ctx, rough_scratch_bytes(g, max_label)))) return st;
    return launch_filtered_roundness(ctx, labels, dtype, g, dist_sq, lt_sq, max_label, half_width, roundness,
                                     ctx->scratch.ptr, (hipStream_t)stream);
}

lt_status lt_remap_roundness(lt_ctx* ctx, const float* roundness, uint32_t n, float r_min, float* out,
                             void* stream) {
    lt::CallScope call_scope_("lt_remap_roundness");
    if (!ctx) return set_error(LT_E_ARG, "ctx is NULL");
    if (n == 0) return LT_OK;
    if (!roundness || !out) return set_error(LT_E_ARG, "roundness or out is NULL");
    if (!isnan(r_min) && !isfinite(r_min)) return set_error(LT_E_ARG, "r_min must be finite or NaN");
    lt_status st = hip_check(hipSetDevice(ctx->device), "hipSetDevice");
    if (st) return st;
    if ((st = ensure_scratch(ctx, 256))) return st;
    return launch_remap(ctx, roundness, n, r_min, out, ctx->scratch.ptr, (hipStream_t)stream);
}

lt_status lt_mesh_table(int ndim, double* out) {
    lt::CallScope call_scope_("lt_mesh_table");
    if (ndim != 2 && ndim != 3) return set_error(LT_E_SHAPE, "ndim must be 2 or 3 (got %d)", ndim);
    if (!out) return set_error(LT_E_ARG, "out is NULL");
    return mesh_table_host(ndim, out);
}

size_t lt_pipeline_static_bytes(int ndim, const int64_t* shape, uint32_t max_label) {
    Geom g;
    if (geom_from(ndim, shape, &g) != LT_OK || max_label > (1u << 28)) return 0;
    return pipeline_scratch_bytes(g, max_label);
}

lt_status lt_pipeline_static(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim, const int64_t* shape,
                             uint32_t max_label, int32_t* dist_sq, int32_t* lt_sq, const lt_measures* out,
                             void* stream) {
    lt::CallScope call_scope_("lt_pipeline_static", ndim, shape, (int)dtype, (long long)max_label);
    // sizes first (host arithmetic only), then the common checks, which select the device
    if (!ctx) return set_error(LT_E_ARG, "ctx is NULL");
    Geom g;
    lt_status st = geom_from(ndim, shape, &g);
    if (st) return st;
    if (max_label > (1u << 28)) return set_error(LT_E_ARG, "max_label %u exceeds 2^28", max_label);
    const size_t need = pipeline_scratch_bytes(g, max_label);
    if (need > STATIC_SCRATCH_BYTES)
        return set_error(LT_E_WORKSPACE, "lt_pipeline_static needs %zu bytes of scratch; its fixed scratch holds %zu",
                         need, STATIC_SCRATCH_BYTES);
    if ((st = common_checks(ctx, labels, dtype, ndim, shape, &g))) return st;
    if (!out || !out->volume || !out->shell_count || !out->max_lt_sq || !out->mean_lt ||
        !out->shell_mean_lt || !out->sphericity || !out->roundness)
        return set_error(LT_E_ARG, "an output array of lt_measures is NULL");
    if (g.n > 0 && (!dist_sq || !lt_sq)) return set_error(LT_E_ARG, "dist_sq or lt_sq is NULL");
    if (!ctx->static_scratch) return set_error(LT_E_NOT_READY, "the context has no fixed scratch address");
    // the per-kernel profiler creates HIP events; this call makes no such call
    const bool prof = ctx->profile;
    ctx->profile = false;
    st = launch_pipeline(ctx, labels, dtype, g, max_label, dist_sq, lt_sq, out, ctx->static_scratch,
                         (hipStream_t)stream);
    ctx->profile = prof;
    return st;
}

lt_status lt_closed_forms(const uint64_t* volume, const uint64_t* sum_lt_q23,
                          const int32_t* max_lt_sq, const uint64_t* shell_count,
                          const uint64_t* shell_sum_q23, uint32_t n, int ndim, float* mean_lt,
                          float* shell_mean_lt, float* sphericity, float* roundness,
                          void* stream) {
    lt::CallScope call_scope_("lt_closed_forms");
    if (ndim != 2 && ndim != 3) return set_error(LT_E_SHAPE, "ndim must be 2 or 3 (got %d)", ndim);
    if (n == 0) return LT_OK;
    if (!volume || !sum_lt_q23 || !max_lt_sq || !shell_count || !shell_sum_q23 || !mean_lt ||
        !shell_mean_lt || !sphericity || !roundness)
        return set_error(LT_E_ARG, "an array is NULL");
    return launch_closed_forms(volume, sum_lt_q23, max_lt_sq, shell_count, shell_sum_q23, n, ndim,
                               mean_lt, shell_mean_lt, sphericity, roundness, (hipStream_t)stream);
}

lt_status lt_ctx_info(lt_ctx* ctx, int* n_cu, uint64_t* lds_per_block, int* paint_tile_rows_out) {
    lt::CallScope call_scope_("lt_ctx_info");
    if (!ctx) return set_error(LT_E_ARG, "ctx is NULL");
    if (n_cu) *n_cu = ctx->n_cu;
    if (lds_per_block) *lds_per_block = ctx->lds_per_block;
    if (paint_tile_rows_out) *paint_tile_rows_out = paint_tile_rows(ctx);
    return LT_OK;
}

lt_status lt_profile_enable(lt_ctx* ctx, int on) {
    lt::CallScope call_scope_("lt_profile_enable");
    if (!ctx) return set_error(LT_E_ARG, "ctx is NULL");
    ctx->profile = on != 0;
    return LT_OK;
}

lt_status lt_profile_read(lt_ctx* ctx, lt_kernel_time* out, int cap, int* n_out) {
    lt::CallScope call_scope_("lt_profile_read");
    if (!ctx || (cap > 0 && !out)) return set_error(LT_E_ARG, "ctx or out is NULL");
    lt_status st = hip_check(hipSetDevice(ctx->device), "hipSetDevice");
    if (st) return st;
    for (const PendingTiming& p : ctx->pending) {
        float ms = 0.f;
        if (!st) st = hip_check(hipEventSynchronize(p.stop), "hipEventSynchronize");
        if (!st) st = hip_check(hipEventElapsedTime(&ms, p.start, p.stop), "hipEventElapsedTime");
        (void)hipEventDestroy(p.start);
        (void)hipEventDestroy(p.stop);
        if (st) continue;
        KernelTotal* t = nullptr;
        for (KernelTotal& k : ctx->totals)
            if (strcmp(k.name, p.name) == 0) t = &k;
        if (!t) {
            ctx->totals.push_back(KernelTotal{p.name, 0.0, 0});
            t = &ctx->totals.back();
        }
        t->ms += ms;
        t->launches += 1;
    }
    ctx->pending.clear();
    if (st) return st;
    int n = 0;
    for (const KernelTotal& k : ctx->totals) {
        if (n < cap) {
            snprintf(out[n].name, sizeof(out[n].name), "%s", k.name);
            out[n].total_ms = k.ms;
            out[n].launches = k.launches;
        }
        ++n;
    }
    if (n_out) *n_out = n;
    return LT_OK;
}

lt_status lt_profile_reset(lt_ctx* ctx) {
    lt::CallScope call_scope_("lt_profile_reset");
    if (!ctx) return set_error(LT_E_ARG, "ctx is NULL");
    int n = 0;
    lt_status st = lt_profile_read(ctx, nullptr, 0, &n);
    ctx->totals.clear();
    return st;
}

lt_status lt_sync_status(lt_ctx* ctx, void* stream) {
    lt::CallScope call_scope_("lt_sync_status");
    if (!ctx) return set_error(LT_E_ARG, "ctx is NULL");
    lt_status st = hip_check(hipSetDevice(ctx->device), "hipSetDevice");
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    uint32_t err = 0;
    if ((st = hip_check(hipStreamSynchronize(s), "hipStreamSynchronize"))) return st;
    if ((st = hip_check(hipMemcpy(&err, ctx->d_err, sizeof(err), hipMemcpyDeviceToHost), "read err")))
        return st;
    if ((st = hip_check(hipMemset(ctx->d_err, 0, sizeof(uint32_t)), "clear err"))) return st;
    if (err & ERR_LABEL) return set_error(LT_E_LABEL_RANGE, "a label exceeded max_label or was negative");
    if (err & ERR_OVERFLOW) return set_error(LT_E_OVERFLOW, "an intermediate exceeded its range");
    return LT_OK;
}

}  // extern "C"
