// Batched form: many volumes of uneven size in one graph launch, and the autotuner
// that chooses the runtime kernel knobs.
//
// lt_batch_create assigns the volumes to `batch_lanes` streams (largest volumes
// first, each to the least-loaded lane), gives every lane its own scratch region,
// and captures the whole pipeline of every volume into one hipGraph: the lanes fork
// from and join back into one origin stream, so independent volumes may run
// concurrently.  lt_batch_run replays it with a single hipGraphLaunch.  The graph
// holds kernel nodes only (no memset or allocation nodes).  Each volume's kernels
// record device-detected errors in that volume's own error word, so one bad volume
// is reported as such and does not mark the others (lt_batch_status).
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lt_internal.h"

struct lt_batch {
    lt_ctx* ctx = nullptr;
    void* scratch = nullptr;
    uint32_t* d_status = nullptr;       // one device error word per volume
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int n = 0;
    int lanes = 0;
};

namespace lt {

static lt_status launch_volume(lt_ctx* ctx, const lt_volume& v, lt_dtype dt, const Geom& g, void* scratch,
                               hipStream_t s) {
    return launch_pipeline(ctx, v.labels, dt, g, v.max_label, v.dist_sq, v.lt_sq, &v.measures, scratch, s);
}

static lt_status check_volume(const lt_volume& v, Geom* g) {
    lt_status st = geom_from(v.ndim, v.shape, g);
    if (st) return st;
    if (g->n > 0 && (!v.labels || !v.dist_sq || !v.lt_sq))
        return set_error(LT_E_ARG, "a volume has a NULL labels / dist_sq / lt_sq pointer");
    const lt_measures& m = v.measures;
    if (!m.volume || !m.shell_count || !m.max_lt_sq || !m.mean_lt || !m.shell_mean_lt ||
        !m.sphericity || !m.roundness)
        return set_error(LT_E_ARG, "a volume has a NULL measures array");
    if (v.max_label > (1u << 28)) return set_error(LT_E_ARG, "max_label exceeds 2^28");
    return LT_OK;
}

}  // namespace lt

using namespace lt;

extern "C" {

lt_status lt_get_tuning(lt_ctx* ctx, lt_tuning* out) {
    lt::CallScope call_scope_("lt_get_tuning");
    if (!ctx || !out) return set_error(LT_E_ARG, "ctx or out is NULL");
    out->paint_tile_rows = paint_tile_rows(ctx);
    out->paint_blocks_per_cu = ctx->tune.paint_blocks_per_cu;
    out->front_chunk = ctx->tune.front_chunk;
    out->batch_lanes = ctx->tune.batch_lanes;
    return LT_OK;
}

lt_status lt_set_tuning(lt_ctx* ctx, const lt_tuning* t) {
    lt::CallScope call_scope_("lt_set_tuning");
    if (!ctx || !t) return set_error(LT_E_ARG, "ctx or tuning is NULL");
    if (t->paint_tile_rows != 0 && t->paint_tile_rows != 32 && t->paint_tile_rows != 64)
        return set_error(LT_E_ARG, "paint_tile_rows must be 0, 32 or 64");
    if (t->paint_blocks_per_cu < 1 || t->paint_blocks_per_cu > 2)
        return set_error(LT_E_ARG, "paint_blocks_per_cu must be 1 or 2");
    if (t->front_chunk != 32 && t->front_chunk != 64 && t->front_chunk != 128)
        return set_error(LT_E_ARG, "front_chunk must be 32, 64 or 128");
    if (t->batch_lanes < 1 || t->batch_lanes > 16) return set_error(LT_E_ARG, "batch_lanes must be 1..16");
    ctx->tune.paint_tile_rows = t->paint_tile_rows;
    ctx->tune.paint_blocks_per_cu = t->paint_blocks_per_cu;
    ctx->tune.front_chunk = t->front_chunk;
    ctx->tune.batch_lanes = t->batch_lanes;
    return LT_OK;
}

lt_status lt_batch_create(lt_ctx* ctx, const lt_volume* vols, int n, lt_dtype dtype, lt_batch** out) {
    lt::CallScope call_scope_("lt_batch_create", 0, nullptr, (int)dtype);
    if (!ctx || !out || (n > 0 && !vols)) return set_error(LT_E_ARG, "ctx, vols or out is NULL");
    *out = nullptr;
    if (n < 0) return set_error(LT_E_ARG, "negative volume count");
    if (dtype != LT_U16 && dtype != LT_I32 && dtype != LT_U32)
        return set_error(LT_E_DTYPE, "unknown label dtype %d", (int)dtype);
    lt_status st = hip_check(hipSetDevice(ctx->device), "hipSetDevice");
    if (st) return st;
    std::vector<Geom> geo(n);
    std::vector<size_t> need(n);
    for (int i = 0; i < n; ++i) {
        if ((st = check_volume(vols[i], &geo[i]))) return st;
        need[i] = pipeline_scratch_bytes(geo[i], vols[i].max_label);
    }
    const int lanes = std::max(1, std::min(ctx->tune.batch_lanes, std::max(n, 1)));
    // largest first onto the least-loaded lane
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return geo[a].n > geo[b].n; });
    std::vector<std::vector<int>> lane_vols(lanes);
    std::vector<size_t> load(lanes, 0), lane_bytes(lanes, 0);
    for (int i : order) {
        const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        lane_vols[k].push_back(i);
        load[k] += geo[i].n + 1;
        lane_bytes[k] = std::max(lane_bytes[k], need[i]);
    }
    std::vector<size_t> lane_off(lanes, 0);
    size_t total = 0;
    for (int k = 0; k < lanes; ++k) {
        lane_off[k] = total;
        total += (lane_bytes[k] + 255) & ~size_t(255);
    }
    lt_batch* b = new (std::nothrow) lt_batch();
    if (!b) return set_error(LT_E_ALLOC, "host allocation failed");
    b->ctx = ctx;
    b->n = n;
    b->lanes = lanes;
    if ((total > 0 && (st = device_alloc(&b->scratch, total, "hipMalloc(batch scratch)"))) ||
        (st = device_alloc((void**)&b->d_status, (size_t)std::max(n, 1) * sizeof(uint32_t),
                           "hipMalloc(batch status)")) ||
        (st = hip_check(hipMemset(b->d_status, 0, (size_t)std::max(n, 1) * sizeof(uint32_t)), "clear batch status"))) {
        lt_batch_destroy(b);
        return st;
    }
    (void)paint_tile_rows(ctx);                 // one-time kernel attributes, outside capture
    hipStream_t origin = nullptr;
    std::vector<hipStream_t> ls(lanes, nullptr);
    std::vector<hipEvent_t> ev(lanes + 1, nullptr);
    bool capturing = false;
    const bool prof = ctx->profile;
    ctx->profile = false;                       // no timing events inside the graph
    auto fail = [&](lt_status s) {
        if (capturing) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(origin, &g);
            if (g) (void)hipGraphDestroy(g);
        }
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto& q : ls)
            if (q) (void)hipStreamDestroy(q);
        if (origin) (void)hipStreamDestroy(origin);
        ctx->profile = prof;
        lt_batch_destroy(b);
        return s;
    };
    if ((st = hip_check(hipStreamCreateWithFlags(&origin, hipStreamNonBlocking), "hipStreamCreate")))
        return fail(st);
    for (int k = 0; k < lanes; ++k)
        if ((st = hip_check(hipStreamCreateWithFlags(&ls[k], hipStreamNonBlocking), "hipStreamCreate")))
            return fail(st);
    for (auto& e : ev)
        if ((st = hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreate")))
            return fail(st);
    if ((st = hip_check(hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal), "begin capture")))
        return fail(st);
    capturing = true;
    if ((st = hip_check(hipEventRecord(ev[lanes], origin), "fork record"))) return fail(st);
    for (int k = 0; k < lanes; ++k) {
        if ((st = hip_check(hipStreamWaitEvent(ls[k], ev[lanes], 0), "fork wait"))) return fail(st);
        void* scr = (char*)b->scratch + lane_off[k];
        for (int i : lane_vols[k]) {
            // the volume's kernels take its own error word while they are captured
            uint32_t* ctx_err = ctx->d_err;
            ctx->d_err = b->d_status + i;
            if (geo[i].n > 0) st = launch_volume(ctx, vols[i], dtype, geo[i], scr, ls[k]);
            ctx->d_err = ctx_err;
            if (st) return fail(st);
        }
        if ((st = hip_check(hipEventRecord(ev[k], ls[k]), "join record"))) return fail(st);
        if ((st = hip_check(hipStreamWaitEvent(origin, ev[k], 0), "join wait"))) return fail(st);
    }
    capturing = false;
    if ((st = hip_check(hipStreamEndCapture(origin, &b->graph), "end capture"))) return fail(st);
    if ((st = hip_check(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "graph instantiate")))
        return fail(st);
    for (auto& e : ev) (void)hipEventDestroy(e);
    for (auto& q : ls) (void)hipStreamDestroy(q);
    (void)hipStreamDestroy(origin);
    ctx->profile = prof;
    *out = b;
    return LT_OK;
}

lt_status lt_batch_run(lt_batch* b, void* stream) {
    lt::CallScope call_scope_("lt_batch_run");
    if (!b) return set_error(LT_E_ARG, "batch is NULL");
    lt_status st = hip_check(hipSetDevice(b->ctx->device), "hipSetDevice");
    if (st) return st;
    if (!b->exec) return LT_OK;
    return hip_check(hipGraphLaunch(b->exec, (hipStream_t)stream), "hipGraphLaunch");
}

lt_status lt_batch_status(lt_batch* b, void* stream, int32_t* status) {
    lt::CallScope call_scope_("lt_batch_status");
    if (!b) return set_error(LT_E_ARG, "batch is NULL");
    lt_status st = hip_check(hipSetDevice(b->ctx->device), "hipSetDevice");
    if (st) return st;
    if ((st = hip_check(hipStreamSynchronize((hipStream_t)stream), "hipStreamSynchronize"))) return st;
    std::vector<uint32_t> w((size_t)std::max(b->n, 1), 0u);
    if ((st = hip_check(hipMemcpy(w.data(), b->d_status, w.size() * sizeof(uint32_t), hipMemcpyDeviceToHost),
                        "read batch status")) ||
        (st = hip_check(hipMemset(b->d_status, 0, w.size() * sizeof(uint32_t)), "clear batch status")))
        return st;
    lt_status first = LT_OK;
    int bad = -1;
    for (int i = 0; i < b->n; ++i) {
        const lt_status v = (w[i] & ERR_LABEL) ? LT_E_LABEL_RANGE : (w[i] & ERR_OVERFLOW) ? LT_E_OVERFLOW : LT_OK;
        if (status) status[i] = (int32_t)v;
        if (v != LT_OK && first == LT_OK) {
            first = v;
            bad = i;
        }
    }
    if (first != LT_OK) return set_error(first, "volume %d of the batch: %s", bad, lt_status_str(first));
    return LT_OK;
}

lt_status lt_batch_destroy(lt_batch* b) {
    lt::CallScope call_scope_("lt_batch_destroy");
    if (!b) return LT_OK;
    (void)hipSetDevice(b->ctx->device);
    (void)hipDeviceSynchronize();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->scratch) (void)hipFree(b->scratch);
    if (b->d_status) (void)hipFree(b->d_status);
    delete b;
    return LT_OK;
}

}  // extern "C"
