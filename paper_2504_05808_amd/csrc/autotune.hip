// Autotuner for the runtime kernel knobs (lt_tuning).
//
// lt_autotune times the whole pipeline on the caller's volume for every candidate
// (paint tile rows x paint blocks per CU x z-front chunk) and keeps the fastest;
// lt_autotune_batch does the same for the number of lanes of a batch graph.  The
// winners are stored in a small JSON file keyed by device architecture, label
// dtype, dimensionality and size class (floor(log2 of the voxel count)), and are
// reused from it on later calls.  Tuning never changes results, only speed.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <string>
#include <vector>

#include "lt_internal.h"

namespace lt {

struct CacheEntry {
    lt_tuning t;
    double ms;
};

static std::map<std::string, CacheEntry> read_cache(const char* path) {
    std::map<std::string, CacheEntry> m;
    if (!path || !*path) return m;
    FILE* f = fopen(path, "r");
    if (!f) return m;
    char line[512];
    while (fgets(line, sizeof(line), f)) {
        char key[256];
        CacheEntry e{};
        if (sscanf(line, " \"%255[^\"]\": {\"paint_tile_rows\": %d, \"paint_blocks_per_cu\": %d, "
                         "\"front_chunk\": %d, \"batch_lanes\": %d, \"ms\": %lf}",
                   key, &e.t.paint_tile_rows, &e.t.paint_blocks_per_cu, &e.t.front_chunk,
                   &e.t.batch_lanes, &e.ms) == 6)
            m[key] = e;
    }
    fclose(f);
    return m;
}

static void write_cache(const char* path, const std::map<std::string, CacheEntry>& m) {
    if (!path || !*path) return;
    std::string tmp = std::string(path) + ".tmp";
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return;
    fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& kv : m) {
        const lt_tuning& t = kv.second.t;
        fprintf(f, "  \"%s\": {\"paint_tile_rows\": %d, \"paint_blocks_per_cu\": %d, \"front_chunk\": %d, "
                   "\"batch_lanes\": %d, \"ms\": %.4f}%s\n",
                kv.first.c_str(), t.paint_tile_rows, t.paint_blocks_per_cu, t.front_chunk, t.batch_lanes,
                kv.second.ms, ++i < m.size() ? "," : "");
    }
    fprintf(f, "}\n");
    fclose(f);
    rename(tmp.c_str(), path);
}

static std::string cache_key(const lt_ctx* ctx, const char* what, lt_dtype dt, int ndim, double voxels) {
    hipDeviceProp_t prop;
    const char* arch = "gfx";
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess) arch = prop.gcnArchName;
    std::string a(arch);
    const size_t colon = a.find(':');
    if (colon != std::string::npos) a = a.substr(0, colon);
    char buf[256];
    snprintf(buf, sizeof(buf), "%s|%s|dtype%d|%dd|n2^%d", a.c_str(), what, (int)dt, ndim,
             voxels > 0 ? (int)floor(log2(voxels)) : 0);
    return buf;
}

// Mean time (ms) of `reps` runs of fn on `s` after one warm-up run.
template <typename F>
static lt_status time_runs(F fn, int reps, hipStream_t s, double* ms) {
    hipEvent_t a, b;
    lt_status st = hip_check(hipEventCreate(&a), "hipEventCreate");
    if (st) return st;
    if ((st = hip_check(hipEventCreate(&b), "hipEventCreate"))) {
        (void)hipEventDestroy(a);
        return st;
    }
    st = fn();
    if (!st) st = hip_check(hipStreamSynchronize(s), "sync");
    if (!st) st = hip_check(hipEventRecord(a, s), "record");
    for (int r = 0; r < reps && !st; ++r) st = fn();
    if (!st) st = hip_check(hipEventRecord(b, s), "record");
    if (!st) st = hip_check(hipEventSynchronize(b), "event sync");
    float t = 0.f;
    if (!st) st = hip_check(hipEventElapsedTime(&t, a, b), "elapsed");
    *ms = t / (reps > 0 ? reps : 1);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return st;
}

}  // namespace lt

using namespace lt;

extern "C" {

lt_status lt_autotune(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim, const int64_t* shape,
                      uint32_t max_label, const char* cache_path, int repeats, lt_tuning* best) {
    lt::CallScope call_scope_("lt_autotune", ndim, shape, (int)dtype, (long long)max_label);
    if (!ctx || !labels) return set_error(LT_E_ARG, "ctx or labels is NULL");
    Geom g;
    lt_status st = geom_from(ndim, shape, &g);
    if (st) return st;
    if (dtype != LT_U16 && dtype != LT_I32 && dtype != LT_U32) return set_error(LT_E_DTYPE, "bad dtype");
    if ((st = hip_check(hipSetDevice(ctx->device), "hipSetDevice"))) return st;
    const std::string key = cache_key(ctx, "pipeline", dtype, ndim, (double)g.n);
    auto cache = read_cache(cache_path);
    auto it = cache.find(key);
    if (it != cache.end()) {
        lt_tuning t = it->second.t;
        t.batch_lanes = ctx->tune.batch_lanes;
        if ((st = lt_set_tuning(ctx, &t))) return st;
        if (best) lt_get_tuning(ctx, best);
        return LT_OK;
    }
    if (g.n == 0) return LT_OK;
    // temporary outputs
    const size_t nlab = (size_t)max_label + 1;
    void* buf = nullptr;
    const size_t fields = 2 * g.n * sizeof(int32_t);
    const size_t per = 2 * sizeof(uint64_t) + sizeof(int32_t) + 4 * sizeof(float);
    if ((st = device_alloc(&buf, fields + nlab * per + 1024, "hipMalloc(autotune)"))) return st;
    char* p = (char*)buf;
    int32_t* dist = (int32_t*)p;
    int32_t* ltq = (int32_t*)(p + g.n * sizeof(int32_t));
    char* q = p + fields;
    lt_measures m;
    m.volume = (uint64_t*)q;           q += nlab * sizeof(uint64_t);
    m.shell_count = (uint64_t*)q;      q += nlab * sizeof(uint64_t);
    m.mean_lt = (float*)q;             q += nlab * sizeof(float);
    m.shell_mean_lt = (float*)q;       q += nlab * sizeof(float);
    m.sphericity = (float*)q;          q += nlab * sizeof(float);
    m.roundness = (float*)q;           q += nlab * sizeof(float);
    m.max_lt_sq = (int32_t*)q;
    m.hist32 = nullptr;
    hipStream_t s = nullptr;
    const lt_tuning saved{ctx->tune.paint_tile_rows, ctx->tune.paint_blocks_per_cu, ctx->tune.front_chunk,
                          ctx->tune.batch_lanes};
    const int rows_opts[] = {64, 32};
    const int chunk_opts[] = {32, 64, 128};
    double best_ms = 1e30;
    lt_tuning win = saved;
    for (int rows : rows_opts)
        for (int per_cu = 1; per_cu <= (rows == 32 ? 2 : 1); ++per_cu)
            for (int chunk : chunk_opts) {
                if (g.ndim == 2 && chunk != 64) continue;      // no z-front pass in 2D
                lt_tuning t{rows, per_cu, chunk, saved.batch_lanes};
                if ((st = lt_set_tuning(ctx, &t))) break;
                if ((st = ensure_scratch(ctx, pipeline_scratch_bytes(g, max_label)))) break;
                void* scr = ctx->scratch.ptr;
                double ms = 0.0;
                st = time_runs([&]() -> lt_status {
                    lt_status r = launch_pipeline(ctx, labels, dtype, g, max_label, dist, ltq, &m, scr, s);
                    return r;
                }, repeats > 0 ? repeats : 3, s, &ms);
                if (st) break;
                if (ms < best_ms) {
                    best_ms = ms;
                    win = t;
                }
            }
    (void)hipDeviceSynchronize();
    (void)hipFree(buf);
    if (st) {
        lt_set_tuning(ctx, &saved);
        return st;
    }
    lt_set_tuning(ctx, &win);
    cache[key] = CacheEntry{win, best_ms};
    write_cache(cache_path, cache);
    if (best) lt_get_tuning(ctx, best);
    return LT_OK;
}

lt_status lt_autotune_batch(lt_ctx* ctx, const lt_volume* vols, int n, lt_dtype dtype,
                            const char* cache_path, int repeats, lt_tuning* best) {
    lt::CallScope call_scope_("lt_autotune_batch", 0, nullptr, (int)dtype);
    if (!ctx || !vols || n <= 0) return set_error(LT_E_ARG, "ctx or vols is NULL / empty");
    double voxels = 0;
    int ndim = vols[0].ndim;
    for (int i = 0; i < n; ++i) {
        Geom g;
        lt_status st = geom_from(vols[i].ndim, vols[i].shape, &g);
        if (st) return st;
        voxels += (double)g.n;
    }
    const std::string key = cache_key(ctx, "batch", dtype, ndim, voxels);
    auto cache = read_cache(cache_path);
    auto it = cache.find(key);
    if (it != cache.end()) {
        lt_tuning t{ctx->tune.paint_tile_rows, ctx->tune.paint_blocks_per_cu, ctx->tune.front_chunk,
                    it->second.t.batch_lanes};
        lt_status st = lt_set_tuning(ctx, &t);
        if (!st && best) lt_get_tuning(ctx, best);
        return st;
    }
    const int saved = ctx->tune.batch_lanes;
    int win = saved;
    double best_ms = 1e30;
    lt_status st = LT_OK;
    for (int lanes : {1, 2, 4, 8}) {
        if (lanes > n && lanes > 1) break;
        ctx->tune.batch_lanes = lanes;
        lt_batch* b = nullptr;
        if ((st = lt_batch_create(ctx, vols, n, dtype, &b))) break;
        double ms = 0.0;
        st = time_runs([&]() { return lt_batch_run(b, nullptr); }, repeats > 0 ? repeats : 3, nullptr, &ms);
        lt_batch_destroy(b);
        if (st) break;
        if (ms < best_ms) {
            best_ms = ms;
            win = lanes;
        }
    }
    ctx->tune.batch_lanes = st ? saved : win;
    if (st) return st;
    lt_tuning t{ctx->tune.paint_tile_rows, ctx->tune.paint_blocks_per_cu, ctx->tune.front_chunk, win};
    cache[key] = CacheEntry{t, best_ms};
    write_cache(cache_path, cache);
    if (best) lt_get_tuning(ctx, best);
    return LT_OK;
}

}  // extern "C"
