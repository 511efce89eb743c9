// Internal declarations shared by the liblt translation units (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include <array>
#include <utility>
#include <vector>

#include "../../include/lt.h"

namespace lt {

// Device error word bits.
enum : uint32_t { ERR_LABEL = 1u, ERR_OVERFLOW = 2u };

// Largest squared radius covered by the exact containment-prune tables.  Centres
// with a larger D are tested against the containment bound (prune_bound), which
// keeps a few more centres than the table would (always exact).
constexpr int PRUNE_DCAP = 16384;

// Paint tile: up to TILE_Y_MAX target rows x TILE_X columns per work item (columns
// along x); the row count is 64 when a block may hold the 7-level table for 64 rows
// in LDS (gfx950: 160 KB), else 32.  Rows are padded to TILE_STRIDE words so that
// the lanes of a wave (one row each) fall in different LDS banks.
constexpr int TILE_Y_MAX = 64;
constexpr int TILE_X = 64;
constexpr int TILE_STRIDE = TILE_X + 1;
constexpr int TILE_LEVELS = 7;                 // interval lengths 1..64 -> levels 0..6
constexpr int PAINT_THREADS = 1024;

// Row scans (EDT pass x): rows up to 2048 voxels = 32 wave chunks.
constexpr int ROW_MAX_CHUNKS = 32;

// Packed z-front entry (3D): bits 0..18 D of the centre, 19..28 dz + 512 (dz is
// the slice minus the centre's z), 29..31 (plane 0 only) number of entries.  The
// count 7 marks a front longer than ZF_PLANES: with ZF_SPILL set, bits 16..23 hold
// its length and either (ZF_POOL clear) bits 0..15 its offset in the spill region of
// the front pass's block (row of 64 columns, z chunk) that owns the voxel, or
// (ZF_POOL set) plane 1 its offset in the shared spill pool; without ZF_SPILL the
// column is rescanned.
constexpr uint32_t ZF_D_BITS = 19;
constexpr uint32_t ZF_D_MASK = (1u << ZF_D_BITS) - 1u;
constexpr uint32_t ZF_DZ_SHIFT = 19;
constexpr uint32_t ZF_DZ_MASK = 1023u;
constexpr uint32_t ZF_N_SHIFT = 29;
constexpr int ZF_PLANES = 4;
constexpr uint32_t ZF_SPILL = 1u << 28;
constexpr uint32_t ZF_POOL = 1u << 24;
constexpr int ZF_LONG_MAX = 255;               // longest front the 8-bit length holds
// Spill words per (row of 64 columns, slice) of the front pass: one word per voxel;
// a block whose long fronts need more takes them from the shared pool.
constexpr int SPILL_ROW_SLICE = 64;

// Shared spill pool of the front passes (one word per voxel): long fronts that do
// not fit their block's region.  `used` counts requested words (64-bit: requests go
// on after the pool is full); a front that does not fit is rescanned instead.
struct SpillPool {
    uint32_t* base;
    unsigned long long* used;
    unsigned long long cap;
};

// Column-list entry (3D): (D << 11) | z.
constexpr uint32_t CL_Z_BITS = 11;
constexpr uint32_t CL_Z_MASK = (1u << CL_Z_BITS) - 1u;

// Anisotropic spacing: integer squared voxel spacings along z, y, x (a distance
// step along axis a costs w_a), and the physical voxel volume (area in 2D)
// sqrt(prod w) that the sphericity's V takes.  Unit spacing is the paper's case.
struct Spacing {
    int wz = 1, wy = 1, wx = 1;
    float vsize = 1.0f;
    bool unit() const { return wz == 1 && wy == 1 && wx == 1; }
};

struct Geom {
    int ndim;
    int nz, ny, nx;     // ndim == 2: nz == 1
    size_t n;           // voxel count
};

struct Scratch {
    void* ptr = nullptr;
    size_t bytes = 0;
};

// Runtime kernel knobs (chosen by the autotuner or set by the caller; 0 = default).
struct Tuning {
    int paint_tile_rows = 0;      // 32 or 64 rows per paint tile (0: 64 when LDS allows)
    int paint_blocks_per_cu = 1;  // persistent paint blocks per compute unit (1 or 2)
    int front_chunk = 64;         // slices per block of the z-front pass (32, 64 or 128)
    int batch_lanes = 4;          // concurrent streams in a captured batch graph
};

// One timed launch: events recorded on the launch stream around the kernel.
struct PendingTiming {
    const char* name;
    hipEvent_t start, stop;
};

struct KernelTotal {
    const char* name;
    double ms;
    uint64_t launches;
};

}  // namespace lt

struct lt_ctx {
    int device = 0;
    int n_cu = 0;
    size_t lds_per_block = 0;
    uint32_t* d_err = nullptr;          // device error word
    int32_t* d_prune3 = nullptr;        // [PRUNE_DCAP + 1][4]: T(|o|^2 = 1, 2, 3) for d, then 0
    int32_t* d_prune2 = nullptr;        // [2][PRUNE_DCAP + 1] (|o|^2 = 1, 2)
    lt::Scratch scratch;                // grows on demand, freed by lt_ctx_destroy
    void* static_scratch = nullptr;     // this device's copy of the fixed scratch of
                                        // lt_pipeline_static (never freed)
    // weighted prune tables per spacing (ndim, wz, wy, wx) -> device table; kept until
    // the context is destroyed (a table in use by queued kernels is never rewritten)
    std::vector<std::pair<std::array<int, 4>, int32_t*>> prune_w;
    lt::Tuning tune;
    bool mesh_ready = false;            // mesh area tables copied to this device
    bool profile = false;               // time every launch with HIP events
    std::vector<lt::PendingTiming> pending;
    std::vector<lt::KernelTotal> totals;
};

namespace lt {

// Host helpers (api.hip).
lt_status set_error(lt_status s, const char* fmt, ...);

// Scope of an exported call on the host: names the call in the LT_LOG lines (level 2
// prints the call with its volume arguments; level 1 prints every error status with
// the name of the call it came from).  Restores the enclosing name on exit.
struct CallScope {
    const char* prev;
    explicit CallScope(const char* fn, int ndim = 0, const int64_t* shape = nullptr, int dtype = -1,
                       long long max_label = -1);
    ~CallScope();
};
lt_status hip_check(hipError_t e, const char* what);
lt_status ensure_scratch(lt_ctx* ctx, size_t bytes);
// hipMalloc through the allocation fault injection (LT_FAULT_INJECT=alloc[:N]).
lt_status device_alloc(void** p, size_t bytes, const char* what);
lt_status geom_from(int ndim, const int64_t* shape, Geom* g);

// Where the EDT x pass records bounding boxes (fused pipeline): device boxes of
// nlab labels, and the largest valid label (larger labels set ERR_LABEL).
struct BoxTarget {
    int32_t* bb;
    uint32_t nlab;
    uint32_t max_label;
};

// Launchers (edt.hip, thickness.hip, measures.hip).  All are stream-ordered, use the
// caller's scratch region (at least *_scratch_bytes bytes, 256-byte aligned) and
// allocate nothing, so they can be captured into a graph.
size_t edt_scratch_bytes(const Geom& g);
// With `box` set, the x pass also records the per-label bounding boxes (fused
// pipeline; the boxes must have been emptied first).
lt_status launch_edt(lt_ctx* ctx, const void* labels, lt_dtype dt, const Geom& g,
                     int32_t* dist_sq, void* scratch, hipStream_t s, const BoxTarget* box = nullptr,
                     const Spacing* sp = nullptr);
lt_status launch_init_boxes(lt_ctx* ctx, int32_t* bb, uint32_t nlab, hipStream_t s);
size_t thickness_scratch_bytes(const Geom& g, uint32_t max_label);
int paint_tile_rows(lt_ctx* ctx);
// Device arrays of the per-object integer sums (zeroed by launch_measures_zero).
struct MeasureSums {
    uint64_t* vol;
    uint64_t* shc;
    int32_t* mx;
    uint64_t* sq;
    uint64_t* ssq;
};
// With `sums` set, the paint pass also accumulates the per-object sums of the
// measures (the fused form); launch_measures_finish then completes them.
// With `boxes` set, the bounding boxes come from the caller (recorded by the EDT x
// pass) and the box pass is skipped.
lt_status launch_thickness(lt_ctx* ctx, const void* labels, lt_dtype dt, const Geom& g,
                           const int32_t* dist_sq, uint32_t max_label, int32_t* lt_sq,
                           void* scratch, hipStream_t s, const MeasureSums* sums = nullptr,
                           int32_t* boxes = nullptr, const Spacing* sp = nullptr);
// Containment tables of the weighted prune for this spacing (one row per offset
// class: 7 in 3D, 3 in 2D), built on the host on first use and kept by the context.
lt_status prune_tables_weighted(lt_ctx* ctx, int ndim, const Spacing& sp, const int32_t** out);
size_t measures_scratch_bytes(uint32_t max_label);
lt_status launch_measures(lt_ctx* ctx, const void* labels, lt_dtype dt, const Geom& g,
                          const int32_t* lt_sq, uint32_t max_label, const lt_measures* out,
                          void* scratch, hipStream_t s, float vsize = 1.0f);
lt_status launch_measures_zero(lt_ctx* ctx, uint32_t max_label, const lt_measures* out, void* scratch,
                               hipStream_t s, MeasureSums* sums);
lt_status launch_measures_finish(lt_ctx* ctx, const void* labels, lt_dtype dt, const Geom& g,
                                 const int32_t* lt_sq, uint32_t max_label, const lt_measures* out,
                                 void* scratch, hipStream_t s, float vsize = 1.0f);
// Mesh-based surface measures (mesh.hip): per-label voxel count, iso-surface area
// (3D) or contour length (2D) and mesh sphericity; any output may be NULL.
size_t mesh_scratch_bytes(uint32_t max_label);
lt_status mesh_table_host(int ndim, double* out);
lt_status launch_mesh(lt_ctx* ctx, const void* labels, lt_dtype dt, const Geom& g, uint32_t max_label,
                      uint64_t* volume, float* area, float* sphericity, void* scratch, hipStream_t s);
// Roughness-filtered roundness (roughness.hip): separable same-label window maxima
// of the shell LT, reduced per label; and the 0-1 remap of roundness values.
size_t rough_scratch_bytes(const Geom& g, uint32_t max_label);
lt_status launch_filtered_roundness(lt_ctx* ctx, const void* labels, lt_dtype dt, const Geom& g,
                                    const int32_t* D, const int32_t* lt, uint32_t max_label, int w,
                                    float* roundness, void* scratch, hipStream_t s);
lt_status launch_remap(lt_ctx* ctx, const float* r, uint32_t n, float r_min, float* out, void* scratch,
                       hipStream_t s);
// Scratch for the fused pipeline: EDT, then thickness with the measures' scratch
// placed after the thickness region (both live during the paint pass).
size_t pipeline_scratch_bytes(const Geom& g, uint32_t max_label);
size_t pipeline_measures_offset(const Geom& g, uint32_t max_label);
// EDT -> thickness with fused sums -> histogram and closed forms.
lt_status launch_pipeline(lt_ctx* ctx, const void* labels, lt_dtype dt, const Geom& g, uint32_t max_label,
                          int32_t* dist_sq, int32_t* lt_sq, const lt_measures* out, void* scratch,
                          hipStream_t s, const Spacing* sp = nullptr);
lt_status launch_closed_forms(const uint64_t* volume, const uint64_t* sum_lt_q,
                              const int32_t* max_lt_sq, const uint64_t* shell_count,
                              const uint64_t* shell_sum_q, uint32_t n, int ndim,
                              float* mean_lt, float* shell_mean_lt, float* sphericity,
                              float* roundness, hipStream_t s);

// Brackets one kernel launch with HIP events on its stream when the context's
// profiler is on (lt_profile_enable); the elapsed times are collected by
// lt_profile_read.
struct ProfScope {
    lt_ctx* ctx;
    hipStream_t s;
    const char* name;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(lt_ctx* c, hipStream_t st, const char* n) : ctx(c), s(st), name(n) {
        if (ctx && ctx->profile && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            (void)hipEventRecord(a, s);
        else
            a = b = nullptr;
    }
    ~ProfScope() {
        if (a && b) {
            (void)hipEventRecord(b, s);
            ctx->pending.push_back(PendingTiming{name, a, b});
        }
    }
};

// Grid extent along a looped dimension: enough blocks to fill the device about
// `per_cu` times over (each block then loops), never more than the dimension.
inline int loop_extent(int n_outer, long other_blocks, const lt_ctx* ctx, int per_cu = 16) {
    const long target = (long)ctx->n_cu * per_cu;
    long g = (target + other_blocks - 1) / (other_blocks > 0 ? other_blocks : 1);
    if (g > n_outer) g = n_outer;
    return g < 1 ? 1 : (int)g;
}

// Fixed-point scale of the deterministic radius sums (Q.23 in uint64).
constexpr double SUM_SCALE = 8388608.0;

// round(sqrt(v) * 2^23) for 0 <= v < 2^24, the per-voxel term of the radius sums
// (every kernel that forms it calls this, so the fused and separate sums agree bit
// for bit).  sqrt starts from the FP32 reciprocal square root (relative error about
// 2^-23) and takes two FP64 corrections y += (v - y^2) * h with h = rsq / 2: the
// error falls to about 2^-46, then below 2^-60, well inside an FP64 ulp.
__device__ __forceinline__ uint64_t radius_q23(int v) {
    const double x = (double)v;
    const float rf = __builtin_amdgcn_rsqf((float)(v > 0 ? v : 1));
    const double h = 0.5 * (double)rf;
    double y = x * (double)rf;
    y = fma(fma(-y, y, x), h, y);
    y = fma(fma(-y, y, x), h, y);
    return v > 0 ? (uint64_t)(y * SUM_SCALE + 0.5) : 0ull;
}

// ---------------------------------------------------------------- device helpers

// floor(sqrt(n)) for 0 <= n < 2^30, exact: float estimate then one-step fix-ups.
__device__ __forceinline__ int isqrt_floor(int n) {
    int r = (int)__fsqrt_rn((float)n);                 // r < 2^15: 24-bit products are exact
    if (__mul24(r, r) > n) --r;
    else if (__mul24(r + 1, r + 1) <= n) ++r;
    return r;
}

// Largest h with h*h < b, for b >= 1 (the reach of an open ball of squared radius b).
__device__ __forceinline__ int open_reach(int b) { return isqrt_floor(b - 1); }

// Largest h >= 0 with w h^2 < b, for 1 <= b < 2^24 and 1 <= w < 256: the reach of an
// open ball of squared radius b along an axis whose squared spacing is w.  The
// float estimate of sqrt((b - 1) / w) is within one of h; integer fix-ups make it
// exact.
__device__ __forceinline__ int open_reach_w(int b, int w) {
    int h = (int)__fsqrt_rn((float)(b - 1) / (float)w);
    if (w * h * h >= b) --h;
    else if (w * (h + 1) * (h + 1) < b) ++h;
    return h;
}

// Containment bound for squared radii beyond the prune tables: for the lattice ball
// of squared radius d (points with |q|^2 <= d - 1) and an offset of squared length
// k, max |q - o|^2 <= (sqrt(d - 1) + sqrt(k))^2 <= d - 1 + k + ceil(2 sqrt(k (d - 1))).
// A neighbour whose D exceeds this contains the ball, so dropping on it is exact
// (T[d] never exceeds the bound).  The product is taken in 64 bits: weighted 2D
// distances reach 2^24 with k up to 510.
__device__ __forceinline__ int prune_bound(int d, int k) {
    const long long s = 4ll * k * (d - 1);
    long long r = (long long)__dsqrt_rn((double)s);    // ceil(sqrt(s)), exact after fix-ups
    if (r * r > s) --r;
    else if ((r + 1) * (r + 1) <= s) ++r;
    if (r * r < s) ++r;
    return d - 1 + k + (int)r;
}

template <typename L>
__device__ __forceinline__ bool label_negative(L v) {
    if constexpr (sizeof(L) == 4 && L(-1) < L(0)) return v < 0;
    else return false;
}

// Per-block label table in LDS: open addressing with linear probing on the key
// (label, 0 = empty).  Returns the slot of `l`, inserting it, or -1 when the table
// is full (the caller then updates global memory directly).
template <int CAP>
__device__ __forceinline__ int lds_slot(uint32_t* keys, uint32_t l) {
    int h = (int)((l * 2654435761u) >> 7) & (CAP - 1);
    for (int probe = 0; probe < CAP; ++probe) {
        const uint32_t k = atomicCAS(&keys[h], 0u, l);
        if (k == 0u || k == l) return h;
        h = (h + 1) & (CAP - 1);
    }
    return -1;
}

// Empty bounding box of label l: bb layout [zmin, zmax, ymin, ymax, xmin, xmax][nlab].
__device__ __forceinline__ void init_box(int32_t* bb, uint32_t nlab, uint32_t l) {
    for (int k = 0; k < 3; ++k) {
        bb[(2 * k) * nlab + l] = 0x7fffffff;
        bb[(2 * k + 1) * nlab + l] = -1;
    }
}

}  // namespace lt
