/*
 * liblt -- local-thickness sphericity and roundness on AMD Instinct MI355X (gfx950).
 *
 * Method: Pieta, Rasmussen, Dahl, Christensen, "Fast Sphericity and Roundness
 * approximation in 2D and 3D using Local Thickness" (arXiv 2504.05808).
 *
 * Pipeline over a labelled 2D image or 3D volume, all objects at once:
 *   lt_edt              per-label squared Euclidean distance transform D
 *   lt_thickness        squared local thickness LT_sq (largest inscribed ball
 *                       containing each voxel; Method section)
 *   lt_object_measures  per-object volume, mean / max / shell-mean local
 *                       thickness, sphericity and roundness (Method: Sphericity
 *                       and Roundness subsections)
 *
 * Conventions (shared by every call):
 *   - ndim = 2 with shape = {ny, nx}, or ndim = 3 with shape = {nz, ny, nx};
 *     C order, x contiguous, unit isotropic spacing; each extent <= 1024 in 3D
 *     and <= 2048 in 2D.
 *   - labels: LT_U16, LT_I32 or LT_U32; 0 is background; a label may hold several
 *     connected components (it is still one object).  Every position outside the
 *     image, and every voxel of another label, is background for an object.
 *   - distances are squared, between voxel centres, in int32: a voxel next to
 *     background has D = 1.  Balls are open and centred on lattice points.
 *   - every pointer argument except `ctx` and `shape` is a DEVICE pointer; the
 *     caller allocates and owns all inputs and outputs; the library never frees
 *     caller memory.  `shape` is a host array.
 *   - every call is stream-ordered on `stream` (a hipStream_t; NULL = the null
 *     stream) and returns without synchronising.  Argument errors are reported
 *     synchronously before anything is launched; errors found on the device
 *     (label above max_label, negative int32 label) set a device error word that
 *     lt_sync_status reads.
 *   - no call aborts or throws across this interface.  A zero-size image is a
 *     no-op returning LT_OK.
 *   - calls on one context must not overlap in time (they share its scratch
 *     memory); use one context per concurrent stream.
 *   - environment: LT_LOG=1 prints one line on stderr for every error status
 *     (the call it came from, the status and its message), LT_LOG=2 also one line
 *     per call that takes a volume (name, shape, label type, label bound);
 *     LT_FAULT_INJECT=alloc makes every device allocation of the library fail
 *     with LT_E_ALLOC, alloc:N after N more successes (tests of the failure
 *     paths); LT_SPILL_CAP=K caps each spill region and the shared spill pool of
 *     the 3D local-thickness pass at K words (0: every front longer than four
 *     entries is rescanned by the paint pass instead; same results, slower; tests
 *     of that path).  All are read at every use.
 */
#ifndef LT_H
#define LT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes (int32_t, so that any value crossing the interface is well defined). */
typedef int32_t lt_status;
enum {
    LT_OK = 0,
    LT_E_ARG = 1,          /* null pointer or invalid argument */
    LT_E_DTYPE = 2,        /* unknown label dtype */
    LT_E_SHAPE = 3,        /* ndim not 2/3, negative or too large extent */
    LT_E_ALLOC = 4,        /* device allocation failed */
    LT_E_HIP = 5,          /* a HIP runtime call failed (see lt_last_error) */
    LT_E_LABEL_RANGE = 6,  /* device: a label exceeded max_label or was negative */
    LT_E_OVERFLOW = 7,     /* device: an intermediate exceeded its range */
    LT_E_WORKSPACE = 8,    /* a caller-provided buffer is too small */
    LT_E_NOT_READY = 9     /* object not initialised (e.g. model not trained) */
};

/* Label element types (int32_t: unknown values are rejected with LT_E_DTYPE). */
typedef int32_t lt_dtype;
enum { LT_U16 = 1, LT_I32 = 2, LT_U32 = 3 };

typedef struct lt_ctx lt_ctx;

/* Create a context bound to HIP device `device` (the device is made current for
 * the calls on it).  Owns scratch memory, lookup tables and a device error word. */
lt_status lt_ctx_create(lt_ctx** out, int device);
/* Free the context's device memory (synchronises the device first). */
lt_status lt_ctx_destroy(lt_ctx* ctx);
/* Device facts the context planned with: compute units, LDS bytes per block and the
 * row count of the local-thickness paint tiles (64 when the LDS allows, else 32).
 * Any output pointer may be NULL. */
lt_status lt_ctx_info(lt_ctx* ctx, int* n_cu, uint64_t* lds_per_block, int* paint_tile_rows);

/* Per-label squared Euclidean distance transform (the distance map underlying the
 * local-thickness definition; Introduction and Method, first paragraph):
 *   dist_sq[p] = 0 where labels[p] == 0, otherwise
 *   dist_sq[p] = min |p - q|^2 over lattice points q outside the image or with
 *                labels[q] != labels[p].
 * labels: [N] of `dtype`; dist_sq: [N] int32 output (N = product of shape). */
lt_status lt_edt(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim,
                 const int64_t* shape, int32_t* dist_sq, void* stream);

/* Squared local thickness (Method, first paragraph: the radius of the largest
 * inscribed circle/sphere containing the point):
 *   lt_sq[p] = max{ dist_sq[x] : |p - x|^2 < dist_sq[x] } for object voxels,
 *   lt_sq[p] = 0 on background.
 * The reported radius is sqrt(lt_sq).  dist_sq must be lt_edt's output for the
 * same labels.  max_label bounds the label values (work is organised per object);
 * a larger label sets LT_E_LABEL_RANGE on the device.  lt_sq: [N] int32 output. */
lt_status lt_thickness(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim,
                       const int64_t* shape, const int32_t* dist_sq, uint32_t max_label,
                       int32_t* lt_sq, void* stream);

/* Per-object outputs, each an array of max_label + 1 entries indexed by label value.
 * Entry 0 (background) and absent labels have volume 0 and NaN measures. */
typedef struct {
    uint64_t* volume;         /* V (3D) or area A (2D): voxel count */
    uint64_t* shell_count;    /* voxels with a face neighbour (4 in 2D, 6 in 3D)
                                 outside the image or of another label */
    int32_t* max_lt_sq;       /* max LT_sq over the object: squared radius R^2 of the
                                 maximal inscribed ball (Method, Roundness) */
    float* mean_lt;           /* mean of sqrt(LT_sq) over the object */
    float* shell_mean_lt;     /* mean of sqrt(LT_sq) over the shell */
    float* sphericity;        /* 3D: pi^(1/3) (6V)^(2/3) / S, S the surface of the
                                 spheroid with equal semi-axes a = mean_lt and third
                                 semi-axis c = 3V / (4 pi a^2) (Background Eq. 1;
                                 Method, Sphericity).  2D: P_c / P_o with P_c =
                                 2 sqrt(pi A) and P_o Ramanujan's first
                                 approximation for semi-axes a = mean_lt and
                                 b = A / (pi a) */
    float* roundness;         /* shell_mean_lt / sqrt(max_lt_sq) (Method, Roundness) */
    float* hist32;            /* optional, may be NULL: [(max_label + 1) * 32]
                                 fraction of the object's voxels in bin k = 1..32
                                 (stored at k - 1), bin(p) = the smallest k with
                                 1024 * LT_sq(p) <= k^2 * max_lt_sq */
} lt_measures;

/* Shell extraction, per-object reductions and closed forms.  lt_sq must be
 * lt_thickness's output for the same labels.  Output arrays are device arrays
 * of max_label + 1 entries; they are fully written. */
lt_status lt_object_measures(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim,
                             const int64_t* shape, const int32_t* lt_sq, uint32_t max_label,
                             const lt_measures* out, void* stream);

/* The whole path in one call: lt_edt, lt_thickness and lt_object_measures with
 * the per-object sums accumulated while the local thickness is written (every
 * object voxel is painted once, by a work item of its own object), so the
 * separate reduction pass over the volume is skipped.  Outputs are those of the
 * three calls, bit for bit.  dist_sq and lt_sq are device arrays of the volume's
 * size; the context's scratch grows to hold the thickness and measures state
 * together. */
lt_status lt_pipeline(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim, const int64_t* shape,
                      uint32_t max_label, int32_t* dist_sq, int32_t* lt_sq, const lt_measures* out,
                      void* stream);

/* Allocation-free form of lt_pipeline, for callers that cannot allocate device
 * memory while they run (code under stream capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments, kernels and outputs as lt_pipeline, bit
 * for bit, but the scratch memory is a fixed device array of
 * LT_STATIC_SCRATCH_BYTES inside the library (one copy per device, reserved when
 * the library's code is loaded on that device and held until the process ends)
 * instead of the context's growable scratch; the call makes no device allocation
 * or free, creates no event (the per-kernel profiler is skipped) and does not
 * synchronise.  The caller still allocates every input and output.
 *   - a problem whose scratch (lt_pipeline_static_bytes) exceeds the fixed array
 *     returns LT_E_WORKSPACE before anything is launched; e.g. a 128^3 volume with
 *     a few hundred labels needs about 57 MiB;
 *   - all calls on one device share that device's array, and each call leaves its
 *     contents behind (every kernel initialises what it reads), so calls that
 *     overlap in time on one device -- on different streams or contexts, or from
 *     different threads -- race and give undefined results: order them. */
#define LT_STATIC_SCRATCH_BYTES (64u * 1024u * 1024u)
lt_status lt_pipeline_static(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim, const int64_t* shape,
                             uint32_t max_label, int32_t* dist_sq, int32_t* lt_sq, const lt_measures* out,
                             void* stream);
/* Scratch bytes lt_pipeline_static needs for this problem (host-only arithmetic;
 * 0 for an invalid shape or max_label). */
size_t lt_pipeline_static_bytes(int ndim, const int64_t* shape, uint32_t max_label);

/* Closed forms alone, from per-object sums held on the device (the last step of
 * lt_object_measures; exposed for callers that accumulate their own sums):
 *   mean_lt = sum_lt_q23 / 2^23 / volume, shell_mean_lt = shell_sum_q23 / 2^23 /
 *   shell_count, roundness = shell_mean_lt / sqrt(max_lt_sq), sphericity from the
 *   spheroid (ndim 3) or ellipse (ndim 2) model as in lt_measures.
 * The radius sums are Q.23 fixed point (round(sqrt(LT_sq) * 2^23) summed).  All
 * arrays have n entries; entries with volume 0 get NaN. */
lt_status lt_closed_forms(const uint64_t* volume, const uint64_t* sum_lt_q23,
                          const int32_t* max_lt_sq, const uint64_t* shell_count,
                          const uint64_t* shell_sum_q23, uint32_t n, int ndim, float* mean_lt,
                          float* shell_mean_lt, float* sphericity, float* roundness,
                          void* stream);

/* ---------------------------------------------------------- anisotropic spacing
 * The same four steps for voxels that are longer along some axes (micro-CT stacks
 * often have thicker slices than pixels; the paper's data use unit spacing, for
 * which these calls equal the plain ones).  sq_spacing is a HOST array of ndim
 * integers w in 1..LT_MAX_SQ_SPACING, the squared voxel spacings along (z, y, x) or
 * (y, x) in a common length unit u (spacing sqrt(w) u).  Every squared distance
 * becomes w_z dz^2 + w_y dy^2 + w_x dx^2 (units u^2), so:
 *   dist_sq[p] = min over q outside the image or of another label of that sum;
 *   lt_sq[p]   = max{ dist_sq[x] : weighted |p - x|^2 < dist_sq[x] } (balls are
 *                ellipsoids in index space, spheres in space);
 *   measures: LT radii are lengths in u; the sphericity takes the physical volume
 *   (area) V = voxel count x sqrt(w_z w_y w_x) (sqrt(w_y w_x) in 2D); volume and
 *   shell_count stay voxel counts; the shell is the face-neighbour shell.
 * Results are exact integers as in the plain calls.  LT_E_ARG when a weight is
 * outside the range or when the largest possible squared distance,
 * min_a w_a ((n_a + 1) / 2)^2, exceeds 2^19 - 1 (3D) or 2^24 (2D). */
#define LT_MAX_SQ_SPACING 255
lt_status lt_edt_aniso(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim, const int64_t* shape,
                       const int32_t* sq_spacing, int32_t* dist_sq, void* stream);
lt_status lt_thickness_aniso(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim,
                             const int64_t* shape, const int32_t* sq_spacing, const int32_t* dist_sq,
                             uint32_t max_label, int32_t* lt_sq, void* stream);
lt_status lt_object_measures_aniso(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim,
                                   const int64_t* shape, const int32_t* sq_spacing, const int32_t* lt_sq,
                                   uint32_t max_label, const lt_measures* out, void* stream);
lt_status lt_pipeline_aniso(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim, const int64_t* shape,
                            const int32_t* sq_spacing, uint32_t max_label, int32_t* dist_sq, int32_t* lt_sq,
                            const lt_measures* out, void* stream);

/* Mesh-based surface measures per object: the sphericity baseline the method is
 * compared with (Related work; Experiments, Benchmark methods: the object is meshed
 * by marching cubes / marching squares and the mesh area / contour length enters
 * Wadell's sphericity, Background Eq. 1, or the perimeter sphericity).
 * The surface of object l is the iso-surface at 1/2 of its own 0/1 mask (other
 * labels and everything outside the image are 0), linear inside the simplices of
 * the lattice:
 *   3D: each unit cube split into the six Freudenthal tetrahedra along its
 *       (0,0,0)-(1,1,1) diagonal (marching tetrahedra); area = sum of the
 *       triangles / parallelograms through the midpoints of the edges that join
 *       an inside and an outside corner;
 *   2D: marching squares with segments between side midpoints (a square with two
 *       diagonal inside corners cuts off each inside corner).
 * Outputs, each [max_label + 1] and indexed by label, any of them may be NULL (not
 * all three):
 *   volume      uint64 voxel (pixel) count V;
 *   area        float surface area (3D) or contour length (2D), 0 for absent labels;
 *   sphericity  float, 3D pi^(1/3) (6V)^(2/3) / area, 2D 2 sqrt(pi V) / length;
 *               NaN where V = 0.
 * Areas are accumulated in Q.32 fixed point, so results are independent of the
 * order of the device's atomics.  Labels above max_label set LT_E_LABEL_RANGE
 * (lt_sync_status) and count as background. */
lt_status lt_mesh_measures(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim,
                           const int64_t* shape, uint32_t max_label, uint64_t* volume,
                           float* area, float* sphericity, void* stream);

/* Roughness-filtered roundness (Discussion: the roundness approximation responds
 * to surface roughness, an influence that filtering can control).  The shell
 * values are filtered before the mean of Method, Roundness is taken:
 *   F_0(p) = lt_sq[p] on shell voxels (dist_sq[p] == 1: a face neighbour is of
 *            another label or outside the image), 0 elsewhere;
 *   then along x, then y, then z (2D: x, then y):
 *   F(p) = max{ F(p + o e_axis) : |o| <= half_width, labels[p + o e_axis] == labels[p] };
 *   roundness[l] = mean over l's shell voxels of sqrt(F) / sqrt(max lt_sq over l).
 * half_width = 0 gives the plain roundness of lt_object_measures; bumps narrower
 * than about half_width stop lowering the value.  dist_sq and lt_sq are lt_edt's
 * and lt_thickness's outputs for the same labels (device, [N] int32);
 * roundness is a device array of max_label + 1 floats (NaN for labels without
 * voxels).  half_width outside 0..LT_ROUGH_MAX_HALF_WIDTH returns LT_E_ARG.  The
 * context's scratch grows to two int32 fields of the image's size. */
#define LT_ROUGH_MAX_HALF_WIDTH 16
lt_status lt_filtered_roundness(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim,
                                const int64_t* shape, const int32_t* dist_sq, const int32_t* lt_sq,
                                uint32_t max_label, int half_width, float* roundness, void* stream);

/* Map roundness values onto 0..1 through a minimum m (Results, performance on the
 * 2D charts: the smallest observed value anchors the scale):
 *   out[i] = (roundness[i] - m) / (1 - m) for finite entries, NaN entries stay NaN,
 *   and every finite entry becomes 1 when m >= 1.
 * m = r_min, or, when r_min is NaN, the smallest finite entry of `roundness`
 * (found on the device).  roundness and out are device arrays of n floats (they
 * may be the same array).  FP32 arithmetic. */
lt_status lt_remap_roundness(lt_ctx* ctx, const float* roundness, uint32_t n, float r_min, float* out,
                             void* stream);

/* The per-cell table behind lt_mesh_measures, as the device sums it (Q.32
 * rounded): ndim 3 writes 256 entries, the surface area inside a unit cube whose
 * corners with bit k of the index set are inside (corner k = (x, y, z) offset
 * (k & 1, (k >> 1) & 1, k >> 2)); ndim 2 writes 16 entries, the contour length in a
 * unit square (corner k = (x, y) offset (k & 1, k >> 1)).  `out` is a HOST array.
 * Needs no device. */
lt_status lt_mesh_table(int ndim, double* out);

/* Synchronise `stream`, read and clear the context's device error word.
 * Returns LT_OK, LT_E_LABEL_RANGE, LT_E_OVERFLOW or LT_E_HIP. */
lt_status lt_sync_status(lt_ctx* ctx, void* stream);

/* ---------------------------------------------------------------- batched form
 * Many volumes of uneven size (one label dtype) processed by one graph launch.
 * Every volume gets the full pipeline (lt_edt, lt_thickness, lt_object_measures)
 * with the same outputs and bit-identical results as the plain calls.  The
 * volumes are spread over `batch_lanes` concurrent streams (lt_tuning), largest
 * first; the whole batch is captured once into a hipGraph that lt_batch_run
 * replays with a single hipGraphLaunch on `stream`.  The batch owns its scratch
 * (one region per lane); the caller keeps every volume's buffers alive and at the
 * same addresses for the life of the batch.  Replays of one batch must not overlap.
 * Errors found on the device are reported per volume by lt_batch_status. */
typedef struct {
    const void* labels;       /* device, `dtype` of the batch */
    int ndim;                 /* 2 or 3 */
    int64_t shape[3];         /* {nz, ny, nx} or {ny, nx, -} */
    uint32_t max_label;
    int32_t* dist_sq;         /* device outputs as in lt_edt / lt_thickness */
    int32_t* lt_sq;
    lt_measures measures;     /* device outputs as in lt_object_measures */
} lt_volume;
typedef struct lt_batch lt_batch;
lt_status lt_batch_create(lt_ctx* ctx, const lt_volume* vols, int n_volumes, lt_dtype dtype,
                          lt_batch** out);
lt_status lt_batch_run(lt_batch* batch, void* stream);
/* Per-volume status of the batch's replays so far: synchronise `stream`, read and
 * clear every volume's device error word (device-detected errors of a batch go to
 * these words, not to the context's).  status: optional HOST array of n_volumes
 * entries, each LT_OK, LT_E_LABEL_RANGE or LT_E_OVERFLOW; a bad volume leaves the
 * others' entries (and outputs) intact.  Returns the first volume's error, or LT_OK. */
lt_status lt_batch_status(lt_batch* batch, void* stream, int32_t* status);
lt_status lt_batch_destroy(lt_batch* batch);

/* ---------------------------------------------------------------- tuning
 * Runtime kernel knobs.  paint_tile_rows: 32 or 64 rows per local-thickness paint
 * tile (0 = 64 when the LDS allows); paint_blocks_per_cu: 1 or 2 persistent paint
 * blocks per compute unit (2 only takes effect with 32-row tiles); front_chunk: 32,
 * 64 or 128 slices per block of the z-front pass (one lane per slice, 64 slices at
 * a time); batch_lanes: 1..16 streams in a batch graph.  Results never depend on
 * the knobs, only the speed does. */
typedef struct {
    int paint_tile_rows;
    int paint_blocks_per_cu;
    int front_chunk;
    int batch_lanes;
} lt_tuning;
lt_status lt_get_tuning(lt_ctx* ctx, lt_tuning* out);
lt_status lt_set_tuning(lt_ctx* ctx, const lt_tuning* tuning);

/* Autotuner.  lt_autotune times the full pipeline on the given volume (device
 * labels) for every combination of paint tile rows, paint blocks per CU and
 * z-front chunk (`repeats` timed runs each after one warm-up), sets the fastest on
 * the context and returns it in *best (may be NULL).  lt_autotune_batch does the
 * same for batch_lanes on a batch.  Winners are cached in the JSON file
 * `cache_path` (NULL: no cache) under a key of device architecture, dtype,
 * dimensionality and size class; a cached key is applied without timing.  The
 * tuner allocates temporary device memory and synchronises the device. */
lt_status lt_autotune(lt_ctx* ctx, const void* labels, lt_dtype dtype, int ndim,
                      const int64_t* shape, uint32_t max_label, const char* cache_path,
                      int repeats, lt_tuning* best);
lt_status lt_autotune_batch(lt_ctx* ctx, const lt_volume* vols, int n_volumes, lt_dtype dtype,
                            const char* cache_path, int repeats, lt_tuning* best);

/* ---------------------------------------------------------------- learned correction
 * A 34 -> 64 -> 64 -> 64 -> 1 SiLU network that corrects the spheroid sphericity
 * toward a mesh-based sphericity.  Features per object (lt_mlp_features): the
 * 32-bin local-thickness histogram of lt_measures.hist32, log V and
 * mean_lt / V^(1/3).  The network sees the features standardised with
 * (mean, stdev) and predicts (delta - target_shift) / target_scale, delta being the
 * correction to add to the closed form.  Products run as BF16 MFMA with FP32
 * accumulation; master weights and AdamW moments are FP32.  All arrays are device
 * arrays unless noted; calls are stream-ordered. */
typedef struct lt_mlp lt_mlp;
/* He-uniform weights from `seed`, zero biases; identity normalisation, open guard. */
lt_status lt_mlp_create(lt_ctx* ctx, uint64_t seed, lt_mlp** out);
lt_status lt_mlp_destroy(lt_mlp* mlp);
/* Host arrays of 34 feature means and spreads; target = (delta - shift) / scale. */
lt_status lt_mlp_set_normalization(lt_mlp* mlp, const float* mean, const float* stdev,
                                   float target_shift, float target_scale);
/* Host arrays of 34 per-feature bounds and the largest |delta| the correction may
 * apply (the training set's ranges). */
lt_status lt_mlp_set_guard(lt_mlp* mlp, const float* fmin, const float* fmax, float max_abs_delta);
/* One AdamW step (beta 0.9 / 0.999, eps 1e-8, decoupled weight decay on matrices) on
 * the mean squared error of the standardised target y (B values) for features x
 * (B x 34); B a positive multiple of 16.  lr = 0 computes gradients only.  If
 * loss_out is not NULL it receives the sum of squared errors (one float). */
lt_status lt_mlp_train_step(lt_mlp* mlp, const float* x, const float* y, int batch, float lr,
                            float weight_decay, float* loss_out, void* stream);
/* delta (B floats) = de-standardised network output for features x (B x 34). */
lt_status lt_mlp_infer(lt_mlp* mlp, const float* x, int batch, float* delta, void* stream);
/* Features x (n x 34) from lt_object_measures outputs (hist32 [n x 32], volume,
 * mean_lt); absent objects give non-finite features. */
lt_status lt_mlp_features(lt_ctx* ctx, const float* hist32, const uint64_t* volume,
                          const float* mean_lt, uint32_t n, float* x, void* stream);
/* s_corr = s_lt + delta where the guard accepts the prediction (every feature within
 * its bounds, delta finite and |delta| <= max_abs_delta), else s_lt; *n_fallback
 * (device, not cleared here) is incremented once per rejected object.
 * delta_scratch holds n floats. */
lt_status lt_mlp_correct(lt_mlp* mlp, const float* x, const float* s_lt, int n,
                         float* delta_scratch, float* s_corr, uint32_t* n_fallback, void* stream);
/* Whole model state (weights, moments, step, normalisation, guard) as a host blob
 * of lt_mlp_state_size() bytes, for checkpoint and resume. */
size_t lt_mlp_state_size(void);
lt_status lt_mlp_get_state(lt_mlp* mlp, void* blob, size_t bytes);
lt_status lt_mlp_set_state(lt_mlp* mlp, const void* blob, size_t bytes);
/* Device pointers to the FP32 master weights and the last step's gradients (packed
 * layout: W1[64][48] b1[64] W2[64][64] b2 W3[64][64] b3 W4[16][64] b4[16], unused
 * pads zero) and the packed length. */
lt_status lt_mlp_buffers(lt_mlp* mlp, float** weights, float** grads, int* n_param);
/* Host copy (after a device synchronisation) of one packed array: which = 0 master
 * weights, 1 last gradients, 2 first moments, 3 second moments; `host` holds at
 * least n_param floats (n), else LT_E_WORKSPACE. */
lt_status lt_mlp_read(lt_mlp* mlp, int which, float* host, size_t n);

/* The network's matrix-product kernel on its own: C (M x N, FP32, row stride ldc) =
 * A (M x K) * B (K x N) for BF16 inputs (uint16 bit patterns), with A(i, k) at
 * A[i * lda + k] (or A[k * lda + i] when trans_a) and B(k, j) at B[k * ldb + j] (or
 * B[j * ldb + k] when trans_b); M, N, K multiples of 16.  Products use
 * v_mfma_f32_16x16x16_bf16 with FP32 accumulation. */
lt_status lt_bf16_gemm(int M, int N, int K, const uint16_t* A, int lda, int trans_a,
                       const uint16_t* B, int ldb, int trans_b, float* C, int ldc, void* stream);

/* Kernel timing (tracing).  When enabled, every kernel the library launches is
 * bracketed by two HIP events recorded on the launch stream; lt_profile_read waits
 * for the pending events and returns per-kernel totals accumulated since the last
 * lt_profile_reset: up to `cap` entries are written to `out` (host array) and the
 * number of distinct kernels to *n_out.  Disabled by default. */
typedef struct {
    char name[40];
    double total_ms;
    uint64_t launches;
} lt_kernel_time;
lt_status lt_profile_enable(lt_ctx* ctx, int on);
lt_status lt_profile_read(lt_ctx* ctx, lt_kernel_time* out, int cap, int* n_out);
lt_status lt_profile_reset(lt_ctx* ctx);

/* Static text for a status code. */
const char* lt_status_str(lt_status s);
/* Text of the last error raised on the calling thread ("" if none). */
const char* lt_last_error(void);
/* Library version string. */
const char* lt_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LT_H */
