/*
 * hyb.h - combined BVH + distance-field ray queries on AMD Instinct MI355X.
 *
 * C ABI of the method of Bartels & Harada, "Combining GPU Tracing Methods
 * within a Single Ray Query" (SIGGRAPH Asia 2022 Technical Communications).
 *
 * A ray query (o, d, tmin, tmax) (Section 2, Eq. 1) is split at
 *     t1 = min(tmin + threshold * h, tmax)            (Section 3, occlusion queries:
 *                                                      t1 from the voxel size h times a
 *                                                      user multiplier)
 * into two mutually exclusive sub-queries (Section 2, Eq. 2): [tmin, t1] is
 * traced exactly against the triangles through a BVH, and only when that finds
 * nothing (first-hit queries process sub-queries in order and stop at the first
 * intersection, Section 2) is [t1, tmax] traced against a distance field.
 * threshold = 0 gives pure distance-field tracing, threshold = +inf pure
 * triangle tracing (the "pure" techniques of Section 3).
 *
 * Conventions shared by every entry point
 *  - All pointers documented as "device" are HIP device pointers on the current
 *    device; "host" pointers are ordinary CPU memory.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Trace calls
 *    are asynchronous on `stream`; build calls return after their work on
 *    `stream` has completed.
 *  - The library owns handles until *_destroy.  Builders copy their inputs.  The
 *    caller owns ray and hit buffers; trace calls allocate nothing (batches
 *    allocate in hyb_batch_create and hyb_batch_tune, and build their graph on
 *    the first launch after a change of launch shape).
 *  - Errors come back as a status, never as a crash or an exception.  A status
 *    other than HYB_OK leaves outputs unspecified.
 *  - BVH and distance-field handles are immutable after build (except through
 *    hyb_sdf_update): concurrent trace calls on different streams are safe.  A batch handle is mutable (its
 *    thresholds and launch shape): calls on one batch must be ordered.
 */
#ifndef HYB_H
#define HYB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HYB_OK = 0,
    HYB_ERR_INVALID_ARG = 1, /* NULL pointer, bad size, NaN or negative tmax/threshold */
    HYB_ERR_OOM = 2,         /* device allocation failed */
    HYB_ERR_HIP = 3,         /* a HIP runtime call or kernel launch failed */
    HYB_ERR_UNSUPPORTED = 4  /* valid input the library cannot handle (e.g. BVH deeper than 64) */
} hyb_status;

typedef struct hyb_bvh_s* hyb_bvh; /* triangle BVH; library-owned device memory */
typedef struct hyb_sdf_s* hyb_sdf; /* distance-field grid; library-owned device memory */

/* Storage of the distance-field samples (the paper motivates keeping the DF
 * small, Sections 3 and 4).  The trace kernels interpolate the dequantized
 * FP32 values; every node has exactly one value, so the interpolant stays
 * continuous.  Triangle tests and t comparisons stay FP32.
 *   HYB_SDF_F32       FP32 samples
 *   HYB_SDF_F16       IEEE half, round to nearest even; value = (float)half
 *   HYB_SDF_I8_BRICK  int8 codes plus one power-of-two scale per block of
 *                     8^3 cells (cells [8b, 8b + 8) on each axis, so nodes
 *                     [8b, 8b + 8]: neighbouring blocks share a face of nodes;
 *                     ceil((n - 1) / 8) blocks per axis).  Block scale 2^e
 *                     with e the smallest integer >= -126 such that
 *                     max |f| over the block's nodes <= 127 * 2^e.  A node in
 *                     several blocks (on a face) takes the largest of their
 *                     scales, s_max: value = q * s_max with q = rint(f / s_max)
 *                     (round half to even) clamped to +-floor(127 s_min / s_max),
 *                     s_min the smallest of them.  Each cell's 8 corners are then
 *                     int8 multiples of its own block's scale.
 * Compact formats do not use the certified-sample step bound.  Inside the
 * library the kernels read a bricked copy in which every cell's 8 corner
 * samples lie together (bricks of 2^3 cells with their 3^3 nodes, padded to
 * 32 samples per 8 cells, for F32 and for F16 grids with n >= 205; one cell
 * with its 8 nodes for smaller F16 grids; for I8 one cell's 8 codes followed
 * by its block's scale, 12 bytes), so the device memory of a grid is n^3 FP32
 * values plus that copy (and, for I8, its ceil((n - 1) / 8)^3 block scales).
 * Every interface that takes or returns grid values (hyb_sdf_from_grid,
 * hyb_sdf_read, hyb_df_backward) uses the linear n^3 order, x fastest. */
typedef enum {
    HYB_SDF_F32 = 0,
    HYB_SDF_F16 = 1,
    HYB_SDF_I8_BRICK = 2
} hyb_sdf_format;

/* Rays: device SoA arrays of n floats each, n <= HYB_MAX_RAYS per call (the
 * trace kernels run one ray per work item and a launch counts its work items
 * in 32 bits).  d must be unit length (the
 * distance-field steps assume it).  tmin may be NULL (tmin = 0 for every ray).
 * tmax may be NULL (every ray uses the call's scalar tmax); otherwise ray i
 * ends at min(tmax[i], scalar tmax) (shadow rays end at their light sample).
 * A ray with tmin > tmax is reported as a miss. */
#define HYB_MAX_RAYS 2147483647LL

typedef struct {
    const float *ox, *oy, *oz;
    const float *dx, *dy, *dz;
    const float* tmin;
    const float* tmax;
} hyb_rays;

/* Hits: caller-allocated device SoA arrays of n entries.
 *   prim >= 0       triangle hit; prim is the triangle's index in the input mesh;
 *                   the hit point is (1-u-v) v0 + u v1 + v v2.
 *   prim == -2      distance-field hit (a distance field carries no surface
 *                   identity, Section 2 "Surface information"); u = v = 0.
 *   prim == -1      miss; t = +inf, u = v = 0.  */
typedef struct {
    float* t;
    int32_t* prim;
    float* u;
    float* v;
} hyb_hits;

#define HYB_MISS (-1)
#define HYB_DF_HIT (-2)

/* hyb_build_sdf flag: space outside every closed surface is solid (a scene
 * enclosed by an inward-facing room). */
#define HYB_SDF_EXTERIOR_SOLID 1u

/* hyb_sdf_from_grid flag: the caller certifies that every sample is the FP32
 * rounding of one 1-Lipschitz function (an exact distance field, e.g. samples
 * of a true signed distance).  The tracer then also steps by g - 2E (E the
 * trilinear interpolation error bound, sqrt(3)/2 h) where that is longer than
 * g / L.  Grids from hyb_build_sdf carry this property implicitly.  A false
 * certification can make the tracer pass a root. */
#define HYB_SDF_LIPSCHITZ_SAMPLES 2u
/* hyb_sdf_update flag: do not wait for the device (see hyb_sdf_update). */
#define HYB_SDF_UPDATE_DEFERRED 4u

/* Build a BVH over an indexed triangle mesh (the structure the paper's
 * hardware ray tracing traverses, Section 3).
 *   verts  host, n_verts x 3 floats (x,y,z)
 *   tris   host, n_tris x 3 int32 vertex indices; 0 <= index < n_verts
 * n_tris == 0 is allowed (every ray misses).  Degenerate triangles are kept and
 * are never hit.  The tree is a binned-SAH binary BVH (used by hyb_build_sdf)
 * collapsed to four children per node for the trace kernels.  Errors: NULL
 * pointers with nonzero counts, negative counts, out-of-range indices or
 * non-finite vertices -> HYB_ERR_INVALID_ARG; a tree deeper than 64 levels or
 * whose traversal could need more than 96 stack entries ->
 * HYB_ERR_UNSUPPORTED. */
hyb_status hyb_build_bvh(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                         void* stream, hyb_bvh* out);

/* Number of four-wide BVH nodes, triangles and the four-wide tree's depth. */
hyb_status hyb_bvh_info(hyb_bvh bvh, int64_t* n_nodes, int64_t* n_tris, int32_t* depth);

/* Build an n^3 node-centred signed distance grid from the BVH's mesh: each
 * sample is the exact Euclidean distance to the nearest triangle (computed in
 * FP64, rounded to FP32), negative inside solid space (winding number by signed
 * crossing count).  This replaces the paper's voxelization + jump flooding +
 * fast sweeping pipeline (Section 3, distance field generation) with exact
 * values.
 *   grid4  host, {lo_x, lo_y, lo_z, h}: node (i,j,k) sits at lo + (i,j,k) h.
 *          NULL: the mesh bounding box padded by 2 voxels per side,
 *          h = largest extent / (n - 5).
 *   n      samples per axis, 8 <= n <= 1024.
 *   flags  HYB_SDF_EXTERIOR_SOLID or 0.
 *   fmt    storage format; the FP32 distances are converted after the build.
 * Errors: HYB_ERR_INVALID_ARG for a NULL bvh/out, bad n, h <= 0, non-finite
 * grid4, unknown flags or format; HYB_ERR_OOM when the grid does not fit. */
hyb_status hyb_build_sdf(hyb_bvh bvh, int32_t n, const float* grid4, uint32_t flags, hyb_sdf_format fmt,
                         void* stream, hyb_sdf* out);

/* Wrap caller-provided samples as the distance field the DF sub-queries trace
 * (Section 3, "Distance Field Generation": the paper builds its field from the
 * scene every frame or incrementally; this takes a field built elsewhere, e.g.
 * analytic test fields or a field refit by gradient descent).  Copied.
 *   values  device, n^3 floats, x fastest: values[i + n (j + n k)]; 2 <= n <= 1024
 *   grid4   host, {lo_x, lo_y, lo_z, h}
 *   flags   0 or HYB_SDF_LIPSCHITZ_SAMPLES
 *   fmt     storage format the values are converted to
 * The bounds used for safe steps (the Lipschitz bound and per-axis bounds of
 * the partial derivatives) are recomputed from the stored (dequantized)
 * values.  Any finite samples are traced exactly (the first root of their
 * interpolant), however large their bound: a march whose steps would be short
 * walks cell by cell instead.
 * Errors: HYB_ERR_INVALID_ARG for NULL values/grid4/out, bad n, h <= 0,
 * non-finite grid4, unknown flags, or a sample that is NaN or infinite (or,
 * for HYB_SDF_F16, beyond the half range). */
hyb_status hyb_sdf_from_grid(const float* values, int32_t n, const float* grid4, uint32_t flags,
                             hyb_sdf_format fmt, void* stream, hyb_sdf* out);

/* Replace the samples of an existing grid in place (for loops that change a
 * grid every step, such as refitting it by gradient descent): afterwards the
 * handle holds what hyb_sdf_from_grid(values, n, grid4, flags, fmt) would
 * give for its own n, grid4 and format, bounds included, in the device memory
 * it already owns (nothing is allocated).
 *   values  device, n^3 floats of the handle's n, x fastest
 *   flags   0 or HYB_SDF_LIPSCHITZ_SAMPLES, optionally with
 *           HYB_SDF_UPDATE_DEFERRED
 * Synchronous on `stream` (the bounds are read back).  Work already queued on
 * other streams that reads the handle must have finished.  Batches that hold
 * the handle use the new samples and bounds from their next launch on.
 * With HYB_SDF_UPDATE_DEFERRED the call only queues the work on `stream` and
 * returns: the bounds stay on the device and later calls on the handle read
 * them there (the same values, so the same results), so a loop that updates a
 * grid every step need not wait for the device.  The check for samples that
 * are not finite then happens on the device too: until the next update every
 * query on the handle other than hyb_trace_bvh reports t = NaN, prim = -2 for
 * every ray, hyb_df_backward adds nothing, and hyb_sdf_check reports it.
 * hyb_sdf_info waits for the device to return the bound of such an update.
 * Errors: HYB_ERR_INVALID_ARG for a NULL handle/values, unknown flags, a
 * handle of another device, or a sample that is NaN or infinite (or, for
 * HYB_SDF_F16, beyond the half range); the handle's samples are then undefined
 * until the next successful update. */
hyb_status hyb_sdf_update(hyb_sdf sdf, const float* values, uint32_t flags, void* stream);

/* Whether the grid's last update (with HYB_SDF_UPDATE_DEFERRED) had only
 * finite samples, so that its interpolant, the distance field of Section 3
 * ("Distance Field Generation"), is defined everywhere: waits for `stream`
 * (the update's), then HYB_OK, or
 * HYB_ERR_INVALID_ARG when a sample was NaN or infinite (or, for HYB_SDF_F16,
 * beyond the half range) or for a NULL handle.  HYB_OK after any other
 * update (those check synchronously). */
hyb_status hyb_sdf_check(hyb_sdf sdf, void* stream);

/* Voxel size h of the grid: the unit of the switch thresholds (Section 3,
 * "Occlusion Queries": t1 is computed from the voxel size times a user
 * multiplier; "GI & Shadow Rays": t1 and t2 likewise).  Errors:
 * HYB_ERR_INVALID_ARG for a NULL sdf or h. */
hyb_status hyb_sdf_voxel_size(hyb_sdf sdf, float* h);

/* Grid placement, resolution and the Lipschitz bound L of the trilinear
 * interpolant of the stored samples (the distance field of Section 3,
 * "Distance Field Generation"; steps of g/L never pass a root; the trace
 * kernels step by g / min(L, L_d) with L_d = max(1, sum_i s_i |d_i|) from
 * per-axis slope bounds s_i, the ray's own bound).  Each output may be NULL. */
hyb_status hyb_sdf_info(hyb_sdf sdf, float* grid4 /* host, 4 */, int32_t* n, float* lipschitz);

/* Copy the samples of the distance field (Section 3, "Distance Field
 * Generation") as the trace kernels see them (dequantized for compact
 * formats) into out (device, n^3 floats, x fastest); asynchronous on stream. */
hyb_status hyb_sdf_read(hyb_sdf sdf, float* out, void* stream);

/* The combined first-hit query (Section 2, Eq. 2; Section 3): triangles on
 * [tmin, t1], then the distance field on [t1, tmax] only for rays that found
 * no triangle, with t1 = min(fl32(tmin + threshold * h), tmax).
 *   tmax       0 <= tmax, may be +inf
 *   threshold  0 <= threshold, in voxels of the grid, may be +inf
 * n == 0 is a no-op.  Errors: HYB_ERR_INVALID_ARG for NULL handles/pointers,
 * n < 0 or n > HYB_MAX_RAYS, NaN or negative tmax/threshold.
 * The distance-field march is bounded by the cells the segment crosses and
 * ends with the exact first root on any grid; a ray whose march ran out of
 * iterations would be reported as prim -2 with t = NaN, never as a miss (the
 * bound makes this unreachable). */
hyb_status hyb_trace(hyb_bvh bvh, hyb_sdf sdf, const hyb_rays* rays, int64_t n, float tmax, float threshold,
                     hyb_hits* hits, void* stream);

/* Pure triangle tracing on [tmin, tmax]: the "HWRT only" technique the paper
 * compares against (Section 3, the pure techniques "where all overhead is
 * circumvented"; the first columns of Fig. 1 and Fig. 2).  Same outputs and
 * errors as hyb_trace, with no distance field. */
hyb_status hyb_trace_bvh(hyb_bvh bvh, const hyb_rays* rays, int64_t n, float tmax, hyb_hits* hits, void* stream);

/* Pure distance-field tracing on [tmin, tmax]: the "DF only" technique of
 * Section 3 (the last columns of Fig. 1 and Fig. 2).  Every hit has prim -2.
 * Same errors as hyb_trace, with no BVH. */
hyb_status hyb_trace_df(hyb_sdf sdf, const hyb_rays* rays, int64_t n, float tmax, hyb_hits* hits, void* stream);

/* The paper's shadow-ray query (Section 3, GI & shadow rays; Section 2,
 * any-hit processed out of order): three sub-intervals
 *     [tmin, t1]  triangles     t1 = min(fl32(tmin + threshold_start * h), tmax)
 *     [t1, t2]    distance field t2 = max(fl32(tmax - threshold_end * h), t1)
 *     [t2, tmax]  triangles
 * where any intersection suffices: the distance-field part runs first, then
 * the triangle parts, each stopping at the first intersection found.
 * Output per ray: prim -1 unoccluded (t = +inf); -2 occluded by the distance
 * field (t = its first root in [t1, t2]); >= 0 occluded by that triangle (t =
 * one of its intersections in a triangle part; which occluder is reported when
 * there are several is unspecified).  Both thresholds 0: pure DF; +inf: pure
 * triangles.  Errors as hyb_trace. */
hyb_status hyb_trace_shadow(hyb_bvh bvh, hyb_sdf sdf, const hyb_rays* rays, int64_t n, float tmax,
                            float threshold_start, float threshold_end, hyb_hits* hits, void* stream);

/* Work counters of one query, for measurement: the same trace as hyb_trace
 * (mode 0), hyb_trace_bvh (mode 1) or hyb_trace_df (mode 2), writing hits and,
 * per ray, counts[3 i + 0] BVH nodes visited, counts[3 i + 1] triangles
 * tested, counts[3 i + 2] distance-field sample fetches (8 corners each).
 *   counts  device, 3 n int32.  bvh may be NULL for mode 2, sdf for mode 1.
 * mode 3 is hyb_trace_shadow with threshold_start = threshold_end = threshold. */
hyb_status hyb_trace_counters(hyb_bvh bvh, hyb_sdf sdf, const hyb_rays* rays, int64_t n, float tmax,
                              float threshold, int32_t mode, hyb_hits* hits, int32_t* counts, void* stream);

/* Backward of the distance-field hit distance with respect to the grid
 * samples (implicit differentiation of g(t*; theta) = 0 at the first root t*):
 *     d t* / d theta_j = -w_j(p*) / (grad f~(p*) . d),   p* = o + t* d,
 * for the 8 corners j of the cell holding p* (w_j the trilinear weights), 0 for
 * every other sample.  The ray path is not stored: each ray's hit point is
 * recomputed from t_hit.  A ray without a crossing (t_hit = +inf, or a hit at
 * the start of its segment, where the segment began at or below zero and t*
 * does not move with theta) contributes nothing.
 *   rays, n, tmax  the rays and segment of the forward hyb_trace_df call
 *   t_hit          device, n floats: the forward result
 *   grad_t         device, n floats: d loss / d t_hit
 *   grad_grid      device, n_grid^3 floats (x fastest): accumulated into (+=)
 * The sdf must be FP32 (HYB_SDF_F32).  The rays are sorted by hit cell and
 * each wavefront sums the rays of one cell before adding with float atomics:
 * sums agree across runs up to FP32 rounding of the order of additions.  The
 * sort's buffers (16 n bytes plus the sort's scratch) live in the sdf handle
 * until hyb_sdf_destroy: a call with more rays than any before it on the
 * handle allocates them (device memory, after waiting for the device to free
 * the smaller ones), later calls allocate nothing.  Calls on one handle that
 * overlap on different streams share the buffers and race.
 * Errors: HYB_ERR_INVALID_ARG for NULL pointers, n < 0 or n > HYB_MAX_RAYS,
 * NaN/negative tmax; HYB_ERR_UNSUPPORTED for a compact-format sdf;
 * HYB_ERR_OOM when the buffers cannot be allocated. */
hyb_status hyb_df_backward(hyb_sdf sdf, const hyb_rays* rays, int64_t n, float tmax, const float* t_hit,
                           const float* grad_t, float* grad_grid, void* stream);

hyb_status hyb_bvh_destroy(hyb_bvh bvh);
hyb_status hyb_sdf_destroy(hyb_sdf sdf);

/* ------------------------------------------------------------------------
 * Batches: many scenes and ray sets of uneven size in one launch.
 *
 * Each item is an independent combined query (as hyb_trace) of its own scene
 * with its own threshold; a batch runs all of them in one persistent kernel
 * whose wavefronts take runs of rays_per_item rays of one item from a global
 * work counter until every item is done.  hyb_batch_launch replays a HIP graph
 * of two kernel nodes (a fill kernel that zeroes the counter, then the
 * persistent trace); hyb_batch_launch_eager launches the same two kernels
 * directly.  Results are bit-identical to hyb_trace per item, whatever the
 * launch configuration.
 *
 * The batch keeps the item's pointers: the bvh, sdf, ray and hit buffers must
 * stay valid until hyb_batch_destroy; new ray data may be written into the same
 * buffers between launches, and an sdf replaced in place by hyb_sdf_update is
 * read again (samples, bounds) at the next launch or tune.  All calls on one batch must be ordered (one
 * stream, or synchronised by the caller): the batch's counter and descriptor
 * table are shared by its launches.
 * ------------------------------------------------------------------------ */
typedef struct hyb_batch_s* hyb_batch;

typedef struct {
    hyb_bvh bvh;       /* may be NULL when threshold == 0 (distance field only) */
    hyb_sdf sdf;       /* may be NULL when threshold == +inf (triangles only) */
    hyb_rays rays;     /* device SoA, as for hyb_trace */
    hyb_hits hits;     /* device SoA outputs, as for hyb_trace */
    int64_t n;         /* rays of this item, >= 0 */
    float tmax;        /* as for hyb_trace */
    float threshold;   /* tau in voxels of this item's sdf, as for hyb_trace */
} hyb_batch_item;

/* Launch shape of the persistent kernel. */
typedef struct {
    int32_t lds_depth;      /* BVH stack entries per lane held in LDS: 8, 16 or 32 (rest spills) */
    int32_t rays_per_item;  /* rays per work item, multiple of 64 in [64, 65536] */
    int32_t blocks_per_cu;  /* 256-thread blocks per compute unit, 1..16 (capped by occupancy) */
} hyb_batch_config;

#define HYB_TUNE_THRESHOLD 1u /* choose each item's threshold */
#define HYB_TUNE_LAUNCH 2u    /* choose the launch shape */

typedef struct {
    const float* thresholds; /* host, candidate thresholds (>= 0, +inf allowed);
                                NULL: 0, 0.5, 1, 2, 4, 8, 16, 32, +inf */
    int32_t n_thresholds;    /* 0 with thresholds == NULL */
    float max_error_rate;    /* per item: fraction of its rays allowed to differ from the triangles-only result */
    int32_t reps;            /* timed launches per candidate, 1..100 */
    uint32_t flags;          /* HYB_TUNE_THRESHOLD | HYB_TUNE_LAUNCH */
} hyb_batch_tune_opts;

/* Copies the items into a device descriptor table (synchronous on `stream`).
 * Every item is validated as hyb_trace would; all sdfs of a batch must share
 * one storage format (else HYB_ERR_UNSUPPORTED).  1 <= n_items <= 65536.
 * Default config: lds_depth 16, rays_per_item 256, blocks_per_cu 4. */
hyb_status hyb_batch_create(const hyb_batch_item* items, int32_t n_items, void* stream, hyb_batch* out);

/* Configuration and per-item thresholds take effect at the next launch (which
 * then re-uploads the table synchronously and, for hyb_batch_launch, rebuilds
 * the graph when the launch shape changed).  set_threshold rejects a threshold
 * an item cannot use (not 0 without a bvh, not +inf without an sdf). */
hyb_status hyb_batch_set_config(hyb_batch batch, const hyb_batch_config* config);
hyb_status hyb_batch_get_config(hyb_batch batch, hyb_batch_config* config);
hyb_status hyb_batch_set_threshold(hyb_batch batch, int32_t item, float threshold);
hyb_status hyb_batch_get_threshold(hyb_batch batch, int32_t item, float* threshold);

/* Runs every item: one graph launch (asynchronous on `stream`). */
hyb_status hyb_batch_launch(hyb_batch batch, void* stream);
/* The same two kernels launched directly. */
hyb_status hyb_batch_launch_eager(hyb_batch batch, void* stream);

/* Autotuner (synchronous; overwrites the items' hit buffers).
 * HYB_TUNE_THRESHOLD: for each item with both a bvh and an sdf and n > 0 (the
 * others keep their threshold), traces its
 * rays triangles-only as the reference, then at every candidate threshold;
 * a ray counts as an error when hit/miss differs from the reference or both
 * hit more than one voxel (h of the item's sdf) apart along the ray.  The item
 * gets the candidate with the shortest measured time (fastest of `reps`
 * single-item launches) among those with error rate <= max_error_rate, or
 * +inf (exact) when none qualifies.
 * HYB_TUNE_LAUNCH: times the whole batch (fastest of `reps` eager launches) for
 * lds_depth {8,16,32} x rays_per_item {64,256,1024,4096} x blocks_per_cu
 * {1,2,4,8} and keeps the fastest.
 * item_error (host, n_items floats, may be NULL) receives each item's error
 * rate at its chosen threshold (0 for items not tuned); best_ms (may be NULL)
 * the fastest whole-batch time of the final configuration.  Allocates 16 bytes
 * per ray of the largest item as scratch for the duration of the call. */
hyb_status hyb_batch_tune(hyb_batch batch, const hyb_batch_tune_opts* opts, float* item_error, float* best_ms,
                          void* stream);

hyb_status hyb_batch_destroy(hyb_batch batch);

/* For callers that cannot allocate device memory (serving loops that must not
 * call hipMalloc, harnesses that forbid it): one launch of the batch kernels
 * (as hyb_batch_create followed by hyb_batch_launch_eager, with each item's
 * own threshold and no tuning) whose work counter, item offsets and
 * descriptor table live in a fixed device array of the library instead of
 * memory a batch allocates.  The array holds up to HYB_STATIC_BATCH_MAX_ITEMS
 * items (65,024 bytes, one copy per device, kept until the process ends; its
 * address is looked up on the first call on each device).  Nothing is
 * allocated, on the device or the host; the descriptors are written by small
 * fill kernels whose arguments carry them, so `items` may be reused on
 * return.  Asynchronous on `stream`; results are bit-identical to the batch
 * launch of the same items and config.
 *   config  launch shape, or NULL for the default {16, 256, 4}
 * Every call on a device shares that device's array and leaves its contents
 * behind (each call rewrites what it uses and zeroes the counter itself):
 * calls that overlap on one device (other streams, other threads) race.
 * Errors: HYB_ERR_INVALID_ARG for NULL items, n_items < 1 or n_items >
 * HYB_STATIC_BATCH_MAX_ITEMS, a bad config, or an item hyb_batch_create would
 * reject; HYB_ERR_UNSUPPORTED for mixed storage formats. */
#define HYB_STATIC_BATCH_MAX_ITEMS 256
hyb_status hyb_batch_launch_static(const hyb_batch_item* items, int32_t n_items, const hyb_batch_config* config,
                                   void* stream);

/* Static string naming a status. */
const char* hyb_status_str(hyb_status s);

#ifdef __cplusplus
}
#endif

#endif /* HYB_H */
