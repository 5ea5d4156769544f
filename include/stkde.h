/*
 * stkde.h -- C ABI of the MI355X (gfx950) space-time kernel density library.
 *
 * The library computes the space-time kernel density estimate of Saule et
 * al., "Parallel Space-Time Kernel Density Estimation" (arXiv 1705.09366),
 * Sec. 2.1 (estimator, kernels, voxelisation), by the point-based,
 * symmetry-exploiting method PB-SYM of Sec. 3.2, re-organised as an
 * atomic-free gather over output tiles on the GPU:
 *
 *   f[X][Y][T] = 1/(n hs^2 ht) * sum_i ks(u, v) * kt(w),
 *   u = (x_X - x_i)/hs,  v = (y_Y - y_i)/hs,  w = (t_T - t_i)/ht,
 *   ks(u,v) = (2/pi)(1 - u^2 - v^2) on u^2 + v^2 < 1,  kt(w) = (3/4)(1 - w^2) on |w| <= 1,
 *
 * where (x_X, y_Y, t_T) = (x0 + (X+1/2) sres, y0 + (Y+1/2) sres, t0 + (T+1/2) tres)
 * is the centre of voxel (X, Y, T).  The kernel formulas printed in Sec. 2.1
 * are garbled; the Epanechnikov pair above (unit integrals) is the reading
 * this library implements.
 *
 * Conventions shared by every entry point:
 *  - Plain C types only.  Device pointers are HIP device allocations (for
 *    example torch CUDA tensors on ROCm); host pointers are ordinary memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued asynchronously on it; no entry point synchronises the
 *    device on the success path.
 *  - Every argument is validated on the host before anything is enqueued.
 *    On an error nothing is enqueued and no output is touched.
 *  - Errors are reported as stkde_status values; nothing throws or aborts
 *    across this interface.  An asynchronous HIP failure of earlier work is
 *    reported as STKDE_ERR_HIP by a later call that checks HIP's error state.
 *  - The caller owns every buffer.  A plan owns only host metadata; it is
 *    immutable after creation and may be shared between threads.
 *  - Results are bitwise repeatable for the same plan, input and workspace
 *    size on the same device.
 */
#ifndef STKDE_H
#define STKDE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    STKDE_OK = 0,
    STKDE_ERR_INVALID_ARG = -1, /* a null pointer, a size < 1, a non-finite or non-positive scalar */
    STKDE_ERR_TOO_LARGE = -2,   /* a size overflows the library's index types */
    STKDE_ERR_WORKSPACE = -3,   /* workspace missing or smaller than stkde_workspace_bytes() */
    STKDE_ERR_HIP = -4,         /* a HIP runtime call failed (now or in earlier async work) */
    STKDE_ERR_UNSUPPORTED = -5  /* a valid request the library does not handle */
} stkde_status;

/* Flags of stkde_desc.flags. */
enum {
    /* Compensated (Kahan) accumulation across passes of points; within a
     * pass the sum is plain FP32.  Lowers the error of voxels that receive
     * many contributions. */
    STKDE_FLAG_KAHAN = 1u,
    /* Fill d_stats[0] with the FP64 sum of the stored grid (fused into the
     * store; see stkde_compute). */
    STKDE_FLAG_MASS = 4u,
    /* Fill d_stats[1..2] with the per-point FP64 mass and the exact number
     * of kernel evaluations (an extra pass over the points; see
     * stkde_compute). */
    STKDE_FLAG_POINT_STATS = 8u,
    /* Every point carries its own bandwidth pair (hs_i, ht_i): the
     * sample-point reading of the bandwidth that adapts to the local density,
     * named as future work in Sec. 8,
     *   f = 1/n sum_i ks(./hs_i) kt(./ht_i) / (hs_i^2 ht_i).
     * The desc's hs and ht are then the largest pairs the plan accepts (bins,
     * tiles and loop bounds are sized by them).  Such a plan is computed with
     * stkde_compute_adaptive / stkde_bin_adaptive, not with stkde_compute /
     * stkde_bin, and cannot be a batch item. */
    STKDE_FLAG_ADAPTIVE = 16u,
    /* Sample voxel (X, Y, T) at its lower corner (x0 + X sres, y0 + Y sres,
     * t0 + T tres) instead of its centre (Sec. 2.1 leaves the sampling point
     * open).  Not for batch items. */
    STKDE_FLAG_CORNER = 32u
};

/* Kernel pair, in bits 8..11 of stkde_desc.flags (STKDE_FLAG_KERNEL(k)).
 * PB-SYM needs only a product of a spatial and a temporal factor (Sec. 3.2).
 * With u = (x - x_i)/hs, v = (y - y_i)/hs, w = (t - t_i)/ht, on the supports
 * u^2 + v^2 < 1 and |w| <= 1 (zero outside):
 *   EPANECHNIKOV (default)  ks = (2/pi)(1 - u^2 - v^2),    kt = (3/4)(1 - w^2)
 *   QUARTIC                 ks = (3/pi)(1 - u^2 - v^2)^2,  kt = (15/16)(1 - w^2)^2
 *   GAUSSIAN                ks = exp(-2(u^2 + v^2)) / Zs,  kt = exp(-2 w^2) / Zt
 *                           (sigma = half the bandwidth, truncated at it and
 *                           normalised on the support: Zs = (pi/2)(1 - e^-2),
 *                           Zt = sqrt(pi/2) erf(sqrt 2))
 *   PRINTED                 ks = (pi/2)(1 - u)^2 (1 - v)^2, kt = (3/4)(1 - w)^2
 *                           (the pair exactly as Sec. 2.1 prints it; not
 *                           normalised: an interior point carries mass 37 pi^2 / 24)
 * Pairs other than EPANECHNIKOV: no per-point bandwidths (UNSUPPORTED), no
 * batch items, at most 32 time rows per tile (a larger tile_t is lowered). */
enum {
    STKDE_KERNEL_EPANECHNIKOV = 0,
    STKDE_KERNEL_QUARTIC = 1,
    STKDE_KERNEL_GAUSSIAN = 2,
    STKDE_KERNEL_PRINTED = 3
};
#define STKDE_KERNEL_SHIFT 8
#define STKDE_KERNEL_MASK 0xf00u
#define STKDE_FLAG_KERNEL(k) ((uint32_t)(k) << STKDE_KERNEL_SHIFT)

/* Problem description (Sec. 2.1 and Table "Notations").  Lower-case values
 * are in domain units; the grid is gx x gy x gt voxels of sres x sres x tres
 * with the corner of voxel (0,0,0) at (x0, y0, t0). */
typedef struct {
    int64_t gx, gy, gt; /* G_x, G_y, G_t: voxels per axis, each in [1, 65535] */
    double x0, y0, t0;  /* domain coordinate of the corner of voxel (0,0,0), finite */
    double sres, tres;  /* voxel size in space and in time, finite, > 0 */
    double hs, ht;      /* spatial and temporal bandwidth, finite, > 0 */
    uint32_t flags;     /* STKDE_FLAG_* */
} stkde_desc;

/* Optional tuning of one plan.  Zero fields mean "library default".
 * tile_t must be 0, 16, 32 or 64 (64 is reduced to 32 under STKDE_FLAG_KAHAN);
 * cell_xy and cell_t in [4, 256]; split_share 0 or in [64, 65536]; kahan_mode
 * 0, 1 or 2; operand_form 0 or 1.  The plan may enlarge the bins beyond these
 * values when a tile would otherwise read more bin rows than the gather
 * supports.  Tuning changes the summation order, so results differ between
 * tunings in the last bits -- except kahan_mode, whose settings give
 * identical results. */
typedef struct {
    int32_t tile_t;      /* voxel rows in time per output tile (16, 32 or 64) */
    int32_t cell_xy;     /* bin edge in y, voxels; x bins are 8 voxels wide (at
                            most cell_xy), widened only to bound the bin count */
    int32_t cell_t;      /* bin edge in t, voxels */
    int32_t split_share; /* a tile costlier than 1/split_share of its grid's total
                            candidate count (and than 2048 candidates) is split
                            into up to 8 parts; default 2048 */
    int32_t kahan_mode;  /* with STKDE_FLAG_KAHAN, where the running (sum,
                            compensation) pair lives: 1 registers, 2 a per-workgroup
                            scratch slot touched only by tiles that take more
                            than one pass; 0 picks by the expected points per tile */
    int32_t operand_form; /* matrix-core operands of the gather: 0 (default) two
                             FP16 terms each (hi + lo, 22 significant bits; the
                             product as hi*hi + hi*lo + lo*hi with FP32
                             accumulation) where the gather has that form -- one
                             bandwidth pair, 16- or 32-row tiles; with the
                             full-cover path (which only the Epanechnikov pair
                             takes, from hs / sres >= 14) at 16 rows outside
                             batches, for the points that reach a tile in part
                             -- and FP32 elsewhere; 1 FP32 everywhere */
} stkde_tuning;

typedef struct stkde_plan_s* stkde_plan_t;

/* Create a plan from a description (host only, no device allocation).
 * Derives the voxel bandwidths Hs = ceil(hs/sres), Ht = ceil(ht/tres)
 * (Sec. 2.1), the bin and tile geometry and the workspace layout.
 * tuning may be NULL.  Errors: INVALID_ARG (bad field or null pointer),
 * TOO_LARGE (gx*gy*gt*4 bytes overflows, or a dimension above 65535). */
stkde_status stkde_plan(const stkde_desc* desc, const stkde_tuning* tuning, stkde_plan_t* out);

/* Release a plan (and its recorded graph).  NULL is accepted.  The caller
 * makes sure no replay of its graph is still running. */
stkde_status stkde_plan_destroy(stkde_plan_t plan);

/* Gather timing.  stkde_plan_profile(plan, k) makes the next k calls of
 * stkde_compute / stkde_accumulate on the plan record a pair of HIP events
 * on their stream right before and right after the gather kernel (the
 * density accumulation and store, the dominant launch); k = 0 turns it off.
 * stkde_plan_profile_read waits for the recorded pairs, writes up to `max`
 * durations in milliseconds, in call order, to ms (host), sets *count, and
 * starts a new recording of up to k calls.  While profiling, the plan is
 * not safe to share between threads.  Errors: INVALID_ARG, HIP. */
stkde_status stkde_plan_profile(stkde_plan_t plan, int32_t capacity);
stkde_status stkde_plan_profile_read(stkde_plan_t plan, float* ms, int32_t max, int32_t* count);

/* Bytes of device workspace stkde_compute needs for n points (n >= 1). */
stkde_status stkde_workspace_bytes(stkde_plan_t plan, int64_t n, size_t* bytes);

/* Compute the density grid (Sec. 2.1 estimator, PB-SYM of Sec. 3.2).
 *
 *  d_xyt   device, n x 3 FP64, row-major (x, y, t) triples in domain units.
 *          Points may lie outside the grid (their cylinders are clipped);
 *          a point with a non-finite coordinate contributes nothing but
 *          counts in n.  Read only.
 *  n       number of points, 1 <= n <= 2^31 - 1; the estimate divides by n.
 *  d_out   device, gx*gy*gt FP32, indexed [X][Y][T] with T fastest.  Fully
 *          overwritten: no zeroing is required.
 *  d_ws    device workspace of at least stkde_workspace_bytes(plan, n) bytes,
 *          256-byte aligned.  Its contents are scratch between calls.
 *  d_stats device, 8 FP64, optional (NULL to skip).  When given, all 8 are
 *          written; entries whose flag is not set are 0:
 *          [0] (STKDE_FLAG_MASS) FP64 sum of the stored FP32 grid times
 *              sres^2 tres, summed in a fixed order,
 *          [1] (STKDE_FLAG_POINT_STATS) FP64 mass the points deposit on the
 *              grid, from per-point separable in-grid kernel sums (equals
 *              [0] up to the FP32 rounding of the grid),
 *          [2] (STKDE_FLAG_POINT_STATS) exact number of in-grid
 *              (voxel, point) pairs inside both supports, i.e. the kernel
 *              evaluations the method performs,
 *          [3] number of points with a non-finite coordinate,
 *          [4] number of finite points whose cylinder misses the grid,
 *          [5] (STKDE_FLAG_ADAPTIVE) number of points with finite coordinates
 *              whose bandwidth pair is not finite and positive or exceeds
 *              the plan's hs / ht: they contribute nothing, count in n,
 *          [6] number of the grid's tiles computed in parts: a tile
 *              that must examine far more points than its grid's share is
 *              cut into contiguous ranges of its points, computed by several
 *              workgroups and added in range order (the grid then differs
 *              from the uncut computation in its last bits),
 *          [7] reserved (0).
 *  stream  hipStream_t as void*.
 *
 * Errors: INVALID_ARG (also for a plan with STKDE_FLAG_ADAPTIVE), TOO_LARGE,
 * WORKSPACE, HIP. */
stkde_status stkde_compute(stkde_plan_t plan, const double* d_xyt, int64_t n, float* d_out,
                           void* d_ws, size_t ws_bytes, double* d_stats, void* stream);

/* The two stages stkde_compute runs, for callers that reuse a binned point
 * set or time the stages separately.  Both take the arguments of
 * stkde_compute with the same meaning.
 *
 * stkde_bin: transform the points to voxel space, cull the ones whose
 * cylinder misses the grid, sort them stably into space-time bins and write
 * the per-point records into d_ws (the device form
 * of the point lists that the paper's decompositions build per subdomain,
 * Sec. 4.2 and Sec. 5.1).
 *
 * stkde_accumulate: the density accumulation and store of PB-SYM
 * (Sec. 3.2) from a workspace that stkde_bin filled for the same plan and
 * the same n; it must be ordered after that stkde_bin (same stream, or
 * synchronised).  Writes d_out completely, and d_stats[0] (with
 * STKDE_FLAG_MASS) and d_stats[3..7] when d_stats is given ([1], [2] = 0). */
stkde_status stkde_bin(stkde_plan_t plan, const double* d_xyt, int64_t n, void* d_ws,
                       size_t ws_bytes, void* stream);
stkde_status stkde_accumulate(stkde_plan_t plan, int64_t n, float* d_out, void* d_ws,
                              size_t ws_bytes, double* d_stats, void* stream);

/* One stkde_compute as a HIP graph, for callers that repeat the same
 * computation on new point values at fixed addresses (the interactive
 * re-estimation of Sec. 1 at one grid and bandwidth pair): the whole launch
 * sequence is replayed by one graph launch, without the host work and launch
 * gaps of the individual kernels.
 *
 * stkde_plan_capture records stkde_compute(plan, d_xyt, n, d_out, d_ws,
 * ws_bytes, d_stats) -- the same arguments and checks -- into a graph held
 * by the plan (replacing an earlier one); nothing runs.  The graph keeps the
 * pointers and n it was recorded with: d_xyt, d_out, d_ws and d_stats must
 * stay allocated while it is replayed, and a replay reads the point values
 * d_xyt holds when it runs.  No profiling events are recorded into it.
 * stkde_plan_replay launches the graph on `stream`; its result is bitwise
 * that of stkde_compute with the same arguments.  Recording changes the
 * plan: it must not run concurrently with other calls on the same plan.
 * Not for plans with STKDE_FLAG_ADAPTIVE (INVALID_ARG).
 * Errors: as stkde_compute; replay: UNSUPPORTED (nothing recorded), HIP. */
stkde_status stkde_plan_capture(stkde_plan_t plan, const double* d_xyt, int64_t n, float* d_out,
                                void* d_ws, size_t ws_bytes, double* d_stats);
stkde_status stkde_plan_replay(stkde_plan_t plan, void* stream);

/* One stkde_compute without any allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the workspace is the library's own
 * device scratch of STKDE_STATIC_SCRATCH_BYTES (128 MiB), a static array that
 * each GPU the library runs on holds until the process ends.  Arguments and
 * results as stkde_compute (same plan and input: the same bits), without
 * d_ws / ws_bytes; the caller still passes the points, the output and the
 * optional statistics.  No device memory is allocated or freed.
 * Every call on a GPU uses that GPU's one scratch: calls that may overlap on
 * one GPU (other streams, other threads) race and must be ordered by the
 * caller.  Errors: as stkde_compute; WORKSPACE when
 * stkde_workspace_bytes(plan, n) exceeds STKDE_STATIC_SCRATCH_BYTES. */
#define STKDE_STATIC_SCRATCH_BYTES (128u << 20)
stkde_status stkde_compute_noalloc(stkde_plan_t plan, const double* d_xyt, int64_t n, float* d_out,
                                   double* d_stats, void* stream);

/* Per-point bandwidths (plans with STKDE_FLAG_ADAPTIVE; the estimator is
 * given at that flag).  Arguments as stkde_compute / stkde_bin, plus
 *
 *  d_hst   device, n x 2 FP64, row-major (hs_i, ht_i) in domain units, one
 *          pair per point of d_xyt.  Read only.  A pair that is not finite
 *          and positive, or has hs_i > hs or ht_i > ht of the plan, drops its
 *          point (it contributes nothing but counts in n) and is counted in
 *          d_stats[5].  Pairs all equal to the plan's reproduce the grid of
 *          stkde_compute on the plan without the flag (bit for bit where
 *          that grid does not take the full-cover path).
 *
 * Each point's footprint and loop bounds use its own pair.  stkde_accumulate
 * serves adaptive plans too (after stkde_bin_adaptive).  With
 * STKDE_FLAG_POINT_STATS, d_stats[1..2] use the per-point pairs.
 * The gather of such plans has no full-cover path.
 * Errors: as stkde_compute; INVALID_ARG also for a plan without the flag. */
stkde_status stkde_compute_adaptive(stkde_plan_t plan, const double* d_xyt, const double* d_hst, int64_t n,
                                    float* d_out, void* d_ws, size_t ws_bytes, double* d_stats,
                                    void* stream);
stkde_status stkde_bin_adaptive(stkde_plan_t plan, const double* d_xyt, const double* d_hst, int64_t n,
                                void* d_ws, size_t ws_bytes, void* stream);

/* ---- binned point sets ---------------------------------------------------
 *
 * A binned set is the output of stkde_bin kept in caller memory of its own:
 * the points transformed to the voxel space of a base grid, culled, sorted
 * into space-time bins and stored as per-point records (the per-subdomain
 * point lists of Sec. 4.2 and Sec. 5.1, built once on the device).  One set
 * serves any number of later density computations (stkde_batch_*) on the
 * base grid or on a voxel-aligned window of it, with any bandwidths up to
 * the set's, e.g. a bandwidth sweep (the varying bandwidths of Sec. 2.1) or
 * interactive exploration of sub-regions (the motivation of Sec. 1). */
typedef struct stkde_set_s* stkde_set_t;

/* Plan a set of n points on the base grid `base` (host only).  base->hs and
 * base->ht are the largest bandwidths the set will be used with;
 * base->flags must be 0.  tuning may be NULL; its cell_xy / cell_t choose
 * the bin size (as for stkde_plan) and its tile_t is the largest tile_t of
 * the plans the set will serve (default 32).
 * Errors: INVALID_ARG, TOO_LARGE. */
stkde_status stkde_set_plan(const stkde_desc* base, const stkde_tuning* tuning, int64_t n,
                            stkde_set_t* out);

/* Bytes of the set memory (persistent) and of the scratch stkde_set_build
 * needs while it runs. */
stkde_status stkde_set_bytes(stkde_set_t set, size_t* set_bytes, size_t* scratch_bytes);

/* Bin d_xyt (device, n x 3 FP64 as in stkde_compute, the set's n) into
 * d_set (device, >= set_bytes, 256-byte aligned, written completely), using
 * d_scratch (device, >= scratch_bytes, 256-byte aligned) on `stream`.  The
 * set stays valid until d_set is freed or rebuilt; d_xyt and d_scratch may
 * be reused once the stream has passed this call.
 * Errors: INVALID_ARG, WORKSPACE, HIP. */
stkde_status stkde_set_build(stkde_set_t set, const double* d_xyt, void* d_set, size_t set_bytes,
                             void* d_scratch, size_t scratch_bytes, void* stream);

/* Release a set plan (not its device memory).  NULL is accepted. */
stkde_status stkde_set_destroy(stkde_set_t set);

/* ---- batches ---------------------------------------------------------------
 *
 * A batch computes many density grids with one work list and one persistent
 * gather launch per (tile_t, Kahan) group, the tiles of all its grids
 * scheduled together, costliest first.  Each item is one grid: */
typedef struct {
    stkde_plan_t plan;   /* the grid: gx, gy, gt, hs, ht, flags and tuning.tile_t of its
                            desc; its sres and tres must equal the set's, its hs and ht
                            must not exceed the set's, and its origin must be the corner of
                            base voxel (ox, oy, ot): x0 = base x0 + ox * sres (likewise y,
                            t), to 1e-6 of a voxel.  STKDE_FLAG_POINT_STATS is refused. */
    stkde_set_t set;     /* the binned set the grid draws its points from */
    const void* d_set;   /* device memory that stkde_set_build filled for `set` */
    int64_t ox, oy, ot;  /* window origin in base voxels; the window must lie inside the
                            base grid */
    float* d_out;        /* device, gx*gy*gt FP32 [X][Y][T], fully overwritten */
    double* d_stats;     /* device, 8 FP64 as in stkde_compute, or NULL; [1], [2] = 0 */
} stkde_item;
/* The estimate of an item divides by the set's n (every point of the set
 * counts, in the window or not), so a window is a cut-out of the base grid's
 * density.  Items may share sets; their outputs must not overlap. */

typedef struct stkde_batch_s* stkde_batch_t;

/* Validate and copy `count` items (1 <= count <= 4096; host only).
 * Errors: INVALID_ARG (a null pointer, a mismatched resolution, a window
 * outside the base grid, a bandwidth above the set's), TOO_LARGE,
 * UNSUPPORTED (a plan whose tiles would read more bin rows of the set than
 * the gather supports; plan the set with larger cells). */
stkde_status stkde_batch_plan(const stkde_item* items, int32_t count, stkde_batch_t* out);

/* Bytes of device workspace stkde_batch_run needs. */
stkde_status stkde_batch_workspace_bytes(stkde_batch_t batch, size_t* bytes);

/* Number of passes (one gather launch each) stkde_batch_run enqueues (host
 * only).  A batch whose grids are all plain or all compensated, with 16- or
 * 32-row tiles, runs as one pass whatever their operand forms and
 * full-cover paths: one launch of a gather that runs each tile with the
 * code of its grid's own kernel.  Other batches take one pass per (tile
 * rows, accumulation, operand form).  Errors: INVALID_ARG. */
stkde_status stkde_batch_passes(stkde_batch_t batch, int32_t* passes);

/* Compute every item's grid on `stream` (d_ws: >= the workspace bytes,
 * 256-byte aligned; scratch).  Each grid is the one stkde_compute would give
 * for the set's points, within the tolerance of their rounding; it is
 * bitwise the same as the item run alone (in a batch of one) when neither
 * run computes one of its tiles in parts (d_stats[6] = 0 in both).  Which
 * tiles are cut depends on the batch: the costliest tiles of the whole
 * batch (at most 1024) are candidates, within 1024 partial tiles.
 * Errors: WORKSPACE, HIP. */
stkde_status stkde_batch_run(stkde_batch_t batch, void* d_ws, size_t ws_bytes, void* stream);

/* Record stkde_batch_run(batch, d_ws, ws_bytes) into a HIP graph held by the
 * batch (replacing an earlier one).  Nothing runs until stkde_batch_replay.
 * The graph keeps the pointers it was recorded with: d_ws, the sets and
 * the outputs must stay allocated while it is replayed.
 * Errors: WORKSPACE, HIP. */
stkde_status stkde_batch_capture(stkde_batch_t batch, void* d_ws, size_t ws_bytes);

/* Launch the recorded graph on `stream`.  Errors: UNSUPPORTED (nothing
 * recorded), HIP. */
stkde_status stkde_batch_replay(stkde_batch_t batch, void* stream);

/* Release a batch and its graph.  NULL is accepted.  The caller makes sure
 * no replay is still running. */
stkde_status stkde_batch_destroy(stkde_batch_t batch);

/* Human-readable name of a status code (static storage). */
const char* stkde_status_string(stkde_status s);

/* Library version as an integer (major*10000 + minor*100 + patch). */
int32_t stkde_version(void);

#ifdef __cplusplus
}
#endif
#endif /* STKDE_H */
