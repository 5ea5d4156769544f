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
    STKDE_ERR_UNSUPPORTED = -5  /* a valid request this build does not handle */
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
    STKDE_FLAG_POINT_STATS = 8u
};

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
 * cell_xy and cell_t in [4, 256].  The plan may
 * enlarge the bins beyond these values when a tile would otherwise read
 * more bin rows than the gather supports.  Tuning changes the summation
 * order, so results differ between tunings in the last bits. */
typedef struct {
    int32_t tile_t;   /* voxel rows in time per output tile (16, 32 or 64) */
    int32_t cell_xy;  /* bin edge in x and y, voxels */
    int32_t cell_t;   /* bin edge in t, voxels */
    int32_t reserved; /* must be 0 */
} stkde_tuning;

typedef struct stkde_plan_s* stkde_plan_t;

/* Create a plan from a description (host only, no device allocation).
 * Derives the voxel bandwidths Hs = ceil(hs/sres), Ht = ceil(ht/tres)
 * (Sec. 2.1), the bin and tile geometry and the workspace layout.
 * tuning may be NULL.  Errors: INVALID_ARG (bad field or null pointer),
 * TOO_LARGE (gx*gy*gt*4 bytes overflows, or a dimension above 65535). */
stkde_status stkde_plan(const stkde_desc* desc, const stkde_tuning* tuning, stkde_plan_t* out);

/* Release a plan.  NULL is accepted. */
stkde_status stkde_plan_destroy(stkde_plan_t plan);

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
 *          [5..7] reserved (0).
 *  stream  hipStream_t as void*.
 *
 * Errors: INVALID_ARG, TOO_LARGE, WORKSPACE, HIP. */
stkde_status stkde_compute(stkde_plan_t plan, const double* d_xyt, int64_t n, float* d_out,
                           void* d_ws, size_t ws_bytes, double* d_stats, void* stream);

/* The two stages stkde_compute runs, for callers that reuse a binned point
 * set or time the stages separately.  Both take the arguments of
 * stkde_compute with the same meaning.
 *
 * stkde_bin: transform the points to voxel space, cull the ones whose
 * cylinder misses the grid, sort them stably into space-time bins and write
 * the per-point records and time-kernel tables into d_ws (the device form
 * of the point lists that the paper's decompositions build per subdomain,
 * Sec. 4.2 and Sec. 5.1).
 *
 * stkde_accumulate: the density accumulation and store of PB-SYM
 * (Sec. 3.2) from a workspace that stkde_bin filled for the same plan and
 * the same n; it must be ordered after that stkde_bin (same stream, or
 * synchronised).  Writes d_out completely, and d_stats[0] (with
 * STKDE_FLAG_MASS) and d_stats[3..7] when d_stats is given ([1], [2] = 0).
 * One kernel launch when d_stats is NULL. */
stkde_status stkde_bin(stkde_plan_t plan, const double* d_xyt, int64_t n, void* d_ws,
                       size_t ws_bytes, void* stream);
stkde_status stkde_accumulate(stkde_plan_t plan, int64_t n, float* d_out, void* d_ws,
                              size_t ws_bytes, double* d_stats, void* stream);

/* Human-readable name of a status code (static storage). */
const char* stkde_status_string(stkde_status s);

/* Library version as an integer (major*10000 + minor*100 + patch). */
int32_t stkde_version(void);

#ifdef __cplusplus
}
#endif
#endif /* STKDE_H */
