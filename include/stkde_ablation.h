/*
 * stkde_ablation.h -- two GPU baselines of the density computation, kept
 * beside the library so that its design can be measured against the shapes
 * it replaces.  They are not part of the production path: they compute the
 * same estimate (Sec. 2.1) from the same binned records as stkde_compute,
 * in plain FP32 without compensation, and serve benchmarks and tests.
 *
 *  STKDE_ABLATION_SCATTER  the point-based algorithm PB (Sec. 3.1) run
 *      point-parallel: a fill kernel zeroes the grid, then one workgroup per
 *      point walks the point's clipped footprint box (its cylinder's
 *      bounding box, Sec. 3.2) and adds each non-zero contribution with a
 *      hardware FP32 atomic.  Concurrent points that share voxels race on
 *      them, the conflict of Sec. 4.1; the atomics make the result correct
 *      but its summation order, and so its last bits, differ from run to
 *      run.
 *  STKDE_ABLATION_VOXEL  the voxel-based algorithm with points partitioned
 *      into bandwidth-sized blocks, VB-DEC (Sec. 3): one thread per voxel
 *      sums over the points of every bin within Hs / Ht (plus one voxel) of
 *      its voxel, in bin order.  Deterministic; every voxel tests every
 *      point of its neighbouring bins.
 *
 * Conventions are those of stkde.h (status codes, streams, ownership).
 */
#ifndef STKDE_ABLATION_H
#define STKDE_ABLATION_H

#include "stkde.h"

#ifdef __cplusplus
extern "C" {
#endif

enum {
    STKDE_ABLATION_SCATTER = 1,
    STKDE_ABLATION_VOXEL = 2
};

/* Density accumulation by one of the baselines over the records that
 * stkde_bin wrote into d_ws for the same plan and n (call stkde_bin first, on
 * the same stream).  The plan's flags are ignored: no compensation, no
 * statistics.
 *
 *  method  STKDE_ABLATION_SCATTER or STKDE_ABLATION_VOXEL.
 *  n       the n given to stkde_bin; the estimate divides by n.
 *  d_out   device, gx*gy*gt FP32, [X][Y][T] with T fastest; fully
 *          overwritten (the scatter zeroes it first, on the same stream).
 *  d_ws    the workspace stkde_bin filled, at least
 *          stkde_workspace_bytes(plan, n) bytes, 256-byte aligned; read only.
 *
 * Errors: INVALID_ARG (null pointer, n < 1, unknown method), TOO_LARGE,
 * WORKSPACE, HIP; UNSUPPORTED for a plan with STKDE_FLAG_ADAPTIVE, or one
 * whose footprint boxes or grid exceed 2^31 - 1 voxels. */
stkde_status stkde_ablation_accumulate(stkde_plan_t plan, int32_t method, int64_t n, float* d_out,
                                       void* d_ws, size_t ws_bytes, void* stream);

/* stkde_bin followed by stkde_ablation_accumulate: the arguments of
 * stkde_compute (without statistics) plus the method. */
stkde_status stkde_ablation_compute(stkde_plan_t plan, int32_t method, const double* d_xyt, int64_t n,
                                    float* d_out, void* d_ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* STKDE_ABLATION_H */
