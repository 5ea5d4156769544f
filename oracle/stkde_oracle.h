/*
 * stkde_oracle.h -- interface of the FP64 CPU oracle (test infrastructure).
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * use this.  It is deliberately separate from the library's public header:
 * the oracle and the GPU path share no declarations.
 *
 * All arrays are host memory.  xyt holds n points as (x, y, t) triples in
 * domain units, row-major.  Grids are FP64, indexed [X][Y][T], T fastest.
 * Functions return 0 on success and a negative value on invalid arguments
 * (-1) or allocation failure (-2).
 */
#ifndef STKDE_ORACLE_H
#define STKDE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int64_t gx, gy, gt;    /* grid size in voxels (Sec. 2.1: G_x, G_y, G_t) */
    double x0, y0, t0;     /* domain coordinate of the corner of voxel (0,0,0) */
    double sres, tres;     /* voxel size in space and time */
    double hs, ht;         /* spatial and temporal bandwidths, domain units */
    int32_t kernel;        /* ORACLE_KERNEL_*: the separable kernel pair */
    int32_t corner;        /* 0: sample voxels at their centres; 1: at their lower corners */
} oracle_grid;

/* Kernel pairs.  Sec. 2.1 prints one pair (garbled: ORACLE_KERNEL_PRINTED is
 * it taken literally) and the method needs only a product of a spatial and a
 * temporal factor; the others are unit-integral pairs on the same supports
 * (disc u^2 + v^2 < 1, window |w| <= 1):
 *   EPANECHNIKOV  (2/pi)(1 - u^2 - v^2)      x  (3/4)(1 - w^2)          (the default reading)
 *   QUARTIC       (3/pi)(1 - u^2 - v^2)^2    x  (15/16)(1 - w^2)^2
 *   GAUSSIAN      exp(-2(u^2 + v^2)) / Zs    x  exp(-2 w^2) / Zt         (sigma = half the bandwidth,
 *                 Zs = (pi/2)(1 - e^-2), Zt = sqrt(pi/2) erf(sqrt 2): normalised on the support)
 *   PRINTED       (pi/2)(1 - u)^2 (1 - v)^2  x  (3/4)(1 - w)^2          (as printed; not normalised)
 * with u = (x - x_i)/hs, v = (y - y_i)/hs, w = (t - t_i)/ht. */
#define ORACLE_KERNEL_EPANECHNIKOV 0
#define ORACLE_KERNEL_QUARTIC 1
#define ORACLE_KERNEL_GAUSSIAN 2
#define ORACLE_KERNEL_PRINTED 3

/* Alg. PB-SYM (Sec. 3.2) in FP64.  grid: gx*gy*gt doubles, overwritten.
 * evals_out (optional): number of (voxel, point) pairs that pass both
 * support tests. */
int oracle_pbsym(const oracle_grid* g, const double* xyt, int64_t n, double* grid,
                 int64_t* evals_out, int nthreads);

/* Alg. VB (Sec. 2.2) evaluated at m voxels vox[3*j .. 3*j+2] = (X, Y, T). */
int oracle_vb_voxels(const oracle_grid* g, const double* xyt, int64_t n, const int64_t* vox,
                     int64_t m, double* out, int nthreads);

/* Per-point in-grid kernel sums and support counts (any pointer may be NULL):
 * Ss = sum over in-grid columns of ks, St = sum over in-grid rows of kt,
 * cs / ct = the numbers of those columns / rows. */
int oracle_point_sums(const oracle_grid* g, const double* xyt, int64_t n, double* Ss, double* St,
                      int64_t* cs, int64_t* ct, int nthreads);

/* Sample-point adaptive estimator (per-point bandwidths; the adaptive
 * bandwidth named as future work in Sec. 8):
 *
 *   f(x,y,t) = 1/n * sum_i ks((x-xi)/hs_i, (y-yi)/hs_i) kt((t-ti)/ht_i) / (hs_i^2 ht_i)
 *
 * hst holds n pairs (hs_i, ht_i) in domain units, row-major.  A point whose
 * pair is not finite and positive, or whose coordinates are not finite,
 * contributes nothing but counts in n.  The grid's hs and ht are only
 * validated, not used.  Same outputs as the fixed-bandwidth functions. */
int oracle_pbsym_adaptive(const oracle_grid* g, const double* xyt, const double* hst, int64_t n,
                          double* grid, int64_t* evals_out, int nthreads);
int oracle_vb_voxels_adaptive(const oracle_grid* g, const double* xyt, const double* hst, int64_t n,
                              const int64_t* vox, int64_t m, double* out, int nthreads);
int oracle_point_sums_adaptive(const oracle_grid* g, const double* xyt, const double* hst, int64_t n,
                               double* Ss, double* St, int64_t* cs, int64_t* ct, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
