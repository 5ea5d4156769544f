/*
 * stkde_oracle.c -- plain FP64 CPU reference for space-time kernel density
 * estimation (Saule et al., "Parallel Space-Time Kernel Density Estimation",
 * arXiv 1705.09366).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the GPU library is
 * checked against.  It shares no code, header, table or constant with the
 * GPU path, and the product never links or calls it: only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * What it computes (Sec. 2.1, the estimator and the kernel pair):
 *
 *   f(x,y,t) = 1/(n hs^2 ht) * sum_i ks((x-xi)/hs, (y-yi)/hs) * kt((t-ti)/ht)
 *
 * with, under the reading of the garbled kernel formulas used throughout this
 * project (Epanechnikov, normalised to unit integral):
 *
 *   ks(u,v) = (2/pi) (1 - u^2 - v^2)   where sqrt(u^2+v^2) < 1, else 0
 *   kt(w)   = (3/4)  (1 - w^2)         where |w| <= 1,          else 0
 *
 * Other separable kernel pairs (quartic, truncated Gaussian, the pair as
 * printed) are selected by oracle_grid.kernel; stkde_oracle.h defines them.
 *
 * The strict "<" in space and "<=" in time follow the tests written in the
 * VB and PB-SYM algorithms (Sec. 2.2 and Sec. 3.2).  Both kernels vanish on
 * their support boundary, so the choice only changes which pairs are counted
 * as evaluated, not any density value.
 *
 * Voxels (Sec. 2.1, discretisation; Table "Notations"): the grid has
 * Gx x Gy x Gt voxels of size sres x sres x tres whose corner (0,0,0) sits at
 * the domain origin (x0,y0,t0).  A voxel is sampled at its centre,
 * x = x0 + (X + 1/2) sres, and likewise in y and t (or, with
 * oracle_grid.corner, at its lower corner x0 + X sres).  The output grid is
 * indexed stkde[X][Y][T], T fastest.  Hs = ceil(hs/sres) and Ht = ceil(ht/tres)
 * are the bandwidths in voxels; they only bound loops.
 *
 * Points outside the grid are legal: their cylinders are clipped to the grid.
 * A point with a non-finite coordinate contributes nothing but still counts
 * in n.
 *
 * Parallelism: threads own disjoint slabs of X.  Every thread visits all
 * points in input order and adds into its own slab only, so each voxel sums
 * the same terms in the same order whatever the thread count, and the result
 * is bitwise independent of it.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (see build.py).
 * No fast-math: the oracle rounds every operation as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "stkde_oracle.h"

static const double ORACLE_PI = 3.14159265358979323846264338327950288;

/* Spatial kernel of Sec. 2.1 (Epanechnikov reading): unit integral over the
 * unit disc.  Called only inside the support. */
static double ks_epan(double u, double v) {
    return (2.0 / ORACLE_PI) * (1.0 - u * u - v * v);
}

/* Temporal kernel of Sec. 2.1 (Epanechnikov reading): unit integral over
 * [-1, 1].  Called only inside the support. */
static double kt_epan(double w) {
    return 0.75 * (1.0 - w * w);
}

/* The other pairs of stkde_oracle.h, each called only inside its support. */
static double ks_quartic(double u, double v) {
    const double e = 1.0 - u * u - v * v;
    return (3.0 / ORACLE_PI) * e * e;
}

static double kt_quartic(double w) {
    const double e = 1.0 - w * w;
    return (15.0 / 16.0) * e * e;
}

static double ks_gauss(double u, double v) {
    return exp(-2.0 * (u * u + v * v)) / (0.5 * ORACLE_PI * (1.0 - exp(-2.0)));
}

static double kt_gauss(double w) {
    return exp(-2.0 * w * w) / (sqrt(0.5 * ORACLE_PI) * erf(sqrt(2.0)));
}

static double ks_printed(double u, double v) {
    return (ORACLE_PI / 2.0) * (1.0 - u) * (1.0 - u) * (1.0 - v) * (1.0 - v);
}

static double kt_printed(double w) {
    return 0.75 * (1.0 - w) * (1.0 - w);
}

static double ks_of(int32_t kernel, double u, double v) {
    switch (kernel) {
    case ORACLE_KERNEL_QUARTIC: return ks_quartic(u, v);
    case ORACLE_KERNEL_GAUSSIAN: return ks_gauss(u, v);
    case ORACLE_KERNEL_PRINTED: return ks_printed(u, v);
    default: return ks_epan(u, v);
    }
}

static double kt_of(int32_t kernel, double w) {
    switch (kernel) {
    case ORACLE_KERNEL_QUARTIC: return kt_quartic(w);
    case ORACLE_KERNEL_GAUSSIAN: return kt_gauss(w);
    case ORACLE_KERNEL_PRINTED: return kt_printed(w);
    default: return kt_epan(w);
    }
}

/* Where a voxel is sampled, in voxels from its lower corner (Sec. 2.1 leaves
 * it open; the centre is the default reading). */
static double sample_offset(const oracle_grid* g) {
    return g->corner ? 0.0 : 0.5;
}

static int check_desc(const oracle_grid* g, int64_t n) {
    if (!g) return -1;
    if (n < 1) return -1;
    if (g->gx < 1 || g->gy < 1 || g->gt < 1) return -1;
    if (!(g->sres > 0.0) || !(g->tres > 0.0) || !(g->hs > 0.0) || !(g->ht > 0.0)) return -1;
    if (!isfinite(g->sres) || !isfinite(g->tres) || !isfinite(g->hs) || !isfinite(g->ht)) return -1;
    if (!isfinite(g->x0) || !isfinite(g->y0) || !isfinite(g->t0)) return -1;
    if (g->kernel < 0 || g->kernel > ORACLE_KERNEL_PRINTED || (g->corner != 0 && g->corner != 1)) return -1;
    return 0;
}

/* Voxel index of a coordinate along one axis (the paper's X_i), as a double
 * so that points far outside the grid do not overflow an integer. */
static double voxel_of(double c, double c0, double res) {
    return floor((c - c0) / res);
}

/* Clip the loop range [V - H, V + H] of Alg. PB-SYM to [lo, hi); returns 0 if
 * the clipped range is empty. */
static int clip_range(double v, int64_t h, int64_t lo, int64_t hi, int64_t* a, int64_t* b) {
    double da = v - (double)h, db = v + (double)h;
    if (db < (double)lo || da > (double)(hi - 1)) return 0;
    *a = da < (double)lo ? lo : (int64_t)da;
    *b = db > (double)(hi - 1) ? hi - 1 : (int64_t)db;
    return *a <= *b;
}

int oracle_pbsym(const oracle_grid* g, const double* xyt, int64_t n, double* grid,
                 int64_t* evals_out, int nthreads) {
    if (check_desc(g, n) || !xyt || !grid) return -1;
    const int64_t Gx = g->gx, Gy = g->gy, Gt = g->gt;
    const int64_t Hs = (int64_t)ceil(g->hs / g->sres);
    const int64_t Ht = (int64_t)ceil(g->ht / g->tres);
    const double norm = 1.0 / ((double)n * g->hs * g->hs * g->ht);
    const int64_t side = 2 * Hs + 1;
    int64_t evals_total = 0;

    if (nthreads < 1) nthreads = 1;
    if ((int64_t)nthreads > Gx) nthreads = (int)Gx;

    /* Zero the grid (first loop of Alg. PB-SYM). */
    memset(grid, 0, (size_t)(Gx * Gy * Gt) * sizeof(double));

    int err = 0;
#pragma omp parallel num_threads(nthreads) reduction(+ : evals_total)
    {
        int tid = 0, nth = 1;
#ifdef _OPENMP
        tid = omp_get_thread_num();
        nth = omp_get_num_threads();
#endif
        const int64_t xa = Gx * tid / nth, xb = Gx * (tid + 1) / nth;
        double* Ks = (double*)malloc((size_t)(side * side) * sizeof(double));
        double* Kt = (double*)malloc((size_t)(2 * Ht + 1) * sizeof(double));
        unsigned char* ins = (unsigned char*)malloc((size_t)(side * side));
        unsigned char* int_ = (unsigned char*)malloc((size_t)(2 * Ht + 1));
        if (!Ks || !Kt || !ins || !int_) {
#pragma omp atomic write
            err = 1;
        } else {
            for (int64_t i = 0; i < n; ++i) {
                const double xi = xyt[3 * i], yi = xyt[3 * i + 1], ti = xyt[3 * i + 2];
                if (!isfinite(xi) || !isfinite(yi) || !isfinite(ti)) continue;
                const double Xi = voxel_of(xi, g->x0, g->sres);
                const double Yi = voxel_of(yi, g->y0, g->sres);
                const double Ti = voxel_of(ti, g->t0, g->tres);
                int64_t Xa, Xb, Ya, Yb, Ta, Tb;
                if (!clip_range(Xi, Hs, xa, xb, &Xa, &Xb)) continue;
                if (!clip_range(Yi, Hs, 0, Gy, &Ya, &Yb)) continue;
                if (!clip_range(Ti, Ht, 0, Gt, &Ta, &Tb)) continue;
                const int64_t ny = Yb - Ya + 1, nt = Tb - Ta + 1;

                /* Spatial invariant Ks[X][Y] over the box, normalisation folded
                 * in (second loop nest of Alg. PB-SYM). */
                for (int64_t X = Xa; X <= Xb; ++X) {
                    const double x = g->x0 + ((double)X + sample_offset(g)) * g->sres;
                    for (int64_t Y = Ya; Y <= Yb; ++Y) {
                        const double y = g->y0 + ((double)Y + sample_offset(g)) * g->sres;
                        const int64_t k = (X - Xa) * ny + (Y - Ya);
                        const double d = sqrt((xi - x) * (xi - x) + (yi - y) * (yi - y));
                        if (d < g->hs) {
                            Ks[k] = ks_of(g->kernel, (x - xi) / g->hs, (y - yi) / g->hs) * norm;
                            ins[k] = 1;
                        } else {
                            Ks[k] = 0.0;
                            ins[k] = 0;
                        }
                    }
                }
                /* Temporal invariant Kt[T] over the window (third loop). */
                int64_t cnt_t = 0;
                for (int64_t T = Ta; T <= Tb; ++T) {
                    const double t = g->t0 + ((double)T + sample_offset(g)) * g->tres;
                    if (fabs(ti - t) <= g->ht) {
                        Kt[T - Ta] = kt_of(g->kernel, (t - ti) / g->ht);
                        int_[T - Ta] = 1;
                        ++cnt_t;
                    } else {
                        Kt[T - Ta] = 0.0;
                        int_[T - Ta] = 0;
                    }
                }
                /* stkde[X][Y][T] += Ks[X][Y] * Kt[T] (last loop nest).  A zero
                 * Ks adds +0.0, which leaves every value unchanged, so the
                 * column is skipped. */
                for (int64_t X = Xa; X <= Xb; ++X) {
                    for (int64_t Y = Ya; Y <= Yb; ++Y) {
                        const int64_t k = (X - Xa) * ny + (Y - Ya);
                        if (!ins[k]) continue;
                        evals_total += cnt_t;
                        const double ks = Ks[k];
                        double* col = grid + (X * Gy + Y) * Gt + Ta;
                        for (int64_t T = 0; T < nt; ++T) col[T] += ks * Kt[T];
                    }
                }
            }
        }
        free(Ks);
        free(Kt);
        free(ins);
        free(int_);
    }
    if (err) return -2;
    if (evals_out) *evals_out = evals_total;
    return 0;
}

/* Alg. VB at a list of voxels: for each voxel, scan every point in input
 * order with the cylinder test and sum the kernel products, then divide by
 * n hs^2 ht.  vox holds m (X, Y, T) triples. */
int oracle_vb_voxels(const oracle_grid* g, const double* xyt, int64_t n, const int64_t* vox,
                     int64_t m, double* out, int nthreads) {
    if (check_desc(g, n) || !xyt || (m > 0 && (!vox || !out))) return -1;
    for (int64_t j = 0; j < m; ++j) {
        if (vox[3 * j] < 0 || vox[3 * j] >= g->gx || vox[3 * j + 1] < 0 || vox[3 * j + 1] >= g->gy ||
            vox[3 * j + 2] < 0 || vox[3 * j + 2] >= g->gt)
            return -1;
    }
    if (nthreads < 1) nthreads = 1;
    const double denom = (double)n * g->hs * g->hs * g->ht;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int64_t j = 0; j < m; ++j) {
        const double x = g->x0 + ((double)vox[3 * j] + sample_offset(g)) * g->sres;
        const double y = g->y0 + ((double)vox[3 * j + 1] + sample_offset(g)) * g->sres;
        const double t = g->t0 + ((double)vox[3 * j + 2] + sample_offset(g)) * g->tres;
        double sum = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            const double xi = xyt[3 * i], yi = xyt[3 * i + 1], ti = xyt[3 * i + 2];
            if (!isfinite(xi) || !isfinite(yi) || !isfinite(ti)) continue;
            if (sqrt((xi - x) * (xi - x) + (yi - y) * (yi - y)) < g->hs && fabs(ti - t) <= g->ht)
                sum += ks_of(g->kernel, (x - xi) / g->hs, (y - yi) / g->hs) * kt_of(g->kernel, (t - ti) / g->ht);
        }
        out[j] = sum / denom;
    }
    return 0;
}

/* Per-point in-grid sums.  For point i: Ss[i] = sum of ks over the in-grid
 * voxel columns (X,Y) inside its disc, St[i] = sum of kt over the in-grid
 * rows T inside its window, and cs[i], ct[i] the numbers of such columns and
 * rows.  Clipping to the grid is a box, so the mass point i deposits on the
 * grid is Ss[i] * St[i] / (n hs^2 ht) and the number of (voxel, point) pairs
 * it is evaluated on is cs[i] * ct[i] (the separability used by PB-SYM,
 * Sec. 3.2). */
int oracle_point_sums(const oracle_grid* g, const double* xyt, int64_t n, double* Ss, double* St,
                      int64_t* cs, int64_t* ct, int nthreads) {
    if (check_desc(g, n) || !xyt) return -1;
    const int64_t Hs = (int64_t)ceil(g->hs / g->sres);
    const int64_t Ht = (int64_t)ceil(g->ht / g->tres);
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double xi = xyt[3 * i], yi = xyt[3 * i + 1], ti = xyt[3 * i + 2];
        double ss = 0.0, st = 0.0;
        int64_t ns = 0, nt = 0;
        if (isfinite(xi) && isfinite(yi) && isfinite(ti)) {
            int64_t Xa = 0, Xb = -1, Ya = 0, Yb = -1, Ta = 0, Tb = -1;
            const int okx = clip_range(voxel_of(xi, g->x0, g->sres), Hs, 0, g->gx, &Xa, &Xb);
            const int oky = clip_range(voxel_of(yi, g->y0, g->sres), Hs, 0, g->gy, &Ya, &Yb);
            const int okt = clip_range(voxel_of(ti, g->t0, g->tres), Ht, 0, g->gt, &Ta, &Tb);
            if (okx && oky) {
                for (int64_t X = Xa; X <= Xb; ++X) {
                    const double x = g->x0 + ((double)X + sample_offset(g)) * g->sres;
                    for (int64_t Y = Ya; Y <= Yb; ++Y) {
                        const double y = g->y0 + ((double)Y + sample_offset(g)) * g->sres;
                        if (sqrt((xi - x) * (xi - x) + (yi - y) * (yi - y)) < g->hs) {
                            ss += ks_of(g->kernel, (x - xi) / g->hs, (y - yi) / g->hs);
                            ++ns;
                        }
                    }
                }
            }
            if (okt) {
                for (int64_t T = Ta; T <= Tb; ++T) {
                    const double t = g->t0 + ((double)T + sample_offset(g)) * g->tres;
                    if (fabs(ti - t) <= g->ht) {
                        st += kt_of(g->kernel, (t - ti) / g->ht);
                        ++nt;
                    }
                }
            }
        }
        if (Ss) Ss[i] = ss;
        if (St) St[i] = st;
        if (cs) cs[i] = ns;
        if (ct) ct[i] = nt;
    }
    return 0;
}

/* ---- sample-point adaptive bandwidths -----------------------------------
 *
 * Sec. 8 names a bandwidth that adapts to the local density of the
 * population as future work, without fixing a rule for choosing it.  The
 * reading taken here is the sample-point estimator: every event i carries
 * its own bandwidth pair (hs_i, ht_i), given as input, and contributes
 * ks(./hs_i) kt(./ht_i) / (n hs_i^2 ht_i), so that each event still carries
 * unit mass.  The algorithms are those above with the event's own pair in
 * place of (hs, ht): its loop bounds ceil(hs_i/sres), ceil(ht_i/tres), its
 * support tests and its normalisation. */

/* clip_range with the loop half-width as a double: an event's own ceil(hs_i /
 * sres) may exceed any integer type while its clipped box stays inside the
 * grid. */
static int clip_range_d(double v, double h, int64_t lo, int64_t hi, int64_t* a, int64_t* b) {
    double da = v - h, db = v + h;
    if (db < (double)lo || da > (double)(hi - 1)) return 0;
    *a = da < (double)lo ? lo : (int64_t)da;
    *b = db > (double)(hi - 1) ? hi - 1 : (int64_t)db;
    return *a <= *b;
}

/* 1 when event i has finite coordinates and a finite positive pair. */
static int adaptive_event_ok(const double* xyt, const double* hst, int64_t i) {
    const double xi = xyt[3 * i], yi = xyt[3 * i + 1], ti = xyt[3 * i + 2];
    const double hs = hst[2 * i], ht = hst[2 * i + 1];
    return isfinite(xi) && isfinite(yi) && isfinite(ti) && isfinite(hs) && isfinite(ht) && hs > 0.0 &&
           ht > 0.0;
}

int oracle_pbsym_adaptive(const oracle_grid* g, const double* xyt, const double* hst, int64_t n,
                          double* grid, int64_t* evals_out, int nthreads) {
    if (check_desc(g, n) || !xyt || !hst || !grid) return -1;
    const int64_t Gx = g->gx, Gy = g->gy, Gt = g->gt;
    /* Tables over an event's clipped box: at most (2 Hs_i + 1) wide and never
     * wider than the grid. */
    double hs_max = 0.0, ht_max = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!adaptive_event_ok(xyt, hst, i)) continue;
        const double hsv = ceil(hst[2 * i] / g->sres), htv = ceil(hst[2 * i + 1] / g->tres);
        if (hsv > hs_max) hs_max = hsv;
        if (htv > ht_max) ht_max = htv;
    }
    const int64_t wx = 2.0 * hs_max + 1.0 < (double)Gx ? (int64_t)(2.0 * hs_max + 1.0) : Gx;
    const int64_t wy = 2.0 * hs_max + 1.0 < (double)Gy ? (int64_t)(2.0 * hs_max + 1.0) : Gy;
    const int64_t wt = 2.0 * ht_max + 1.0 < (double)Gt ? (int64_t)(2.0 * ht_max + 1.0) : Gt;
    int64_t evals_total = 0;
    if (nthreads < 1) nthreads = 1;
    if ((int64_t)nthreads > Gx) nthreads = (int)Gx;

    memset(grid, 0, (size_t)(Gx * Gy * Gt) * sizeof(double));

    int err = 0;
#pragma omp parallel num_threads(nthreads) reduction(+ : evals_total)
    {
        int tid = 0, nth = 1;
#ifdef _OPENMP
        tid = omp_get_thread_num();
        nth = omp_get_num_threads();
#endif
        const int64_t xa = Gx * tid / nth, xb = Gx * (tid + 1) / nth;
        double* Ks = (double*)malloc((size_t)(wx * wy) * sizeof(double));
        double* Kt = (double*)malloc((size_t)wt * sizeof(double));
        unsigned char* ins = (unsigned char*)malloc((size_t)(wx * wy));
        if (!Ks || !Kt || !ins) {
#pragma omp atomic write
            err = 1;
        } else {
            for (int64_t i = 0; i < n; ++i) {
                if (!adaptive_event_ok(xyt, hst, i)) continue;
                const double xi = xyt[3 * i], yi = xyt[3 * i + 1], ti = xyt[3 * i + 2];
                const double hs = hst[2 * i], ht = hst[2 * i + 1];
                /* the event's own loop bounds Hs_i, Ht_i and normalisation */
                const double Hs = ceil(hs / g->sres), Ht = ceil(ht / g->tres);
                const double norm = 1.0 / ((double)n * hs * hs * ht);
                int64_t Xa, Xb, Ya, Yb, Ta, Tb;
                if (!clip_range_d(voxel_of(xi, g->x0, g->sres), Hs, xa, xb, &Xa, &Xb)) continue;
                if (!clip_range_d(voxel_of(yi, g->y0, g->sres), Hs, 0, Gy, &Ya, &Yb)) continue;
                if (!clip_range_d(voxel_of(ti, g->t0, g->tres), Ht, 0, Gt, &Ta, &Tb)) continue;
                const int64_t ny = Yb - Ya + 1, nt = Tb - Ta + 1;
                for (int64_t X = Xa; X <= Xb; ++X) {
                    const double x = g->x0 + ((double)X + sample_offset(g)) * g->sres;
                    for (int64_t Y = Ya; Y <= Yb; ++Y) {
                        const double y = g->y0 + ((double)Y + sample_offset(g)) * g->sres;
                        const int64_t k = (X - Xa) * ny + (Y - Ya);
                        const double d = sqrt((xi - x) * (xi - x) + (yi - y) * (yi - y));
                        if (d < hs) {
                            Ks[k] = ks_of(g->kernel, (x - xi) / hs, (y - yi) / hs) * norm;
                            ins[k] = 1;
                        } else {
                            Ks[k] = 0.0;
                            ins[k] = 0;
                        }
                    }
                }
                int64_t cnt_t = 0;
                for (int64_t T = Ta; T <= Tb; ++T) {
                    const double t = g->t0 + ((double)T + sample_offset(g)) * g->tres;
                    if (fabs(ti - t) <= ht) {
                        Kt[T - Ta] = kt_of(g->kernel, (t - ti) / ht);
                        ++cnt_t;
                    } else {
                        Kt[T - Ta] = 0.0;
                    }
                }
                for (int64_t X = Xa; X <= Xb; ++X) {
                    for (int64_t Y = Ya; Y <= Yb; ++Y) {
                        const int64_t k = (X - Xa) * ny + (Y - Ya);
                        if (!ins[k]) continue;
                        evals_total += cnt_t;
                        const double ks = Ks[k];
                        double* col = grid + (X * Gy + Y) * Gt + Ta;
                        for (int64_t T = 0; T < nt; ++T) col[T] += ks * Kt[T];
                    }
                }
            }
        }
        free(Ks);
        free(Kt);
        free(ins);
    }
    if (err) return -2;
    if (evals_out) *evals_out = evals_total;
    return 0;
}

/* Alg. VB with per-event bandwidths at m voxels: each event's term carries
 * its own 1/(hs_i^2 ht_i); the sum is divided by n at the end. */
int oracle_vb_voxels_adaptive(const oracle_grid* g, const double* xyt, const double* hst, int64_t n,
                              const int64_t* vox, int64_t m, double* out, int nthreads) {
    if (check_desc(g, n) || !xyt || !hst || (m > 0 && (!vox || !out))) return -1;
    for (int64_t j = 0; j < m; ++j) {
        if (vox[3 * j] < 0 || vox[3 * j] >= g->gx || vox[3 * j + 1] < 0 || vox[3 * j + 1] >= g->gy ||
            vox[3 * j + 2] < 0 || vox[3 * j + 2] >= g->gt)
            return -1;
    }
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int64_t j = 0; j < m; ++j) {
        const double x = g->x0 + ((double)vox[3 * j] + sample_offset(g)) * g->sres;
        const double y = g->y0 + ((double)vox[3 * j + 1] + sample_offset(g)) * g->sres;
        const double t = g->t0 + ((double)vox[3 * j + 2] + sample_offset(g)) * g->tres;
        double sum = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (!adaptive_event_ok(xyt, hst, i)) continue;
            const double xi = xyt[3 * i], yi = xyt[3 * i + 1], ti = xyt[3 * i + 2];
            const double hs = hst[2 * i], ht = hst[2 * i + 1];
            if (sqrt((xi - x) * (xi - x) + (yi - y) * (yi - y)) < hs && fabs(ti - t) <= ht)
                sum += ks_of(g->kernel, (x - xi) / hs, (y - yi) / hs) * kt_of(g->kernel, (t - ti) / ht) / (hs * hs * ht);
        }
        out[j] = sum / (double)n;
    }
    return 0;
}

/* Per-event in-grid sums with the event's own bandwidths (as
 * oracle_point_sums); the mass event i deposits is
 * Ss[i] St[i] / (n hs_i^2 ht_i) sres^2 tres. */
int oracle_point_sums_adaptive(const oracle_grid* g, const double* xyt, const double* hst, int64_t n,
                               double* Ss, double* St, int64_t* cs, int64_t* ct, int nthreads) {
    if (check_desc(g, n) || !xyt || !hst) return -1;
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double ss = 0.0, st = 0.0;
        int64_t ns = 0, nt = 0;
        if (adaptive_event_ok(xyt, hst, i)) {
            const double xi = xyt[3 * i], yi = xyt[3 * i + 1], ti = xyt[3 * i + 2];
            const double hs = hst[2 * i], ht = hst[2 * i + 1];
            const double Hs = ceil(hs / g->sres), Ht = ceil(ht / g->tres);
            int64_t Xa = 0, Xb = -1, Ya = 0, Yb = -1, Ta = 0, Tb = -1;
            const int okx = clip_range_d(voxel_of(xi, g->x0, g->sres), Hs, 0, g->gx, &Xa, &Xb);
            const int oky = clip_range_d(voxel_of(yi, g->y0, g->sres), Hs, 0, g->gy, &Ya, &Yb);
            const int okt = clip_range_d(voxel_of(ti, g->t0, g->tres), Ht, 0, g->gt, &Ta, &Tb);
            if (okx && oky) {
                for (int64_t X = Xa; X <= Xb; ++X) {
                    const double x = g->x0 + ((double)X + sample_offset(g)) * g->sres;
                    for (int64_t Y = Ya; Y <= Yb; ++Y) {
                        const double y = g->y0 + ((double)Y + sample_offset(g)) * g->sres;
                        if (sqrt((xi - x) * (xi - x) + (yi - y) * (yi - y)) < hs) {
                            ss += ks_of(g->kernel, (x - xi) / hs, (y - yi) / hs);
                            ++ns;
                        }
                    }
                }
            }
            if (okt) {
                for (int64_t T = Ta; T <= Tb; ++T) {
                    const double t = g->t0 + ((double)T + sample_offset(g)) * g->tres;
                    if (fabs(ti - t) <= ht) {
                        st += kt_of(g->kernel, (t - ti) / ht);
                        ++nt;
                    }
                }
            }
        }
        if (Ss) Ss[i] = ss;
        if (St) St[i] = st;
        if (cs) cs[i] = ns;
        if (ct) ct[i] = nt;
    }
    return 0;
}
