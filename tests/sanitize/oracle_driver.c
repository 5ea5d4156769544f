/*
 * oracle_driver.c -- exercises every function of the FP64 oracle on small
 * random cases (points inside, near and outside the grid, non-finite ones,
 * each kernel pair, centre and corner sampling, fixed and per-point
 * bandwidths) and its argument checks, for a build under AddressSanitizer
 * and UndefinedBehaviorSanitizer.  Beside the sanitizers' own checks it
 * verifies that Alg. VB at every voxel equals Alg. PB-SYM and that the grid
 * sum equals the separable per-point mass.  Exit status 0 when all holds.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/stkde_oracle.h"

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;

static double uni(void) { /* splitmix64 -> [0, 1) */
    uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static int failures = 0;

static void check(int ok, const char* what, int k) {
    if (!ok) {
        fprintf(stderr, "case %d: %s\n", k, what);
        ++failures;
    }
}

static void one_case(int k) {
    oracle_grid g;
    g.gx = 2 + (int64_t)(uni() * 14);
    g.gy = 2 + (int64_t)(uni() * 14);
    g.gt = 2 + (int64_t)(uni() * 12);
    g.sres = 0.5 + uni();
    g.tres = 0.5 + 2.0 * uni();
    g.hs = (0.4 + 4.0 * uni()) * g.sres;
    g.ht = (0.4 + 3.0 * uni()) * g.tres;
    g.x0 = 20.0 * uni() - 10.0;
    g.y0 = 20.0 * uni() - 10.0;
    g.t0 = 20.0 * uni() - 10.0;
    g.kernel = k % 4;
    g.corner = (k / 4) % 2;
    const int64_t n = 1 + (int64_t)(uni() * 60);
    const int64_t G = g.gx * g.gy * g.gt;
    double* xyt = malloc((size_t)n * 3 * sizeof(double));
    double* hst = malloc((size_t)n * 2 * sizeof(double));
    for (int64_t i = 0; i < n; ++i) {
        xyt[3 * i] = g.x0 + (1.4 * uni() - 0.2) * (double)g.gx * g.sres;
        xyt[3 * i + 1] = g.y0 + (1.4 * uni() - 0.2) * (double)g.gy * g.sres;
        xyt[3 * i + 2] = g.t0 + (1.4 * uni() - 0.2) * (double)g.gt * g.tres;
        hst[2 * i] = g.hs * (0.2 + 0.8 * uni());
        hst[2 * i + 1] = g.ht * (0.2 + 0.8 * uni());
    }
    if (n > 3) {
        xyt[0] = NAN;
        xyt[4] = INFINITY;
        hst[2] = -1.0;
    }
    double* grid = malloc((size_t)G * sizeof(double));
    double* grid2 = malloc((size_t)G * sizeof(double));
    double* vb = malloc((size_t)G * sizeof(double));
    int64_t* vox = malloc((size_t)G * 3 * sizeof(int64_t));
    double* Ss = malloc((size_t)n * sizeof(double));
    double* St = malloc((size_t)n * sizeof(double));
    int64_t* cs = malloc((size_t)n * sizeof(int64_t));
    int64_t* ct = malloc((size_t)n * sizeof(int64_t));
    for (int64_t X = 0, j = 0; X < g.gx; ++X)
        for (int64_t Y = 0; Y < g.gy; ++Y)
            for (int64_t T = 0; T < g.gt; ++T, ++j) {
                vox[3 * j] = X;
                vox[3 * j + 1] = Y;
                vox[3 * j + 2] = T;
            }
    for (int adaptive = 0; adaptive < 2; ++adaptive) {
        int64_t ev1 = -1, ev2 = -1;
        int st;
        if (!adaptive) {
            st = oracle_pbsym(&g, xyt, n, grid, &ev1, 1);
            check(st == 0, "pbsym", k);
            st = oracle_pbsym(&g, xyt, n, grid2, &ev2, 3);
            check(st == 0, "pbsym 3 threads", k);
            st = oracle_vb_voxels(&g, xyt, n, vox, G, vb, 2);
            check(st == 0, "vb", k);
            st = oracle_point_sums(&g, xyt, n, Ss, St, cs, ct, 2);
            check(st == 0, "point sums", k);
        } else {
            st = oracle_pbsym_adaptive(&g, xyt, hst, n, grid, &ev1, 1);
            check(st == 0, "pbsym adaptive", k);
            st = oracle_pbsym_adaptive(&g, xyt, hst, n, grid2, &ev2, 3);
            check(st == 0, "pbsym adaptive 3 threads", k);
            st = oracle_vb_voxels_adaptive(&g, xyt, hst, n, vox, G, vb, 2);
            check(st == 0, "vb adaptive", k);
            st = oracle_point_sums_adaptive(&g, xyt, hst, n, Ss, St, cs, ct, 2);
            check(st == 0, "point sums adaptive", k);
        }
        check(ev1 == ev2, "evaluation counts differ between thread counts", k);
        double peak = 0.0, sum = 0.0, mass = 0.0;
        int64_t pairs = 0;
        for (int64_t j = 0; j < G; ++j) {
            check(grid[j] == grid2[j], "thread count changed a value", k);
            if (fabs(grid[j]) > peak) peak = fabs(grid[j]);
            sum += grid[j];
        }
        for (int64_t j = 0; j < G; ++j)
            if (fabs(vb[j] - grid[j]) > 1e-12 * (peak > 0.0 ? peak : 1.0)) {
                check(0, "VB differs from PB-SYM", k);
                break;
            }
        for (int64_t i = 0; i < n; ++i) {
            const double h = adaptive ? hst[2 * i] : g.hs, t = adaptive ? hst[2 * i + 1] : g.ht;
            if (isfinite(Ss[i] * St[i]) && h > 0.0) mass += Ss[i] * St[i] / (h * h * t);
            pairs += cs[i] * ct[i];
        }
        mass /= (double)n;
        check(fabs(mass - sum) <= 1e-10 * (fabs(sum) > 1e-300 ? fabs(sum) : 1.0) + 1e-300,
              "grid sum differs from the separable mass", k);
        check(pairs == ev1, "evaluation count differs from the per-point counts", k);
    }
    /* argument checks */
    check(oracle_pbsym(NULL, xyt, n, grid, NULL, 1) < 0, "null grid accepted", k);
    check(oracle_pbsym(&g, xyt, -1, grid, NULL, 1) < 0, "negative n accepted", k);
    free(xyt);
    free(hst);
    free(grid);
    free(grid2);
    free(vb);
    free(vox);
    free(Ss);
    free(St);
    free(cs);
    free(ct);
}

int main(void) {
    for (int k = 0; k < 48; ++k) one_case(k);
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("oracle sanitizer driver: 48 cases ok\n");
    return 0;
}
