// stats.hip -- per-point FP64 checks of a computed grid (not on the hot path).
//
// Because clipping a cylinder to the grid is a box and the kernel is a
// product of a spatial and a temporal factor (the separability PB-SYM
// exploits, Sec. 3.2), the mass point i deposits on the grid is
// Ss(i) * St(i) / (n hs^2 ht), with Ss(i) the sum of ks over its in-grid
// columns and St(i) the sum of kt over its in-grid rows, and the number of
// (voxel, point) pairs it is evaluated on is cs(i) * ct(i).  This kernel
// evaluates those sums in FP64 with the support tests of Alg. VB / PB-SYM
// written in domain units (spatial distance < hs via a square root, time
// distance <= ht), in the same precision and the same form as the CPU
// reference, so that the integer counts agree exactly.  With per-point
// bandwidths each point uses its own pair and loop bounds and its mass
// carries (hs^2 ht) / (hs_i^2 ht_i) relative to the instance's pair; a
// pair that binning drops (not finite and positive, or above the
// instance's) contributes nothing here either.
#include "stkde_internal.h"

namespace stkde {
namespace {

// The kernel pairs in FP64, each evaluated only inside its support
// (u = (x - x_i)/hs, v = (y - y_i)/hs, w = (t - t_i)/ht).
__device__ inline double spatial_kernel(int32_t kernel, double u, double v) {
    const double r2 = u * u + v * v;
    switch (kernel) {
    case kKernelQuartic: return (3.0 / 3.14159265358979323846) * (1.0 - r2) * (1.0 - r2);
    case kKernelGauss: return exp(-2.0 * r2) / (0.5 * 3.14159265358979323846 * (1.0 - exp(-2.0)));
    case kKernelPrinted: return (0.5 * 3.14159265358979323846) * (1.0 - u) * (1.0 - u) * (1.0 - v) * (1.0 - v);
    default: return (2.0 / 3.14159265358979323846) * (1.0 - u * u - v * v);
    }
}

__device__ inline double temporal_kernel(int32_t kernel, double w) {
    switch (kernel) {
    case kKernelQuartic: return 0.9375 * (1.0 - w * w) * (1.0 - w * w);
    case kKernelGauss: return exp(-2.0 * w * w) / (sqrt(0.5 * 3.14159265358979323846) * erf(sqrt(2.0)));
    case kKernelPrinted: return 0.75 * (1.0 - w) * (1.0 - w);
    default: return 0.75 * (1.0 - w * w);
    }
}

__device__ inline bool clip_rng(double v, double h, int32_t lo, int32_t hi, int32_t* a, int32_t* b) {
    const double da = v - h, db = v + h;
    if (db < (double)lo || da > (double)(hi - 1)) return false;
    *a = da < (double)lo ? lo : (int32_t)da;
    *b = db > (double)(hi - 1) ? hi - 1 : (int32_t)db;
    return *a <= *b;
}

__global__ __launch_bounds__(kStatBlock) void k_point_stats(InstGeom g, const double* __restrict__ xyt,
                                                            const double* __restrict__ hst, int32_t n,
                                                            double* __restrict__ part) {
#pragma clang fp contract(off)
    __shared__ double sm[kStatBlock];
    __shared__ double se[kStatBlock];
    const int32_t i = blockIdx.x * kStatBlock + threadIdx.x;
    double mass = 0.0, evals = 0.0;
    if (i < n) {
        const double xi = xyt[3 * (size_t)i], yi = xyt[3 * (size_t)i + 1], ti = xyt[3 * (size_t)i + 2];
        double hs = g.hs, ht = g.ht, Hs = g.Hs_d, Ht = g.Ht_d, wi = 1.0;
        bool ok = true;
        if (hst) {
            hs = hst[2 * (size_t)i];
            ht = hst[2 * (size_t)i + 1];
            ok = isfinite(hs) && isfinite(ht) && hs > 0.0 && ht > 0.0 && hs / g.sres <= g.hv &&
                 ht / g.tres <= g.tv;
            if (ok) {
                Hs = ceil(hs / g.sres);
                Ht = ceil(ht / g.tres);
                wi = (g.hs * g.hs * g.ht) / (hs * hs * ht);
            }
        }
        if (ok && isfinite(xi) && isfinite(yi) && isfinite(ti)) {
            const double Xi = floor((xi - g.x0) / g.sres);
            const double Yi = floor((yi - g.y0) / g.sres);
            const double Ti = floor((ti - g.t0) / g.tres);
            int32_t xa, xb, ya, yb, ta, tb;
            double ss = 0.0, st = 0.0;
            long long cs = 0, ct = 0;
            if (clip_rng(Xi, Hs, 0, g.gx, &xa, &xb) && clip_rng(Yi, Hs, 0, g.gy, &ya, &yb)) {
                for (int32_t X = xa; X <= xb; ++X) {
                    const double x = g.x0 + ((double)X + 0.5) * g.sres;
                    for (int32_t Y = ya; Y <= yb; ++Y) {
                        const double y = g.y0 + ((double)Y + 0.5) * g.sres;
                        const double d = sqrt((xi - x) * (xi - x) + (yi - y) * (yi - y));
                        if (d < hs) {
                            const double u = (x - xi) / hs, v = (y - yi) / hs;
                            ss += spatial_kernel(g.kernel, u, v);
                            ++cs;
                        }
                    }
                }
            }
            if (clip_rng(Ti, Ht, 0, g.gt, &ta, &tb)) {
                for (int32_t T = ta; T <= tb; ++T) {
                    const double t = g.t0 + ((double)T + 0.5) * g.tres;
                    if (fabs(ti - t) <= ht) {
                        const double w = (t - ti) / ht;
                        st += temporal_kernel(g.kernel, w);
                        ++ct;
                    }
                }
            }
            mass = ss * st * wi;
            evals = (double)(cs * ct);
        }
    }
    sm[threadIdx.x] = mass;
    se[threadIdx.x] = evals;
    __syncthreads();
    for (int w = kStatBlock / 2; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sm[threadIdx.x] += sm[threadIdx.x + w];
            se[threadIdx.x] += se[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[4 * (size_t)blockIdx.x + 0] = sm[0];
        part[4 * (size_t)blockIdx.x + 1] = se[0];
        part[4 * (size_t)blockIdx.x + 2] = 0.0;
        part[4 * (size_t)blockIdx.x + 3] = 0.0;
    }
}

// d_stats[1] = sum of mass partials / (n hs^2 ht) * sres^2 tres;
// d_stats[2] = sum of evaluation counts (exact below 2^53).
__global__ __launch_bounds__(1024) void k_stats_final(const double* __restrict__ part, int32_t nblk,
                                                      double scale, double* __restrict__ stats) {
    __shared__ double sm[1024];
    __shared__ double se[1024];
    double a = 0.0, b = 0.0;
    for (int32_t k = threadIdx.x; k < nblk; k += 1024) {
        a += part[4 * (size_t)k];
        b += part[4 * (size_t)k + 1];
    }
    sm[threadIdx.x] = a;
    se[threadIdx.x] = b;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) {
            sm[threadIdx.x] += sm[threadIdx.x + w];
            se[threadIdx.x] += se[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        stats[1] = sm[0] * scale;
        stats[2] = se[0];
    }
}

}  // namespace

hipError_t launch_point_stats(const InstGeom& g, int64_t n_norm, const double* d_xyt, int32_t n,
                              double* d_stats, double* part, int32_t nblk, hipStream_t s,
                              const double* d_hst) {
    hipLaunchKernelGGL(k_point_stats, dim3(nblk), dim3(kStatBlock), 0, s, g, d_xyt, d_hst, n, part);
    const double scale = g.sres * g.sres * g.tres / ((double)n_norm * g.hs * g.hs * g.ht);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(1024), 0, s, (const double*)part, nblk, scale,
                       d_stats);
    return hipGetLastError();
}

}  // namespace stkde
