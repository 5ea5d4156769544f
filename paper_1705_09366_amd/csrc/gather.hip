// gather.hip -- the density accumulation of PB-SYM (Sec. 3.2), as an
// atomic-free gather over output tiles.
//
// PB-SYM adds, for every point, the outer product of a spatial table
// Ks[X][Y] and a temporal table Kt[T] into the grid.  Here every voxel is
// owned by exactly one lane, which sums the contributions of all points
// whose cylinder covers it, in a fixed order (bins in order, points in
// sorted order within a bin), and stores the result once:
//
//  * a workgroup owns a 16 x 16 x TT tile; each of its four waves owns an
//    8 x 8 patch of columns; each lane owns one column (X, Y) and holds its
//    TT rows of the tile in registers;
//  * a wave walks the bins that can hold points reaching its patch, tests 64
//    candidates at a time (one per lane) against the patch, and then
//    visits the hits one by one with wave-uniform (scalar) loads;
//  * per visit the lane evaluates the spatial factor of its column,
//    ks = max(0, 1 - (dx^2 + dy^2)/hv^2), once (the Ks table entry), and
//    accumulates ks * kt(T) over the rows of the point's window that fall in
//    the tile, 4 rows per table chunk (the Kt table entries come from the
//    point's precomputed table as scalar operands);
//  * the normalisation (2/pi)(3/4)/(n hs^2 ht) is applied once at the store.
//
// There is no zeroing pass and no read-modify-write of the grid: each voxel
// is written exactly once (the initialisation cost the paper measures,
// Sec. 6.2, disappears into the store).
#include "stkde_internal.h"

namespace stkde {
namespace {

struct GatherArgs {
    const uint32_t* cell_start;
    const PointRec* recs;
    const float* kt;
    float* out;
    double* tile_part;
    int32_t gx, gy, gt;
    int32_t Hs, Ht;
    int32_t cxy, ct, ncx, ncy, nct;
    int32_t ntx, nty, ntiles;
    int32_t ktw;
    float inv_hv2;
    float cnorm;
};

__device__ inline int32_t floordiv_d(int32_t a, int32_t b) {
    int32_t q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}

__device__ inline int32_t clampi(int32_t v, int32_t lo, int32_t hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

template <int TT>
__device__ inline void kahan_fold(float (&acc)[TT], float (&comp)[TT], float (&pass)[TT]) {
#pragma unroll
    for (int r = 0; r < TT; ++r) {
        const float y = __fsub_rn(pass[r], comp[r]);
        const float t = __fadd_rn(acc[r], y);
        comp[r] = __fsub_rn(__fsub_rn(t, acc[r]), y);
        acc[r] = t;
        pass[r] = 0.0f;
    }
}

template <int TT, bool KAHAN, bool MASS>
__global__ __launch_bounds__(kThreads) void k_gather(GatherArgs a) {
    constexpr int NCH = TT / kChunk;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    // Tiles are dealt to the 8 XCDs in contiguous ranges (workgroup i runs on
    // XCD i mod 8), so neighbouring tiles, which read the same bins, share
    // an L2.
    const int32_t bid = blockIdx.x;
    const int32_t per = a.ntiles >> 3, rem = a.ntiles & 7;
    const int32_t xcd = bid & 7, slot = bid >> 3;
    const int32_t tile = xcd * per + min(xcd, rem) + slot;
    const int32_t tx = tile % a.ntx;
    const int32_t rest = tile / a.ntx;
    const int32_t ty = rest % a.nty;
    const int32_t tt = rest / a.nty;

    const int32_t PX0 = tx * kTileXY + (wave & 1) * kPatch;
    const int32_t PY0 = ty * kTileXY + (wave >> 1) * kPatch;
    const int32_t T0 = tt * TT;
    const int32_t X = PX0 + (lane & 7), Y = PY0 + (lane >> 3);
    const float Xc = (float)X + 0.5f, Yc = (float)Y + 0.5f;

    float acc[TT];
    float comp[KAHAN ? TT : 1];
    float pass[KAHAN ? TT : 1];
#pragma unroll
    for (int r = 0; r < TT; ++r) acc[r] = 0.0f;
    if constexpr (KAHAN) {
#pragma unroll
        for (int r = 0; r < TT; ++r) {
            comp[r] = 0.0f;
            pass[r] = 0.0f;
        }
    }

    if (PX0 < a.gx && PY0 < a.gy) {
        // Bins that can hold a point reaching this patch: a point reaches
        // column X only if floor(xr) lies in [X - Hs, X + Hs]; one voxel of
        // margin absorbs rounding of the footprint bounds.
        const int32_t PX1 = PX0 + kPatch - 1, PY1 = PY0 + kPatch - 1, T1 = T0 + TT - 1;
        const int32_t cx0 = clampi(floordiv_d(PX0 - a.Hs - 1, a.cxy), 0, a.ncx - 1);
        const int32_t cx1 = clampi(floordiv_d(PX1 + a.Hs + 1, a.cxy), 0, a.ncx - 1);
        const int32_t cy0 = clampi(floordiv_d(PY0 - a.Hs - 1, a.cxy), 0, a.ncy - 1);
        const int32_t cy1 = clampi(floordiv_d(PY1 + a.Hs + 1, a.cxy), 0, a.ncy - 1);
        const int32_t ct0 = clampi(floordiv_d(T0 - a.Ht - 1, a.ct), 0, a.nct - 1);
        const int32_t ct1 = clampi(floordiv_d(T1 + a.Ht + 1, a.ct), 0, a.nct - 1);

        for (int32_t cz = ct0; cz <= ct1; ++cz) {
            for (int32_t cy = cy0; cy <= cy1; ++cy) {
                const int32_t row = (cz * a.ncy + cy) * a.ncx;
                const int32_t beg = (int32_t)a.cell_start[row + cx0];
                const int32_t end = (int32_t)a.cell_start[row + cx1 + 1];
                for (int32_t base = beg; base < end; base += 64) {
                    const int32_t j = base + lane;
                    bool hit = false;
                    if (j < end) {
                        const uint4 q = reinterpret_cast<const uint4*>(a.recs + j)[1];
                        const int32_t xlo = (int32_t)(q.x & 0xffffu), xhi = (int32_t)(q.x >> 16);
                        const int32_t ylo = (int32_t)(q.y & 0xffffu), yhi = (int32_t)(q.y >> 16);
                        const int32_t tlo = (int32_t)q.z, thi = (int32_t)q.w;
                        hit = xlo <= PX1 && xhi >= PX0 && ylo <= PY1 && yhi >= PY0 && tlo <= T1 &&
                              thi >= T0;
                    }
                    unsigned long long m = __ballot(hit);
                    if (m == 0ull) continue;
                    while (m) {
                        const int b = __builtin_ctzll(m);
                        m &= m - 1ull;
                        const int32_t p = base + b;
                        const PointRec r = a.recs[p];
                        const float dx = (Xc - r.xh) - r.xl;
                        const float dy = (Yc - r.yh) - r.yl;
                        const float ks = fmaxf(0.0f, fmaf(-(dx * dx + dy * dy), a.inv_hv2, 1.0f));
                        // chunks of 4 rows of this tile inside [tlo, thi]
                        const int32_t c0 = max(0, (r.tlo - T0) >> 2);
                        const int32_t c1 = min(NCH - 1, (r.thi - T0) >> 2);
                        const float* ktp = a.kt + (size_t)p * a.ktw - (r.tlo & ~3) + T0;
#pragma unroll
                        for (int c = 0; c < NCH; ++c) {
                            if (c >= c0 && c <= c1) {
                                const float4 k4 = *reinterpret_cast<const float4*>(ktp + 4 * c);
                                if constexpr (KAHAN) {
                                    pass[4 * c + 0] = fmaf(ks, k4.x, pass[4 * c + 0]);
                                    pass[4 * c + 1] = fmaf(ks, k4.y, pass[4 * c + 1]);
                                    pass[4 * c + 2] = fmaf(ks, k4.z, pass[4 * c + 2]);
                                    pass[4 * c + 3] = fmaf(ks, k4.w, pass[4 * c + 3]);
                                } else {
                                    acc[4 * c + 0] = fmaf(ks, k4.x, acc[4 * c + 0]);
                                    acc[4 * c + 1] = fmaf(ks, k4.y, acc[4 * c + 1]);
                                    acc[4 * c + 2] = fmaf(ks, k4.z, acc[4 * c + 2]);
                                    acc[4 * c + 3] = fmaf(ks, k4.w, acc[4 * c + 3]);
                                }
                            }
                        }
                    }
                    if constexpr (KAHAN) kahan_fold<TT>(acc, comp, pass);
                }
            }
        }
    }

    // Store the tile once, FP32, [X][Y][T] with T fastest.
    double msum = 0.0;
    if (X < a.gx && Y < a.gy) {
        float* o = a.out + ((size_t)X * a.gy + Y) * a.gt + T0;
        float v[TT];
#pragma unroll
        for (int r = 0; r < TT; ++r) v[r] = acc[r] * a.cnorm;
        if (T0 + TT <= a.gt && (a.gt & 3) == 0) {
#pragma unroll
            for (int r = 0; r < TT; r += 4)
                *reinterpret_cast<float4*>(o + r) = make_float4(v[r], v[r + 1], v[r + 2], v[r + 3]);
            if constexpr (MASS) {
#pragma unroll
                for (int r = 0; r < TT; ++r) msum += (double)v[r];
            }
        } else {
#pragma unroll
            for (int r = 0; r < TT; ++r) {
                if (T0 + r < a.gt) {
                    o[r] = v[r];
                    if constexpr (MASS) msum += (double)v[r];
                }
            }
        }
    }
    if constexpr (MASS) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) msum += __shfl_xor(msum, d, 64);
        if (lane == 0) a.tile_part[(size_t)tile * kWaves + wave] = msum;
    }
}

// Fixed-order FP64 sum of `count` partials into *dst (times `scale`), by one
// workgroup: strided per-thread sums, then a tree in LDS.
__global__ __launch_bounds__(1024) void k_sum_partials(const double* __restrict__ part,
                                                       int64_t count, double scale,
                                                       double* __restrict__ dst) {
    __shared__ double sh[1024];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < count; i += 1024) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *dst = sh[0] * scale;
}

template <int TT, bool K, bool M>
void launch_one(const GatherArgs& ga, hipStream_t s) {
    hipLaunchKernelGGL((k_gather<TT, K, M>), dim3(ga.ntiles), dim3(kThreads), 0, s, ga);
}

}  // namespace

hipError_t launch_gather(const Geometry& g, float cnorm, bool kahan, bool mass, float* d_out,
                         uint8_t* ws, const Workspace& w, hipStream_t s) {
    GatherArgs ga;
    ga.cell_start = reinterpret_cast<const uint32_t*>(ws + w.cell_start);
    ga.recs = reinterpret_cast<const PointRec*>(ws + w.recs);
    ga.kt = reinterpret_cast<const float*>(ws + w.kt);
    ga.out = d_out;
    ga.tile_part = reinterpret_cast<double*>(ws + w.tile_part);
    ga.gx = g.gx;
    ga.gy = g.gy;
    ga.gt = g.gt;
    ga.Hs = g.Hs;
    ga.Ht = g.Ht;
    ga.cxy = g.cxy;
    ga.ct = g.ct;
    ga.ncx = g.ncx;
    ga.ncy = g.ncy;
    ga.nct = g.nct;
    ga.ntx = g.ntx;
    ga.nty = g.nty;
    ga.ntiles = g.ntiles;
    ga.ktw = g.ktw;
    ga.inv_hv2 = g.inv_hv2;
    ga.cnorm = cnorm;
    if (g.tile_t == 16) {
        if (kahan) mass ? launch_one<16, true, true>(ga, s) : launch_one<16, true, false>(ga, s);
        else mass ? launch_one<16, false, true>(ga, s) : launch_one<16, false, false>(ga, s);
    } else {
        if (kahan) mass ? launch_one<32, true, true>(ga, s) : launch_one<32, true, false>(ga, s);
        else mass ? launch_one<32, false, true>(ga, s) : launch_one<32, false, false>(ga, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipSuccess;
}

hipError_t launch_mass_reduce(const Geometry& g, double* d_dst, uint8_t* ws, const Workspace& w,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, s,
                       reinterpret_cast<const double*>(ws + w.tile_part),
                       (int64_t)g.ntiles * kWaves, g.sres * g.sres * g.tres, d_dst);
    return hipGetLastError();
}

}  // namespace stkde
