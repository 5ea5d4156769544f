// ablation.hip -- two baselines that the tile gather is measured against.
// They compute the same estimate from the same binned records, so their
// difference from the gather is the design alone:
//
//  * scatter: the point-based algorithm PB (Sec. 3.1) run point-parallel, one
//    workgroup per point, adding every contribution into the grid with a
//    hardware FP32 atomic after a zeroing pass.  This is the write race that
//    the paper's decompositions exist to avoid (Sec. 4.1); on a GPU the atomics
//    resolve it, at the price of a zeroing pass, one atomic per (voxel, point)
//    pair and a summation order that changes from run to run.
//  * voxel: the voxel-based algorithm with points partitioned into
//    bandwidth-sized blocks, VB-DEC (Sec. 3), one thread per voxel reading the
//    points of the bins within reach -- the voxel-based shape of earlier GPU
//    estimators (Sec. 7).  Deterministic, no atomics, but every voxel tests
//    every point of its neighbouring bins.
#include "stkde_internal.h"

namespace stkde {
namespace {

__device__ inline float half_lo_a(uint32_t v) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(v & 0xffffu));
}

__device__ inline float half_hi_a(uint32_t v) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(v >> 16));
}

__global__ __launch_bounds__(256) void k_fill_zero(float* __restrict__ out, size_t count) {
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256)
        out[i] = 0.0f;
}

// One workgroup per valid point (grid-stride); its threads walk the point's
// clipped footprint box, T fastest.
__global__ __launch_bounds__(256) void k_scatter_points(const PointRec* __restrict__ recs,
                                                        const uint32_t* __restrict__ cell_start,
                                                        int32_t ncell, int32_t gx, int32_t gy,
                                                        int32_t gt, float inv_hv2, float inv_tv2,
                                                        float cnorm, float* __restrict__ out) {
    const uint32_t nvalid = cell_start[ncell];
    for (uint32_t p = blockIdx.x; p < nvalid; p += gridDim.x) {
        const PointRec r = recs[p];
        const int32_t xlo = (int32_t)(r.xb & 0xffffu), xhi = (int32_t)(r.xb >> 16);
        const int32_t ylo = (int32_t)(r.yb & 0xffffu), yhi = (int32_t)(r.yb >> 16);
        const int32_t tlo = (int32_t)(r.tb & 0xffffu), thi = (int32_t)(r.tb >> 16);
        const int32_t nx = min(xhi, gx - 1) - xlo + 1, ny = min(yhi, gy - 1) - ylo + 1;
        const int32_t nt = min(thi, gt - 1) - tlo + 1;
        if (nx <= 0 || ny <= 0 || nt <= 0) continue;
        const float xt = half_lo_a(r.xl_yl), yt = half_hi_a(r.xl_yl), tt = half_lo_a(r.tl);
        const int32_t vol = nx * ny * nt;
        for (int32_t v = threadIdx.x; v < vol; v += 256) {
            const int32_t T = tlo + v % nt;
            const int32_t rest = v / nt;
            const int32_t Y = ylo + rest % ny;
            const int32_t X = xlo + rest / ny;
            const float dx = (((float)X + 0.5f) - r.xh) - xt;
            const float dy = (((float)Y + 0.5f) - r.yh) - yt;
            const float dt = (((float)T + 0.5f) - r.th) - tt;
            const float ks = 1.0f - (dx * dx + dy * dy) * inv_hv2;
            const float kt = 1.0f - dt * dt * inv_tv2;
            if (ks > 0.0f && kt >= 0.0f)
                unsafeAtomicAdd(&out[((size_t)X * gy + Y) * gt + T], cnorm * ks * kt);
        }
    }
}

// One thread per voxel, T fastest: every point of the bins within Hs / Ht
// (plus one voxel of margin) of the voxel, in bin order.
__global__ __launch_bounds__(256) void k_voxel_gather(const PointRec* __restrict__ recs,
                                                      const uint32_t* __restrict__ cell_start,
                                                      SetGeom sg, int32_t Hs, int32_t Ht,
                                                      float inv_hv2, float inv_tv2, float cnorm,
                                                      float* __restrict__ out) {
    const size_t nvox = (size_t)sg.gx * sg.gy * sg.gt;
    const size_t v = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= nvox) return;
    const int32_t T = (int32_t)(v % sg.gt);
    const size_t rest = v / sg.gt;
    const int32_t Y = (int32_t)(rest % sg.gy);
    const int32_t X = (int32_t)(rest / sg.gy);
    const int32_t cx0 = clamp_i32(floordiv_i(X - Hs - 1, sg.cx), 0, sg.ncx - 1);
    const int32_t cx1 = clamp_i32(floordiv_i(X + Hs + 1, sg.cx), 0, sg.ncx - 1);
    const int32_t cy0 = clamp_i32(floordiv_i(Y - Hs - 1, sg.cxy), 0, sg.ncy - 1);
    const int32_t cy1 = clamp_i32(floordiv_i(Y + Hs + 1, sg.cxy), 0, sg.ncy - 1);
    const int32_t ct0 = clamp_i32(floordiv_i(T - Ht - 1, sg.ct), 0, sg.nct - 1);
    const int32_t ct1 = clamp_i32(floordiv_i(T + Ht + 1, sg.ct), 0, sg.nct - 1);
    const float xc = (float)X + 0.5f, yc = (float)Y + 0.5f, tc = (float)T + 0.5f;
    float sum = 0.0f;
    for (int32_t cz = ct0; cz <= ct1; ++cz) {
        for (int32_t cy = cy0; cy <= cy1; ++cy) {
            const int32_t row = (cz * sg.ncy + cy) * sg.ncx;
            const uint32_t b = cell_start[row + cx0], e = cell_start[row + cx1 + 1];
            for (uint32_t p = b; p < e; ++p) {
                const PointRec r = recs[p];
                const float dx = (xc - r.xh) - half_lo_a(r.xl_yl);
                const float dy = (yc - r.yh) - half_hi_a(r.xl_yl);
                const float dt = (tc - r.th) - half_lo_a(r.tl);
                const float ks = 1.0f - (dx * dx + dy * dy) * inv_hv2;
                const float kt = 1.0f - dt * dt * inv_tv2;
                if (ks > 0.0f && kt >= 0.0f) sum += ks * kt;
            }
        }
    }
    out[v] = sum * cnorm;
}

}  // namespace

hipError_t launch_ablation_scatter(const SetGeom& sg, const InstGeom& ig, const uint8_t* set,
                                   const SetLayout& sl, float cnorm, float* d_out, hipStream_t s) {
    const size_t nvox = (size_t)ig.gx * ig.gy * ig.gt;
    hipLaunchKernelGGL(k_fill_zero, dim3(4096), dim3(256), 0, s, d_out, nvox);
    hipLaunchKernelGGL(k_scatter_points, dim3(65536), dim3(256), 0, s,
                       reinterpret_cast<const PointRec*>(set + sl.recs),
                       reinterpret_cast<const uint32_t*>(set + sl.cell_start), sg.ncell, ig.gx, ig.gy,
                       ig.gt, ig.inv_hv2, ig.inv_tv2, cnorm, d_out);
    return hipGetLastError();
}

hipError_t launch_ablation_voxel(const SetGeom& sg, const InstGeom& ig, const uint8_t* set,
                                 const SetLayout& sl, float cnorm, float* d_out, hipStream_t s) {
    const size_t nvox = (size_t)sg.gx * sg.gy * sg.gt;
    const size_t nb = (nvox + 255) / 256;
    hipLaunchKernelGGL(k_voxel_gather, dim3((uint32_t)nb), dim3(256), 0, s,
                       reinterpret_cast<const PointRec*>(set + sl.recs),
                       reinterpret_cast<const uint32_t*>(set + sl.cell_start), sg, ig.Hs, ig.Ht,
                       ig.inv_hv2, ig.inv_tv2, cnorm, d_out);
    return hipGetLastError();
}

}  // namespace stkde
