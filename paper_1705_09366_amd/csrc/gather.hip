// gather.hip -- the density accumulation of PB-SYM (Sec. 3.2) as an
// atomic-free gather over output tiles, on the FP32 matrix cores.
//
// PB-SYM adds, for every point, the outer product of a spatial table
// Ks[X][Y] and a temporal table Kt[T] into the grid.  Restricted to one tile
// of the grid this is a rank-k update
//
//     out[T][XY] += sum_p Kt[T][p] * Ks[p][XY]
//
// over the k points whose cylinder meets the tile, i.e. a dense contraction
// over points, which maps onto v_mfma_f32_16x16x4f32 (16 rows x 16 columns,
// 4 points per instruction).  Every voxel is owned by exactly one lane of
// one workgroup, which sums all contributions in a fixed order (bins in
// order, points in sorted order within a bin, four at a time) and stores the
// result once; there is no zeroing pass and no read-modify-write of the
// grid.
//
// Per workgroup (256 threads) and 16 x 16 x TT tile:
//   setup   the bin rows (t, y) whose bins can hold points reaching the tile
//           become a list of candidate ranges in LDS;
//   stage   128 candidates at a time, one per thread of the first two waves:
//           test the point's clipped footprint box against the tile; each
//           survivor writes its PB-SYM tables for this tile into LDS -- the
//           temporal table Kt[T] = max(0, 1 - dt^2/tv^2) over the tile rows
//           and the separable pieces of the spatial table, AX[X] =
//           1 - dx^2/hv^2 and BY[Y] = dy^2/hv^2 (Ks = max(0, AX - BY), the
//           Epanechnikov disc) -- and the set of blocks (4 x 4 columns x 16
//           rows) its cylinder reaches; repeat while the list has room;
//   lists   each wave owns 4 x TT/16 blocks (its 8 x 8 quadrant of columns
//           times every 16-row block) as matrix-core accumulators and builds,
//           for each block, the ordered list of survivors that reach it;
//   mma     for each block, per group of 4 consecutive survivors of its list
//           each lane reads its operands from the tables -- Kt of one
//           (point, row) and Ks of one (point, column) -- and the wave issues
//           one v_mfma_f32_16x16x4f32; the next group's operands are read
//           while the current instruction runs;
//   store   each lane writes 4 consecutive rows of one column per block,
//           scaled by the normalisation (2/pi)(3/4)/(n hs^2 ht).
// With compensated accumulation each matrix-core phase accumulates into a
// fresh pass accumulator that is then added into (sum, compensation) by
// Kahan's rule; within a pass the sum is plain FP32.
#include "stkde_internal.h"

namespace stkde {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kCap = 255;     // survivors per matrix-core phase (8-bit list entries)
constexpr int kRound = 128;   // candidates tested per staging round

struct GatherArgs {
    const uint32_t* cell_start;
    const PointRec* recs;
    float* out;
    double* tile_part;
    int32_t gx, gy, gt;
    int32_t Hs, Ht;
    int32_t cxy, ct, ncx, ncy, nct;
    int32_t ntx, nty, ntiles;
    float hv, inv_hv2, inv_tv2;
    float cnorm;
};

__device__ inline int32_t floordiv_d(int32_t a, int32_t b) {
    const int32_t q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}

__device__ inline int32_t clampi(int32_t v, int32_t lo, int32_t hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

__device__ inline float half_lo(uint32_t v) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(v & 0xffffu));
}

__device__ inline float half_hi(uint32_t v) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(v >> 16));
}


template <int CG>
__device__ inline void kahan_fold(f32x4 (&acc)[CG], f32x4 (&comp)[CG], f32x4 (&pass)[CG]) {
#pragma unroll
    for (int q = 0; q < CG; ++q) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float y = __fsub_rn(pass[q][e], comp[q][e]);
            const float t = __fadd_rn(acc[q][e], y);
            comp[q][e] = __fsub_rn(__fsub_rn(t, acc[q][e]), y);
            acc[q][e] = t;
            pass[q][e] = 0.0f;
        }
    }
}

// Bit (g * NB + b): the cylinder of a point at tile-local (px, py) with rows
// [tlo, thi] (tile-local) reaches a column centre of column group g (4 x 4
// columns, g = 4 gy + gx) and a row of block b.
template <int NB>
__device__ inline uint64_t touch_mask(float px, float py, int32_t tlo, int32_t thi, float inv_hv2) {
    const int32_t b0 = max(0, tlo >> 4), b1 = min(NB - 1, thi >> 4);
    const uint64_t rb = (uint64_t)(((1u << (b1 + 1)) - 1u) & ~((1u << b0) - 1u));
    float ex[4], ey[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float nx = fminf(fmaxf(px, 4.0f * k + 0.5f), 4.0f * k + 3.5f) - px;
        const float ny = fminf(fmaxf(py, 4.0f * k + 0.5f), 4.0f * k + 3.5f) - py;
        ex[k] = nx * nx * inv_hv2;
        ey[k] = ny * ny * inv_hv2;
    }
    uint64_t m = 0;
#pragma unroll
    for (int g = 0; g < 16; ++g)
        if (ex[g & 3] + ey[g >> 2] < 1.0f + 1e-3f) m |= rb << (g * NB);
    return m;
}

template <int TT, bool KAHAN, bool MASS>
__global__ __launch_bounds__(kThreads, 2) void k_gather(GatherArgs a) {
    constexpr int NB = TT / 16;   // 16-row blocks per tile
    constexpr int CG = 4 * NB;    // blocks (accumulators) per wave
    constexpr int kZero = kCap;   // table row of zeros, used to pad groups
    constexpr int kTW = TT + 32;  // floats per survivor: Kt[TT], AX[16], BY[16]
    constexpr int kLL = kCap + 4; // entries per block list
    __shared__ __align__(16) float sTab[(kCap + 1) * kTW];
    __shared__ uint64_t sM[kCap];
    __shared__ uint8_t sL[kWaves][CG][kLL];
    __shared__ int32_t sRB[kMaxRanges];
    __shared__ int32_t sRP[kMaxRanges + 1];
    __shared__ int32_t sWC[2];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    // Tiles are dealt to the 8 XCDs in contiguous ranges (workgroup i runs on
    // XCD i mod 8) so that neighbouring tiles, which read the same bins,
    // share an L2.
    const int32_t bid = blockIdx.x;
    const int32_t per = a.ntiles >> 3, rem = a.ntiles & 7;
    const int32_t xcd = bid & 7, slot_in_xcd = bid >> 3;
    const int32_t tile = xcd * per + min(xcd, rem) + slot_in_xcd;
    const int32_t tx = tile % a.ntx;
    const int32_t rest = tile / a.ntx;
    const int32_t ty = rest % a.nty;
    const int32_t tt = rest / a.nty;
    const int32_t X0 = tx * kTileXY, Y0 = ty * kTileXY, T0 = tt * TT;

    // ---- setup: candidate ranges ------------------------------------------
    // A point reaches column X only if floor(xr) lies in [X - Hs, X + Hs]; one
    // voxel of margin absorbs rounding of the footprint bounds.
    const int32_t cx0 = clampi(floordiv_d(X0 - a.Hs - 1, a.cxy), 0, a.ncx - 1);
    const int32_t cx1 = clampi(floordiv_d(X0 + kTileXY - 1 + a.Hs + 1, a.cxy), 0, a.ncx - 1);
    const int32_t cy0 = clampi(floordiv_d(Y0 - a.Hs - 1, a.cxy), 0, a.ncy - 1);
    const int32_t cy1 = clampi(floordiv_d(Y0 + kTileXY - 1 + a.Hs + 1, a.cxy), 0, a.ncy - 1);
    const int32_t ct0 = clampi(floordiv_d(T0 - a.Ht - 1, a.ct), 0, a.nct - 1);
    const int32_t ct1 = clampi(floordiv_d(T0 + TT - 1 + a.Ht + 1, a.ct), 0, a.nct - 1);
    const int32_t nyr = cy1 - cy0 + 1;
    const int32_t nranges = nyr * (ct1 - ct0 + 1);  // <= kMaxRanges (the plan guarantees it)
    if (wave == 0) {
        int32_t beg = 0, len = 0;
        if (lane < nranges) {
            const int32_t cz = ct0 + lane / nyr, cy = cy0 + lane % nyr;
            const int32_t row = (cz * a.ncy + cy) * a.ncx;
            beg = (int32_t)a.cell_start[row + cx0];
            len = (int32_t)a.cell_start[row + cx1 + 1] - beg;
        }
        int32_t inc = len;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t o = __shfl_up(inc, d, 64);
            if (lane >= d) inc += o;
        }
        if (lane < nranges) {
            sRB[lane] = beg;
            sRP[lane] = inc - len;
        }
        if (lane == nranges - 1) sRP[nranges] = inc;
    }
    if (tid < kTW) sTab[kZero * kTW + tid] = 0.0f;
    __syncthreads();
    const int32_t total = sRP[nranges];

    // ---- accumulators: block q * NB + b = (column group q of the quadrant,
    // row block b) --------------------------------------------------------------
    f32x4 acc[CG];
    f32x4 comp[KAHAN ? CG : 1];
    f32x4 pass[KAHAN ? CG : 1];
#pragma unroll
    for (int q = 0; q < CG; ++q) {
        acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (KAHAN) {
            comp[q] = f32x4{0.f, 0.f, 0.f, 0.f};
            pass[q] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    }
    const int gqx = 2 * (wave & 1), gqy = 2 * (wave >> 1);
    const int32_t QX0 = X0 + 4 * gqx, QY0 = Y0 + 4 * gqy;
    const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    // lane roles: point k of the group; row i of the block (Kt operand);
    // column (lane & 3, (lane >> 2) & 3) of the column group (Ks operand)
    const int kq = lane >> 4, ri = lane & 15;
    const int jx = lane & 3, jy = (lane >> 2) & 3;

    int32_t bb = 0;
    while (bb < total) {
        // ---- stage ---------------------------------------------------------
        int32_t count = 0;
        while (bb < total && count <= kCap - kRound) {
            const int32_t c = bb + tid;
            bool surv = false;
            PointRec r{};
            if (tid < kRound && c < total) {
                int32_t lo = 0, hi = nranges - 1;  // last range with sRP <= c
                while (lo < hi) {
                    const int32_t mid = (lo + hi + 1) >> 1;
                    if (sRP[mid] <= c) lo = mid;
                    else hi = mid - 1;
                }
                r = a.recs[sRB[lo] + (c - sRP[lo])];
                const int32_t xlo = (int32_t)(r.xb & 0xffffu), xhi = (int32_t)(r.xb >> 16);
                const int32_t ylo = (int32_t)(r.yb & 0xffffu), yhi = (int32_t)(r.yb >> 16);
                const int32_t tlo = (int32_t)(r.tb & 0xffffu), thi = (int32_t)(r.tb >> 16);
                surv = xlo <= X0 + kTileXY - 1 && xhi >= X0 && ylo <= Y0 + kTileXY - 1 &&
                       yhi >= Y0 && tlo <= T0 + TT - 1 && thi >= T0;
            }
            if (wave < 2) {
                const unsigned long long m = __ballot(surv);
                if (lane == 0) sWC[wave] = __popcll(m);
                __syncthreads();
                const int32_t add = sWC[0] + sWC[1];
                if (surv) {
                    const int s = count + (wave ? sWC[0] : 0) + __popcll(m & lt);
                    // head - origin is exact for the offsets that reach the tile
                    const float pxh = r.xh - (float)X0, pxl = half_lo(r.xl_yl);
                    const float pyh = r.yh - (float)Y0, pyl = half_hi(r.xl_yl);
                    const float pth = r.th - (float)T0, ptl = half_lo(r.tl);
                    float* tb = sTab + s * kTW;
#pragma unroll
                    for (int rr = 0; rr < TT; rr += 4) {
                        float v[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const float dt = ((float)(rr + e) + 0.5f - pth) - ptl;
                            v[e] = fmaxf(0.0f, fmaf(-dt * dt, a.inv_tv2, 1.0f));
                        }
                        *reinterpret_cast<float4*>(tb + rr) = make_float4(v[0], v[1], v[2], v[3]);
                    }
#pragma unroll
                    for (int k = 0; k < 16; k += 4) {
                        float u[4], w[4];
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const float dx = ((float)(k + e) + 0.5f - pxh) - pxl;
                            const float dy = ((float)(k + e) + 0.5f - pyh) - pyl;
                            u[e] = fmaf(-dx * dx, a.inv_hv2, 1.0f);
                            w[e] = dy * dy * a.inv_hv2;
                        }
                        *reinterpret_cast<float4*>(tb + TT + k) = make_float4(u[0], u[1], u[2], u[3]);
                        *reinterpret_cast<float4*>(tb + TT + 16 + k) = make_float4(w[0], w[1], w[2], w[3]);
                    }
                    sM[s] = touch_mask<NB>(pxh + pxl, pyh + pyl, (int32_t)(r.tb & 0xffffu) - T0,
                                           (int32_t)(r.tb >> 16) - T0, a.inv_hv2);
                }
                count += add;
            } else {
                __syncthreads();
                count += sWC[0] + sWC[1];
            }
            bb += kRound;
            __syncthreads();  // sWC is rewritten by the next round
        }

        // ---- per-block lists of this wave -----------------------------------
        int32_t nl[CG];
#pragma unroll
        for (int q = 0; q < CG; ++q) nl[q] = 0;
        for (int32_t base = 0; base < count; base += 64) {
            const int32_t s = base + lane;
            const uint64_t mk = s < count ? sM[s] : 0ull;
#pragma unroll
            for (int q = 0; q < CG; ++q) {
                const int g = (gqy + ((q / NB) >> 1)) * 4 + gqx + ((q / NB) & 1);
                const bool hit = (mk >> (g * NB + (q % NB))) & 1ull;
                const unsigned long long bm = __ballot(hit);
                if (hit) sL[wave][q][nl[q] + __popcll(bm & lt)] = (uint8_t)s;
                nl[q] += __popcll(bm);
            }
        }
#pragma unroll
        for (int q = 0; q < CG; ++q)
            if (lane < ((4 - (nl[q] & 3)) & 3)) sL[wave][q][nl[q] + lane] = (uint8_t)kZero;

        // ---- matrix-core accumulation, block by block -----------------------
#pragma unroll
        for (int q = 0; q < CG; ++q) {
            const int cq = q / NB, b = q % NB;
            const int gx = gqx + (cq & 1), gy = gqy + (cq >> 1);
            const int ngr = (nl[q] + 3) >> 2;
            const uint8_t* L = sL[wave][q];
            const int offA = 16 * b + ri, offX = TT + 4 * gx + jx, offY = TT + 16 + 4 * gy + jy;
            float an = 0.f, xn = 0.f, yn = 0.f;
            if (ngr > 0) {
                const float* tb = sTab + (int)L[kq] * kTW;
                an = tb[offA];
                xn = tb[offX];
                yn = tb[offY];
            }
            for (int g = 0; g < ngr; ++g) {
                const float av = an, ks = fmaxf(0.0f, xn - yn);
                if (g + 1 < ngr) {
                    const float* tb = sTab + (int)L[4 * (g + 1) + kq] * kTW;
                    an = tb[offA];
                    xn = tb[offX];
                    yn = tb[offY];
                }
                if constexpr (KAHAN)
                    pass[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, ks, pass[q], 0, 0, 0);
                else
                    acc[q] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, ks, acc[q], 0, 0, 0);
            }
        }
        if constexpr (KAHAN) kahan_fold<CG>(acc, comp, pass);
        __syncthreads();  // tables and lists are refilled next
    }

    // ---- store: lane holds rows 16 b + 4 (lane / 16) + e of column
    // (lane % 4, (lane / 4) % 4) of each of its blocks ---------------------------
    double msum = 0.0;
    const bool vec = (a.gt & 3) == 0;
#pragma unroll
    for (int cq = 0; cq < 4; ++cq) {
        const int32_t X = QX0 + 4 * (cq & 1) + jx;
        const int32_t Y = QY0 + 4 * (cq >> 1) + jy;
        if (X >= a.gx || Y >= a.gy) continue;
        float* col = a.out + ((size_t)X * a.gy + Y) * a.gt;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int32_t T = T0 + 16 * b + 4 * kq;
            const f32x4 v = acc[cq * NB + b] * a.cnorm;
            if (vec && T + 3 < a.gt) {
                *reinterpret_cast<f32x4*>(col + T) = v;
                if constexpr (MASS) msum += (double)v[0] + (double)v[1] + (double)v[2] + (double)v[3];
            } else {
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    if (T + e < a.gt) {
                        col[T + e] = v[e];
                        if constexpr (MASS) msum += (double)v[e];
                    }
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

// Fixed-order FP64 sum of `count` partials: workgroup b sums the contiguous
// chunk b (strided per-thread sums, then a tree in LDS) and writes
// dst[b] = chunk sum * scale.
__global__ __launch_bounds__(1024) void k_sum_partials(const double* __restrict__ part,
                                                       int64_t count, double scale,
                                                       double* __restrict__ dst) {
    __shared__ double sh[1024];
    const int64_t chunk = (count + gridDim.x - 1) / gridDim.x;
    const int64_t beg = (int64_t)blockIdx.x * chunk;
    const int64_t end = beg + chunk < count ? beg + chunk : count;
    double s = 0.0;
    for (int64_t i = beg + threadIdx.x; i < end; i += 1024) s += part[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) dst[blockIdx.x] = sh[0] * scale;
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
    ga.hv = (float)g.hv;
    ga.inv_hv2 = g.inv_hv2;
    ga.inv_tv2 = g.inv_tv2;
    ga.cnorm = cnorm;
    if (g.tile_t == 16) {
        if (kahan) mass ? launch_one<16, true, true>(ga, s) : launch_one<16, true, false>(ga, s);
        else mass ? launch_one<16, false, true>(ga, s) : launch_one<16, false, false>(ga, s);
    } else if (g.tile_t == 32) {
        if (kahan) mass ? launch_one<32, true, true>(ga, s) : launch_one<32, true, false>(ga, s);
        else mass ? launch_one<32, false, true>(ga, s) : launch_one<32, false, false>(ga, s);
    } else {
        if (kahan) mass ? launch_one<64, true, true>(ga, s) : launch_one<64, true, false>(ga, s);
        else mass ? launch_one<64, false, true>(ga, s) : launch_one<64, false, false>(ga, s);
    }
    return hipGetLastError();
}

hipError_t launch_mass_reduce(const Geometry& g, double* d_dst, uint8_t* ws, const Workspace& w,
                              hipStream_t s) {
    double* mid = reinterpret_cast<double*>(ws + w.mass_part);
    hipLaunchKernelGGL(k_sum_partials, dim3(kMassBlocks), dim3(1024), 0, s,
                       reinterpret_cast<const double*>(ws + w.tile_part),
                       (int64_t)g.ntiles * kWaves, 1.0, mid);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1024), 0, s, (const double*)mid,
                       (int64_t)kMassBlocks, g.sres * g.sres * g.tres, d_dst);
    return hipGetLastError();
}

}  // namespace stkde
