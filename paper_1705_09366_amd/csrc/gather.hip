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
//   stage   256 candidates at a time, one per thread: test the point's
//           clipped footprint box against the tile and append the survivors'
//           tile-local coordinates to an LDS list, together with the set of
//           4 x 4 column groups and 16-row blocks its cylinder touches (a
//           disc-versus-group test); repeat until the list is nearly full or
//           the candidates are exhausted;
//   lists   each wave owns an 8 x 8 quadrant (four 4 x 4 column groups) x
//           TT/16 blocks of 16 rows as matrix-core accumulators, and keeps,
//           in list order, the survivors whose footprint box meets its
//           quadrant;
//   mma     per group of 4 consecutive survivors of its list, each lane
//           builds its matrix-core operands in registers -- the Kt entries
//           of one point for one row of every block, and the separable pieces
//           1 - dx^2/hv^2 and dy^2/hv^2 of the Ks entries of one point for its
//           column in each column group, Ks = max(0, 1 - dx^2/hv^2 -
//           dy^2/hv^2) (the Epanechnikov disc), Kt = max(0, 1 - dt^2/tv^2) --
//           and the wave issues one instruction per (column group, row
//           block).  The loop has no branches; the next group's coordinates
//           are fetched while the current group's instructions run;
//   store   each lane writes 4 consecutive rows of one column per block,
//           scaled by the normalisation (2/pi)(3/4)/(n hs^2 ht).
// With compensated accumulation each matrix-core phase (up to kCap points)
// accumulates into a fresh pass accumulator that is then added into
// (sum, compensation) by Kahan's rule; within a pass the sum is plain FP32.
#include "stkde_internal.h"

namespace stkde {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kCap = 1024;  // survivors held in LDS between matrix-core phases

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

template <int TT, bool KAHAN, bool MASS>
__global__ __launch_bounds__(kThreads) void k_gather(GatherArgs a) {
    constexpr int NB = TT / 16;  // 16-row blocks per tile
    constexpr int CG = 4 * NB;   // accumulator blocks per wave
    constexpr int kPad = kCap;   // index of the padding survivor
    // survivor list: tile-local coordinates as (head, tail) pairs and the
    // quadrants its footprint box meets; entry kPad is a point far outside
    // the tile
    __shared__ float2 sX[kCap + 1], sY[kCap + 1], sT[kCap + 1];
    __shared__ uint8_t sQ[kCap];
    // per-wave lists of survivor indices
    __shared__ uint16_t sL[kWaves][kCap + 8];
    __shared__ int32_t sRB[kMaxRanges];
    __shared__ int32_t sRP[kMaxRanges + 1];
    __shared__ int32_t sWC[kWaves];

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
    if (tid == 0) {
        sX[kPad] = make_float2(-1.0e6f, 0.f);
        sY[kPad] = make_float2(-1.0e6f, 0.f);
        sT[kPad] = make_float2(-1.0e6f, 0.f);
    }
    __syncthreads();
    const int32_t total = sRP[nranges];

    // ---- accumulators: [column group q][row block b] ------------------------
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
    // this wave's quadrant: column groups gx in {gqx, gqx + 1}, gy in {gqy, gqy + 1}
    const int gqx = 2 * (wave & 1), gqy = 2 * (wave >> 1);
    const int32_t QX0 = X0 + 4 * gqx, QY0 = Y0 + 4 * gqy;
    const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    // lane roles in the matrix-core operands: point k of the group, row i of
    // a block (Kt operand), column j = (lane & 3, (lane >> 2) & 3) of a column
    // group (Ks operand)
    const int kq = lane >> 4;
    const float rowc = (float)(lane & 15) + 0.5f;
    const float xc0 = (float)(4 * gqx + (lane & 3)) + 0.5f;
    const float yc0 = (float)(4 * gqy + ((lane >> 2) & 3)) + 0.5f;
    uint16_t* myL = sL[wave];

    // one group: operands from the coordinates of this lane's point, then
    // all CG instructions
    auto group = [&](const float2 cx, const float2 cy, const float2 ctt) {
        float av[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const float dt = ((rowc + 16.0f * b) - ctt.x) - ctt.y;
            av[b] = fmaxf(0.0f, fmaf(-dt * dt, a.inv_tv2, 1.0f));
        }
        float ux[2], uy[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const float dx = ((xc0 + 4.0f * h) - cx.x) - cx.y;
            const float dy = ((yc0 + 4.0f * h) - cy.x) - cy.y;
            ux[h] = fmaf(-dx * dx, a.inv_hv2, 1.0f);
            uy[h] = dy * dy * a.inv_hv2;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float ks = fmaxf(0.0f, ux[q & 1] - uy[q >> 1]);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if constexpr (KAHAN)
                    pass[q * NB + b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[b], ks, pass[q * NB + b], 0, 0, 0);
                else
                    acc[q * NB + b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[b], ks, acc[q * NB + b], 0, 0, 0);
            }
        }
    };

    int32_t bb = 0;
    while (bb < total) {
        // ---- stage: fill the survivor list ---------------------------------
        int32_t count = 0;
        while (bb < total && count <= kCap - kThreads) {
            const int32_t c = bb + tid;
            bool surv = false;
            PointRec r{};
            uint32_t qm = 0;
            if (c < total) {
                int32_t lo = 0, hi = nranges - 1;  // last range with sRP <= c
                while (lo < hi) {
                    const int32_t mid = (lo + hi + 1) >> 1;
                    if (sRP[mid] <= c) lo = mid;
                    else hi = mid - 1;
                }
                r = a.recs[sRB[lo] + (c - sRP[lo])];
                const int32_t xlo = (int32_t)(r.xb & 0xffffu) - X0, xhi = (int32_t)(r.xb >> 16) - X0;
                const int32_t ylo = (int32_t)(r.yb & 0xffffu) - Y0, yhi = (int32_t)(r.yb >> 16) - Y0;
                const int32_t tlo = (int32_t)(r.tb & 0xffffu), thi = (int32_t)(r.tb >> 16);
                if (tlo <= T0 + TT - 1 && thi >= T0) {
                    // quadrants (qx, qy) whose 8 x 8 columns the footprint box meets
                    const bool x0 = xlo <= 7 && xhi >= 0, x1 = xlo <= 15 && xhi >= 8;
                    const bool y0 = ylo <= 7 && yhi >= 0, y1 = ylo <= 15 && yhi >= 8;
                    qm = (uint32_t)(x0 && y0) | ((uint32_t)(x1 && y0) << 1) |
                         ((uint32_t)(x0 && y1) << 2) | ((uint32_t)(x1 && y1) << 3);
                }
                surv = qm != 0;
            }
            const unsigned long long m = __ballot(surv);
            if (lane == 0) sWC[wave] = __popcll(m);
            __syncthreads();
            int32_t off = count, add = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const int32_t cw = sWC[w];
                off += (w < wave) ? cw : 0;
                add += cw;
            }
            if (surv) {
                const int s = off + __popcll(m & lt);
                // head - origin is exact for the offsets that reach the tile
                sX[s] = make_float2(r.xh - (float)X0, half_lo(r.xl_yl));
                sY[s] = make_float2(r.yh - (float)Y0, half_hi(r.xl_yl));
                sT[s] = make_float2(r.th - (float)T0, half_lo(r.tl));
                sQ[s] = (uint8_t)qm;
            }
            count += add;
            bb += kThreads;
            __syncthreads();  // sWC is rewritten by the next round
        }

        // ---- this wave's list: survivors meeting its quadrant ---------------
        int32_t nw = 0;
        for (int32_t base = 0; base < count; base += 64) {
            const int32_t s = base + lane;
            const bool mine = s < count && ((sQ[s] >> wave) & 1u);
            const unsigned long long bm = __ballot(mine);
            if (mine) myL[nw + __popcll(bm & lt)] = (uint16_t)s;
            nw += __popcll(bm);
        }
        // pad to a whole number of pairs of groups
        if (lane < ((8 - (nw & 7)) & 7)) myL[nw + lane] = (uint16_t)kPad;
        const int32_t npairs = (nw + 7) >> 3;

        // ---- matrix-core accumulation, two groups per iteration -------------
        if (npairs > 0) {
            int s = myL[kq];
            float2 ax = sX[s], ay = sY[s], at = sT[s];
            for (int32_t pr = 0; pr < npairs; ++pr) {
                s = myL[8 * pr + 4 + kq];
                const float2 bx = sX[s], by = sY[s], bt = sT[s];
                group(ax, ay, at);
                if (pr + 1 < npairs) {
                    s = myL[8 * pr + 8 + kq];
                    ax = sX[s];
                    ay = sY[s];
                    at = sT[s];
                }
                group(bx, by, bt);
            }
        }
        if constexpr (KAHAN) kahan_fold<CG>(acc, comp, pass);
        __syncthreads();  // the lists are refilled next
    }

    // ---- store: lane holds rows 16 b + 4 (lane / 16) + e of column
    // (lane % 4, (lane / 4) % 4) of each of its column groups -------------------
    double msum = 0.0;
    const bool vec = (a.gt & 3) == 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int32_t X = QX0 + 4 * (q & 1) + (lane & 3);
        const int32_t Y = QY0 + 4 * (q >> 1) + ((lane >> 2) & 3);
        if (X >= a.gx || Y >= a.gy) continue;
        float* col = a.out + ((size_t)X * a.gy + Y) * a.gt;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int32_t T = T0 + 16 * b + 4 * (lane >> 4);
            const f32x4 v = acc[q * NB + b] * a.cnorm;
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
