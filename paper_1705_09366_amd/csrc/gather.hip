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
// Scheduling.  The kernel is persistent: each workgroup takes work items --
// a tile, or one part of a tile whose candidate sequence was split into
// contiguous ranges -- first from the heaviest-first queue (the costliest
// tiles, longest processing time first), then from the spatial queue: every
// tile of every instance with t fastest, minus those the first queue took,
// so that the tiles in flight at any time are neighbours that read the same
// bins.  Each queue is served by interleaved counters that only grow, so
// every workgroup leaves after one failed fetch per counter.  One launch serves any number of
// instances (grids with their own bandwidths and windows over their own
// binned sets).
//
// Per work item (256 threads, 16 x 16 x TT tile):
//   setup   the bin rows (t, y) whose bins can hold points reaching the tile
//           become a list of candidate ranges in LDS;
//   stage   256 candidates at a time, one per thread: test the point's
//           clipped footprint box against the tile, and its disc against the
//           tile's four 8 x 8 quadrants, and append the survivors' tile-local
//           coordinates to an LDS list, together with the set of quadrants
//           its disc reaches; repeat until the list is nearly full or the
//           candidates are exhausted;
//   lists   each wave owns an 8 x 8 quadrant (four 4 x 4 column groups) x
//           TT/16 blocks of 16 rows as matrix-core accumulators, and keeps,
//           in list order, the survivors whose disc reaches its
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
//           scaled by the normalisation (2/pi)(3/4)/(n hs^2 ht); a part of a
//           split tile writes its unscaled sums to a partial slot instead,
//           and the split reduction adds the parts in part order.
// With compensated accumulation each matrix-core phase (up to kCap points)
// accumulates into a fresh pass accumulator that is then added into
// (sum, compensation) by Kahan's rule; within a pass the sum is plain FP32.
//
// Two-term FP16 operands (variant H16: the Epanechnikov pair, one bandwidth
// pair, no full-cover path, 16- or 32-row tiles).  The FP32 operands above
// are built the same way, then each is written as hi + lo with hi its FP16
// truncation and lo the FP16 truncation of the exact remainder, and the
// product as hi*hi + hi*lo + lo*hi on v_mfma_f32_16x16x32_f16 (32 points per
// instruction, FP32 accumulation) -- the splitting scheme of Markidis et al.
// (2018) and Ootomo and Yokota (2022) for FP32 products on half-precision
// matrix units.  Each operand keeps 22 significant bits (truncation error
// below 2^-21 of its value; below 2^-24 absolute where lo falls in FP16's
// subnormal range, which the matrix cores honour), the dropped lo*lo term is
// below 2^-20 of the product, so a product is low by less than 2^-19 of
// itself, and all products are non-negative, so every voxel's sum is too,
// beyond its FP32 accumulation error.  The three instructions cost 3/16 of
// the FP32 form's matrix-core time per point; operand construction (VALU)
// bounds the loop instead.
#include <atomic>

#include "stkde_internal.h"

namespace stkde {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// survivors held in LDS between matrix-core phases: FP32-operand kernels, and
// two-term FP16 kernels (at most four workgroups per compute unit, as their
// registers allow; fewer phases, so fewer Kahan folds and scratch round trips)
constexpr int kCapF32 = 768;
constexpr int kCapH16 = 1152;
// Survivor mask: bits 0..3 the quadrants its footprint box meets but its disc
// does not cover (full-cover kernels: covers every column centre, with a
// margin), bits 4..7 the quadrants it covers; all four covered = the whole
// tile.
constexpr uint32_t kCoverAll = 0xF0u;
constexpr float kFullMargin = 0.99998f;    // largest a + b at a tile corner for that
// A quadrant whose nearest column centre lies farther than the disc's radius
// (beyond 1.0001 hv^2, after moving the point 0.001 voxel closer) holds no
// evaluation of the point: its FP32 operands there are 0 by a wide margin.
constexpr float kCullMargin = 1.0001f;
constexpr int kMaxDevices = 64;
// Pairs that are not zero on their support boundary decide membership near it
// in FP64: within this band of the FP32 test (|1 - u^2 - v^2| or |w^2 - 1|),
// far wider than its rounding, the record's FP64 coordinates are read.
constexpr float kExactBand = 1.0e-4f;

__device__ inline float half_lo(uint32_t v) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(v & 0xffffu));
}

__device__ inline float half_hi(uint32_t v) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(v >> 16));
}

typedef _Float16 h16x8 __attribute__((ext_vector_type(8)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// x = hi + lo + e and y likewise, hi and lo packed FP16 pairs (x in the low
// halves): hi truncates x to FP16, lo truncates the remainder x - hi, which
// is exact in FP32.  The remainder is one mixed-precision FMA per value,
// -hi * 1 + x with hi read as FP16 (the compiler does not select it here).
__device__ inline void split_pair(float x, float y, uint32_t& hi, uint32_t& lo) {
    hi = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(x, y));
    float rx, ry;
    asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel_hi:[1,0,0]" : "=v"(rx) : "v"(hi), "v"(x));
    asm("v_fma_mix_f32 %0, -%1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(ry) : "v"(hi), "v"(y));
    lo = __builtin_bit_cast(uint32_t, __builtin_amdgcn_cvt_pkrtz(rx, ry));
}

// Value of v in lane ^ 8 (a rotation by 8 within each row of 16 lanes) and
// in lane ^ 2 (a permutation within each group of 4 lanes).
__device__ inline float dpp_xor8(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x128, 0xf, 0xf, false));
}

__device__ inline float dpp_xor2(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x4e, 0xf, 0xf, false));
}

// Position of list entry p in a two-term FP16 kernel's wave list: within each
// group of 32, element j of lane group k (k = lane / 16) is entry 4 j + k, and
// lane group k reads its 8 elements as one 16-byte word.
__device__ inline int32_t h16_slot(int32_t p) { return (p & ~31) | ((p & 3) << 3) | ((p & 31) >> 2); }

// Matrix-core operands of each kernel pair, without its constant factors
// (applied at the store).  e = 1 - u^2 - v^2 for the (point, column), so the
// disc is e > 0; dt, dx, dy are voxel minus point offsets in voxels.
//   Epanechnikov  Kt' = 1 - w^2,        Ks' = e            (both clamped at 0;
//                 the operands never exceed 1, so max(0, .) is a clamp to [0, 1],
//                 which folds into the producing instruction)
//   quartic       Kt' = (1 - w^2)^2,    Ks' = e^2
//   Gaussian      Kt' = exp(-2 w^2),    Ks' = exp(-2 u^2) exp(-2 v^2)   on the supports
//   as printed    Kt' = (1 - w)^2,      Ks' = (1 - u)^2 (1 - v)^2        on the supports
template <int KF>
__device__ inline float kt_operand(float dt, float inv_tv2, float inv_tv) {
    if constexpr (KF == kKernelEpan) {
        return __builtin_amdgcn_fmed3f(fmaf(-dt * dt, inv_tv2, 1.0f), 0.0f, 1.0f);
    } else if constexpr (KF == kKernelQuartic) {
        const float e = __builtin_amdgcn_fmed3f(fmaf(-dt * dt, inv_tv2, 1.0f), 0.0f, 1.0f);
        return e * e;
    } else if constexpr (KF == kKernelGauss) {
        const float w2 = dt * dt * inv_tv2;
        return w2 <= 1.0f ? __builtin_amdgcn_exp2f(-2.0f * 1.44269504088896340736f * w2) : 0.0f;
    } else {
        const float w = dt * inv_tv;
        return dt * dt * inv_tv2 <= 1.0f ? (1.0f - w) * (1.0f - w) : 0.0f;
    }
}

// The per-axis factor of a multiplicatively separable spatial operand (1
// for the additive ones).
template <int KF>
__device__ inline float ks_factor(float d, float inv_hv2, float inv_hv) {
    if constexpr (KF == kKernelGauss) {
        return __builtin_amdgcn_exp2f(-2.0f * 1.44269504088896340736f * (d * d * inv_hv2));
    } else if constexpr (KF == kKernelPrinted) {
        const float u = d * inv_hv;
        return (1.0f - u) * (1.0f - u);
    } else {
        return 1.0f;
    }
}

// Value of the temporal operand ignoring the support (pairs tested exactly).
template <int KF>
__device__ inline float kt_value(float dt, float inv_tv2, float inv_tv) {
    if constexpr (KF == kKernelGauss) {
        return __builtin_amdgcn_exp2f(-2.0f * 1.44269504088896340736f * (dt * dt * inv_tv2));
    } else {
        const float w = dt * inv_tv;
        return (1.0f - w) * (1.0f - w);
    }
}

template <int KF>
__device__ inline float ks_operand(float e, float fx, float fy) {
    if constexpr (KF == kKernelEpan) {
        return __builtin_amdgcn_fmed3f(e, 0.0f, 1.0f);
    } else if constexpr (KF == kKernelQuartic) {
        const float c = __builtin_amdgcn_fmed3f(e, 0.0f, 1.0f);
        return c * c;
    } else {
        return e > 0.0f ? fx * fy : 0.0f;
    }
}

// (sum, comp) += pass by Kahan's rule; pass is cleared.
template <int CG>
__device__ inline void kahan_fold(f32x4 (&sum)[CG], f32x4 (&comp)[CG], f32x4 (&pass)[CG]) {
#pragma unroll
    for (int q = 0; q < CG; ++q) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const float y = __fsub_rn(pass[q][e], comp[q][e]);
            const float t = __fadd_rn(sum[q][e], y);
            comp[q][e] = __fsub_rn(__fsub_rn(t, sum[q][e]), y);
            sum[q][e] = t;
            pass[q][e] = 0.0f;
        }
    }
}

// At most 128 VGPRs, so that four workgroups fit on a compute unit also with
// the three accumulator sets of compensated 32-row tiles (a few registers
// spill outside the matrix-core loop; measured 4-7 % faster than three
// workgroups).  With 768 survivors the LDS holds five workgroups where the
// registers allow it.
// ADAPT: every record carries its own bandwidth terms (1/hv_i^2, 1/tv_i^2,
// weight); they are staged beside the coordinates and enter the operands of
// each point (the weight scales its Kt operand).
// KF: the kernel pair (kKernel*); its constants are applied at the store.
// FP64 support tests of one (record, column) and one (record, row), in base
// voxels with the sampling point at +1/2 (products and sums rounded as
// written, without contraction).
__device__ inline bool exact_disc(const double* __restrict__ x64, uint32_t ri, int32_t X, int32_t Y,
                                  double hv) {
    const double dx = __dadd_rn((double)X + 0.5, -as_global(x64)[3 * (size_t)ri]);
    const double dy = __dadd_rn((double)Y + 0.5, -as_global(x64)[3 * (size_t)ri + 1]);
    return __dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)) < __dmul_rn(hv, hv);
}

__device__ inline bool exact_window(const double* __restrict__ x64, uint32_t ri, int32_t T, double tv) {
    return fabs(__dadd_rn((double)T + 0.5, -as_global(x64)[3 * (size_t)ri + 2])) <= tv;
}

// H16: two-term FP16 operands (see the header).
template <int TT, int MODE, bool FULL, bool ADAPT, int KF, bool H16>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(
    (MODE == kAccKahanReg || FULL || ADAPT || TT == 64 || H16) ? 4 : 6, 8))) void k_gather_items(
    const InstDev* __restrict__ descs, int32_t count, int32_t ntiles_total,
    const WorkItem* __restrict__ items, const uint32_t* __restrict__ bits,
    const uint32_t* __restrict__ sc, uint32_t* __restrict__ ctr, float* __restrict__ partials,
    float* __restrict__ kscratch) {
    static_assert(!(FULL && ADAPT), "the full-cover path assumes one bandwidth pair");
    static_assert(KF == kKernelEpan || (!FULL && !ADAPT), "other pairs: no full-cover path, one pair");
    static_assert(!H16 || (!FULL && !ADAPT && TT <= 32 && MODE != kAccKahanReg),
                  "two-term FP16 operands: one bandwidth pair, no full-cover path, 16/32 rows");
    constexpr int kCap = H16 ? kCapH16 : kCapF32;
    constexpr int kLPad = H16 ? 32 : 8;  // wave lists are padded to this many entries
    constexpr int NB = TT / 16;  // 16-row blocks per tile
    constexpr int CG = 4 * NB;   // accumulator blocks per wave
    constexpr bool EXACT = KF == kKernelGauss || KF == kKernelPrinted;
    // Kahan with the running (sum, compensation) in memory: this thread's
    // slot of kscratch, sum of block k at [k], compensation at [CG + k]
    f32x4* __restrict__ kslot =
        MODE == kAccKahanMem
            ? reinterpret_cast<f32x4*>(kscratch) + ((size_t)blockIdx.x * kThreads + threadIdx.x) * (2 * CG)
            : nullptr;
    constexpr int kPad = kCap;   // index of the padding survivor
    // survivor list: tile-local coordinates as (head, tail) pairs and the
    // quadrants its footprint box meets; entry kPad is a point far outside
    // every tile
    // (one block, so that the full-cover partial sums can reuse it)
    __shared__ float2 sXYT[3 * (kCap + 1)];
    float2* const sX = sXYT;
    float2* const sY = sXYT + (kCap + 1);
    float2* const sT = sXYT + 2 * (kCap + 1);
    __shared__ uint8_t sQ[kCap];
    // per-point bandwidth terms of the survivors (ADAPT only)
    __shared__ float4 sB[ADAPT ? kCap + 1 : 1];
    // record index of each survivor (pairs with exact support tests only)
    __shared__ uint32_t sI[EXACT ? kCap + 1 : 1];
    // per-wave lists of survivor indices meeting the wave's quadrant, padded to
    // kLPad (two-term FP16 kernels: in h16_slot order)
    __shared__ __align__(16) uint16_t sL[kWaves][kCap + kLPad];
    // full-cover kernels: each wave's share of the tile-cover survivors and its
    // quadrant-cover survivors (one scan fills all three lists)
    __shared__ uint16_t sF[FULL ? kWaves : 1][FULL ? kCap / 4 + 8 : 1];
    __shared__ uint16_t sQL[FULL ? kWaves : 1][FULL ? kCap + 8 : 1];
    __shared__ int32_t sRB[kMaxRanges];
    __shared__ int32_t sRP[kMaxRanges + 1];
    __shared__ int32_t sWC[kWaves];
    __shared__ uint32_t sIdx;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (tid == 0) {
        sX[kPad] = make_float2(-1.0e6f, 0.f);
        sY[kPad] = make_float2(-1.0e6f, 0.f);
        sT[kPad] = make_float2(-1.0e6f, 0.f);
        if constexpr (ADAPT) sB[kPad] = make_float4(1.0f, 1.0f, 0.0f, 0.0f);
        if constexpr (EXACT) sI[kPad] = 0u;  // never read: the pad is far from every boundary
    }

    // this wave's quadrant: column groups gx in {gqx, gqx + 1}, gy in {gqy, gqy + 1}
    const int gqx = 2 * (wave & 1), gqy = 2 * (wave >> 1);
    const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    // lane roles in the matrix-core operands: point k of the group, row i of
    // a block (Kt operand), column j = (lane & 3, (lane >> 2) & 3) of a column
    // group (Ks operand)
    const int kq = lane >> 4;
    const float rowc = (float)(lane & 15) + 0.5f;
    const float xc0 = (float)(4 * gqx + (lane & 3)) + 0.5f;
    const float yc0 = (float)(4 * gqy + ((lane >> 2) & 3)) + 0.5f;
    // Which columns a lane's column-group slots hold.  Slot g holds tile-local
    // column (colx(g), coly(g)); the x half and the y half of slot 0 differ per
    // lane (swx, swy), so that of the two x offsets of a Ks column a lane
    // computes one and takes the other from lane ^ 8, and likewise the y
    // offset from lane ^ 2: in both operand forms the 16 lanes of a row hold
    // one point, and lane ^ 8 (lane ^ 2) has the same x (y) with the other
    // half.
    const int swx = (lane >> 3) & 1;
    const int swy = (lane >> 1) & 1;
    auto colx = [&](int g) { return 4 * gqx + 4 * ((g & 1) ^ swx) + (lane & 3); };
    auto coly = [&](int g) { return 4 * gqy + 4 * ((g >> 1) ^ swy) + ((lane >> 2) & 3); };
    const float xcs = xc0 + 4.0f * (float)swx, ycs = yc0 + 4.0f * (float)swy;
    uint16_t* myL = sL[wave];

    const uint32_t T = (uint32_t)ntiles_total;
    const uint32_t home = blockIdx.x % kFetchLanes;
    for (int q = 0; q < 2; ++q) {
        const uint32_t qlen = q == 0 ? sc[kScHeavyItems] : T;
        for (uint32_t lane_off = 0; lane_off < (uint32_t)kFetchLanes; ++lane_off) {
            const uint32_t k = (home + lane_off) % kFetchLanes;
            uint32_t* c = ctr + (q * kFetchLanes + k) * kCtrStride;
            // spatial queue: after the set-up of a tile that takes one phase, the
            // next position of this counter is taken at once, so that the
            // atomic's latency is hidden behind the tile's work (taking it
            // early for longer tiles costs more in balance than it saves)
            bool pend = false;
            uint32_t pnext = 0;
            for (;;) {
                if (tid == 0) {
                    uint32_t v;
                    if (pend) {
                        v = pnext;
                        pend = false;
                    } else {
                        // a counter only grows: when even a stale value shows it
                        // exhausted it is, and the atomic can be skipped
                        const uint32_t seen = __hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        v = (k + kFetchLanes * seen >= qlen) ? 0xffffffffu : k + kFetchLanes * atomicAdd(c, 1u);
                    }
                    sIdx = v;
                }
                __syncthreads();
                const uint32_t idx = __builtin_amdgcn_readfirstlane(sIdx);
                __syncthreads();  // sIdx is rewritten by the next fetch
                if (idx >= qlen) break;
                WorkItem it;
                // spatial queue: every tile in spatial order, minus those the
                // heaviest-first queue took (tested after the set-up, so that the
                // mask's load overlaps the set-up's)
                uint32_t taken = 0;
                if (q == 0) {
                    it = items[idx];
                } else {
                    taken = (bits[idx >> 5] >> (idx & 31)) & 1u;
                    it.tile = spatial_tile(descs[find_inst(descs, count, idx)], idx);
                    it.cbeg = 0;
                    it.cend = kAll;
                    it.slot = kNoSlot;
                }
                const int32_t inst = find_inst(descs, count, it.tile);
                const InstDev& D = descs[inst];
                const float inv_hv2 = D.inv_hv2, inv_tv2 = D.inv_tv2;
                const float inv_hv = D.inv_hv, inv_tv = D.inv_tv;

                const int32_t tile = (int32_t)(it.tile - (uint32_t)D.tile_base);
                const int32_t tx = tile % D.ntx;
                const int32_t rest = tile / D.ntx;
                const int32_t ty = rest % D.nty;
                const int32_t tt = rest / D.nty;
                // tile origin in the instance grid and in the set's base grid
                const int32_t X0 = tx * kTileXY, Y0 = ty * kTileXY, T0 = tt * TT;
                const int32_t BX0 = X0 + D.ox, BY0 = Y0 + D.oy, BT0 = T0 + D.ot;

                // ---- setup: candidate ranges (one per bin row (t, y)) -----------
                const TileBins tb = tile_bins(D, BX0, BY0, BT0, TT);
                const int32_t nyr = tb.cy1 - tb.cy0 + 1;
                const int32_t nranges = nyr * (tb.ct1 - tb.ct0 + 1);
                if (wave == 0) {
                    int32_t beg = 0, len = 0;
                    if (lane < nranges) {
                        const int32_t cz = tb.ct0 + lane / nyr, cy = tb.cy0 + lane % nyr;
                        const int32_t row = (cz * D.ncy + cy) * D.ncx;
                        beg = (int32_t)as_global(D.cell_start)[row + tb.cx0];
                        len = (int32_t)as_global(D.cell_start)[row + tb.cx1 + 1] - beg;
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
                __syncthreads();
                if (taken) continue;
                const int32_t total = sRP[nranges];
                const int32_t cend = it.cend == kAll ? total : min((int32_t)it.cend, total);
                if (q == 1 && tid == 0 && total <= kCap) {
                    pend = true;
                    pnext = k + kFetchLanes * atomicAdd(c, 1u);
                }
                const PointRec* __restrict__ recs = D.recs;

                // ---- accumulators: [column group q][row block b].  acc is the
                // matrix-core target: the whole sum in plain mode, the current
                // phase's sum with Kahan; sum and comp hold the running Kahan
                // pair in registers (in kslot in memory mode).
                constexpr bool REG = MODE == kAccKahanReg;
                f32x4 acc[CG];
                f32x4 sum[REG ? CG : 1];
                f32x4 comp[REG ? CG : 1];
#pragma unroll
                for (int k = 0; k < CG; ++k) {
                    acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
                    if constexpr (REG) {
                        sum[k] = f32x4{0.f, 0.f, 0.f, 0.f};
                        comp[k] = f32x4{0.f, 0.f, 0.f, 0.f};
                    }
                }
                int32_t nphase = 0;

                // one group: operands from the coordinates (and, ADAPT, the
                // bandwidth terms pb) of this lane's point, then all CG
                // instructions
                // this lane's operands for one point: the Kt entries of its row in
                // every block (av) and the Ks entries of its column in every
                // column group (ks)
                auto operands = [&](const float2 cx, const float2 cy, const float2 ctt, const float4 pb,
                                    const uint32_t ri, float (&av)[NB], float (&kso)[4]) {
                    const float ihv2 = ADAPT ? pb.x : inv_hv2;
                    const float itv2 = ADAPT ? pb.y : inv_tv2;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const float dt = ((rowc + 16.0f * b) - ctt.x) - ctt.y;
                        if constexpr (EXACT) {
                            const float w2 = dt * dt * itv2;
                            bool in = w2 <= 1.0f;
                            if (fabsf(w2 - 1.0f) < kExactBand)
                                in = exact_window(D.x64, ri, BT0 + 16 * b + (lane & 15), D.tv64);
                            av[b] = in ? kt_value<KF>(dt, itv2, inv_tv) : 0.0f;
                        } else {
                            av[b] = kt_operand<KF>(dt, itv2, inv_tv);
                        }
                        if constexpr (ADAPT) av[b] *= pb.z;
                    }
                    // ux = 1 - dx^2/hv^2 and dy^2 of the two x and two y offsets
                    // of this lane's columns, e = ux - dy^2/hv^2
                    float ux[2], uy[2], fx[2], fy[2];
                    {
                        const float dx = (xcs - cx.x) - cx.y;
                        const float dy = (ycs - cy.x) - cy.y;
                        ux[0] = fmaf(-dx * dx, ihv2, 1.0f);
                        uy[0] = dy * dy;
                        ux[1] = dpp_xor8(ux[0]);
                        uy[1] = dpp_xor2(uy[0]);
                        fx[0] = ks_factor<KF>(dx, ihv2, inv_hv);
                        fy[0] = ks_factor<KF>(dy, ihv2, inv_hv);
                        if constexpr (EXACT) {
                            fx[1] = dpp_xor8(fx[0]);
                            fy[1] = dpp_xor2(fy[0]);
                        } else {
                            fx[1] = fy[1] = 1.0f;
                        }
                    }
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const float e = fmaf(-uy[g >> 1], ihv2, ux[g & 1]);
                        float ks = ks_operand<KF>(e, fx[g & 1], fy[g >> 1]);
                        if constexpr (EXACT) {
                            if (fabsf(e) < kExactBand) {
                                const int32_t X = BX0 + colx(g);
                                const int32_t Y = BY0 + coly(g);
                                ks = exact_disc(D.x64, ri, X, Y, D.hv64) ? fx[g & 1] * fy[g >> 1] : 0.0f;
                            }
                        }
                        kso[g] = ks;
                    }
                };
                auto group = [&](const float2 cx, const float2 cy, const float2 ctt, const float4 pb,
                                 const uint32_t ri) {
                    float av[NB], ks[4];
                    operands(cx, cy, ctt, pb, ri, av, ks);
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
#pragma unroll
                        for (int b = 0; b < NB; ++b)
                            acc[g * NB + b] =
                                __builtin_amdgcn_mfma_f32_16x16x4f32(av[b], ks[g], acc[g * NB + b], 0, 0, 0);
                    }
                };

                // full-cover group: A = Kt of one (point, row), B = a(x) - 1 and
                // b(y) of one (point, column), a = dx^2/hv^2, b = dy^2/hv^2
                f32x4 fa[FULL ? NB : 1], fb[FULL ? NB : 1];
#pragma unroll
                for (int b = 0; b < (FULL ? NB : 1); ++b) {
                    fa[b] = f32x4{0.f, 0.f, 0.f, 0.f};
                    fb[b] = f32x4{0.f, 0.f, 0.f, 0.f};
                }
                // quadrant-cover group (a disc covering this wave's quadrant but
                // not the tile): one instruction per row block, its 16 columns
                // the quadrant's 8 x-columns (B = a - 1) and 8 y-columns (B = b)
                f32x4 fq[FULL ? NB : 1];
#pragma unroll
                for (int b = 0; b < (FULL ? NB : 1); ++b) fq[b] = f32x4{0.f, 0.f, 0.f, 0.f};
                const float qx0 = (float)(8 * (wave & 1) + (lane & 7)) + 0.5f;
                const float qy0 = (float)(8 * (wave >> 1) + (lane & 7)) + 0.5f;
                const bool qxcol = (lane & 15) < 8;
                auto group_quad = [&](const float2 cx, const float2 cy, const float2 ctt) {
                    float av[NB];
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const float dt = ((rowc + 16.0f * b) - ctt.x) - ctt.y;
                        av[b] = __builtin_amdgcn_fmed3f(fmaf(-dt * dt, inv_tv2, 1.0f), 0.0f, 1.0f);
                    }
                    const float dx = (qx0 - cx.x) - cx.y;
                    const float dy = (qy0 - cy.x) - cy.y;
                    const float bq = qxcol ? fmaf(dx * dx, inv_hv2, -1.0f) : dy * dy * inv_hv2;
#pragma unroll
                    for (int b = 0; b < NB; ++b)
                        fq[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[b], bq, fq[b], 0, 0, 0);
                };
                auto group_full = [&](const float2 cx, const float2 cy, const float2 ctt) {
                    float av[NB];
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const float dt = ((rowc + 16.0f * b) - ctt.x) - ctt.y;
                        av[b] = __builtin_amdgcn_fmed3f(fmaf(-dt * dt, inv_tv2, 1.0f), 0.0f, 1.0f);
                    }
                    const float dx = (rowc - cx.x) - cx.y;  // column x = lane % 16
                    const float dy = (rowc - cy.x) - cy.y;  // column y = lane % 16
                    const float am1 = fmaf(dx * dx, inv_hv2, -1.0f);
                    const float bv = dy * dy * inv_hv2;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        fa[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[b], am1, fa[b], 0, 0, 0);
                        fb[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[b], bv, fb[b], 0, 0, 0);
                    }
                };

                // two-term FP16 group of 32 list entries from `base`, nv of them valid:
                // lane group k = lane / 16 supplies points 4 j + k (j = 0..7) as the
                // eight elements of its operands; pairs of elements holding only
                // padding in every lane group are zero without being computed
                auto group16 = [&](const int32_t base, const int32_t nv) {
                    const int32_t npv = (nv + 7) >> 3;
                    u32x4 ah[NB], al[NB], bh[4], bl[4];
                    const uint4 ix = *reinterpret_cast<const uint4*>(myL + base + 8 * kq);
                    const uint32_t ixa[4] = {ix.x, ix.y, ix.z, ix.w};
#pragma unroll
                    for (int jp = 0; jp < 4; ++jp) {
                        if (jp > 0 && jp >= npv) {
#pragma unroll
                            for (int b = 0; b < NB; ++b) ah[b][jp] = al[b][jp] = 0u;
#pragma unroll
                            for (int g = 0; g < 4; ++g) bh[g][jp] = bl[g][jp] = 0u;
                            continue;
                        }
                        float kt[2][NB], ks[2][4];
#pragma unroll
                        for (int jj = 0; jj < 2; ++jj) {
                            const int s = jj == 0 ? (int)(ixa[jp] & 0xffffu) : (int)(ixa[jp] >> 16);
                            operands(sX[s], sY[s], sT[s], float4{}, EXACT ? sI[s] : 0u, kt[jj], ks[jj]);
                        }
#pragma unroll
                        for (int b = 0; b < NB; ++b) {
                            uint32_t h, l;
                            split_pair(kt[0][b], kt[1][b], h, l);
                            ah[b][jp] = h;
                            al[b][jp] = l;
                        }
#pragma unroll
                        for (int g = 0; g < 4; ++g) {
                            uint32_t h, l;
                            split_pair(ks[0][g], ks[1][g], h, l);
                            bh[g][jp] = h;
                            bl[g][jp] = l;
                        }
                    }
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
#pragma unroll
                        for (int b = 0; b < NB; ++b) {
                            const h16x8 Ah = __builtin_bit_cast(h16x8, ah[b]), Al = __builtin_bit_cast(h16x8, al[b]);
                            const h16x8 Bh = __builtin_bit_cast(h16x8, bh[g]), Bl = __builtin_bit_cast(h16x8, bl[g]);
                            f32x4 a = acc[g * NB + b];
                            a = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ah, Bh, a, 0, 0, 0);
                            a = __builtin_amdgcn_mfma_f32_16x16x32_f16(Ah, Bl, a, 0, 0, 0);
                            a = __builtin_amdgcn_mfma_f32_16x16x32_f16(Al, Bh, a, 0, 0, 0);
                            acc[g * NB + b] = a;
                        }
                    }
                };

                // the ranges in registers: lane r holds range r's first
                // candidate (past the last range: larger than any) and the
                // record index minus candidate index within it
                const int32_t rpl = lane < nranges ? sRP[lane] : 0x7fffffff;
                const int32_t rol = lane < nranges ? sRB[lane] - sRP[lane] : 0;
                // record (and bandwidth terms) of candidate cw + lane, if any
                // (cw: the wave's first candidate).  Its range is the last one
                // starting at or before it: the ranges starting at or before
                // cw form a prefix of the lanes, and the few starting within
                // the wave's 64 candidates are stepped over in order.
                auto fetch = [&](const int32_t cw_, PointRec& r, uint32_t& rix, float4& pbw) {
                    const int32_t cw = __builtin_amdgcn_readfirstlane(cw_);
                    const int32_t c = cw + lane;
                    int32_t lo = __popcll(__ballot(rpl <= cw)) - 1;  // sRP[0] = 0 <= cw
                    for (unsigned long long in = __ballot(rpl > cw && rpl <= cw + 63); in != 0ull; in &= in - 1ull)
                        lo += c >= __builtin_amdgcn_readlane(rpl, __builtin_ctzll(in)) ? 1 : 0;
                    const int32_t roff = __shfl(rol, lo, 64);  // every lane takes part
                    if (c < cend) {
                        const int32_t ri = roff + c;
                        rix = (uint32_t)ri;
                        {
                            const auto* q = reinterpret_cast<const __attribute__((address_space(1))) u32x4*>(
                                as_global(recs + ri));
                            const u32x4 a = q[0], b2 = q[1];
                            r.xh = __uint_as_float(a.x);
                            r.yh = __uint_as_float(a.y);
                            r.th = __uint_as_float(a.z);
                            r.xb = a.w;
                            r.yb = b2.x;
                            r.tb = b2.y;
                            r.xl_yl = b2.z;
                            r.tl = b2.w;
                        }
                        if constexpr (ADAPT) {
                            const f32x4 v = *reinterpret_cast<const __attribute__((address_space(1))) f32x4*>(
                                as_global(D.bw + ri));
                            pbw = make_float4(v.x, v.y, v.z, v.w);
                        }
                    }
                };
                int32_t bb = (int32_t)min(it.cbeg, (uint32_t)cend);
                while (bb < cend) {
                    // ---- stage: fill the survivor list; each round's records are
                    // loaded during the round before it ----------------------------
                    int32_t count_s = 0;
                    PointRec rn{};
                    float4 pbn{};
                    uint32_t rin = 0;
                    fetch(bb + 64 * wave, rn, rin, pbn);
                    while (bb < cend && count_s <= kCap - kThreads) {
                        const int32_t c = bb + tid;
                        bool surv = false;
                        const PointRec r = rn;
                        const float4 pbw = pbn;
                        const uint32_t rix = rin;
                        fetch(bb + kThreads + 64 * wave, rn, rin, pbn);
                        uint32_t qm = 0;
                        if (c < cend) {
                            const int32_t xlo = (int32_t)(r.xb & 0xffffu) - BX0, xhi = (int32_t)(r.xb >> 16) - BX0;
                            const int32_t ylo = (int32_t)(r.yb & 0xffffu) - BY0, yhi = (int32_t)(r.yb >> 16) - BY0;
                            const int32_t tlo = (int32_t)(r.tb & 0xffffu), thi = (int32_t)(r.tb >> 16);
                            if (tlo <= BT0 + TT - 1 && thi >= BT0) {
                                // quadrants (qx, qy) whose 8 x 8 columns the footprint box meets
                                const bool x0 = xlo <= 7 && xhi >= 0, x1 = xlo <= 15 && xhi >= 8;
                                const bool y0 = ylo <= 7 && yhi >= 0, y1 = ylo <= 15 && yhi >= 8;
                                qm = (uint32_t)(x0 && y0) | ((uint32_t)(x1 && y0) << 1) |
                                     ((uint32_t)(x0 && y1) << 2) | ((uint32_t)(x1 && y1) << 3);
                                // of those, the quadrants the disc reaches: nearest column
                                // centre per axis and quadrant half
                                const float px = (r.xh - (float)BX0) + half_lo(r.xl_yl);
                                const float py = (r.yh - (float)BY0) + half_hi(r.xl_yl);
                                {
                                    const float ihv2p = ADAPT ? pbw.x : inv_hv2;
                                    float nx2[2], ny2[2];
#pragma unroll
                                    for (int h = 0; h < 2; ++h) {
                                        const float ex = fmaxf(fabsf(px - (8.0f * h + 4.0f)) - 3.501f, 0.0f);
                                        const float ey = fmaxf(fabsf(py - (8.0f * h + 4.0f)) - 3.501f, 0.0f);
                                        nx2[h] = ex * ex;
                                        ny2[h] = ey * ey;
                                    }
#pragma unroll
                                    for (int q = 0; q < 4; ++q)
                                        if ((nx2[q & 1] + ny2[q >> 1]) * ihv2p > kCullMargin) qm &= ~(1u << q);
                                }
                                if (FULL && (D.flags & kInstFull)) {
                                    // quadrants whose every column centre the disc
                                    // covers (farthest corner, with a margin): the
                                    // spatial kernel is 1 - a(x) - b(y) there,
                                    // separable in x and y
                                    // farthest column centre per axis and quadrant half
                                    float ax2[2], ay2[2];
#pragma unroll
                                    for (int h = 0; h < 2; ++h) {
                                        const float ex = fmaxf(fabsf(8.0f * h + 0.5f - px), fabsf(8.0f * h + 7.5f - px));
                                        const float ey = fmaxf(fabsf(8.0f * h + 0.5f - py), fabsf(8.0f * h + 7.5f - py));
                                        ax2[h] = ex * ex;
                                        ay2[h] = ey * ey;
                                    }
                                    uint32_t qc = 0;
#pragma unroll
                                    for (int q = 0; q < 4; ++q)
                                        if (((qm >> q) & 1u) && (ax2[q & 1] + ay2[q >> 1]) * inv_hv2 <= kFullMargin)
                                            qc |= 1u << q;
                                    qm = (qm & ~qc) | (qc << 4);
                                }
                            }
                            surv = qm != 0;
                        }
                        const unsigned long long m = __ballot(surv);
                        if (lane == 0) sWC[wave] = __popcll(m);
                        __syncthreads();
                        int32_t off = count_s, add = 0;
#pragma unroll
                        for (int w = 0; w < kWaves; ++w) {
                            const int32_t cw = sWC[w];
                            off += (w < wave) ? cw : 0;
                            add += cw;
                        }
                        if (surv) {
                            const int s = off + __popcll(m & lt);
                            // head - origin is exact for the offsets that reach the tile
                            sX[s] = make_float2(r.xh - (float)BX0, half_lo(r.xl_yl));
                            sY[s] = make_float2(r.yh - (float)BY0, half_hi(r.xl_yl));
                            sT[s] = make_float2(r.th - (float)BT0, half_lo(r.tl));
                            if constexpr (ADAPT) sB[s] = pbw;
                            if constexpr (EXACT) sI[s] = rix;
                            sQ[s] = (uint8_t)qm;
                        }
                        count_s += add;
                        bb += kThreads;
                        __syncthreads();  // sWC is rewritten by the next round
                    }

                    // ---- this wave's lists, in one scan of the survivors: those
                    // meeting its quadrant; (full-cover kernels) its share of
                    // those covering the tile, dealt to the waves in groups of 4
                    // by rank; and those covering its quadrant only --------------
                    int32_t nw = 0, nfull = 0, nf = 0, nq = 0;
                    for (int32_t base = 0; base < count_s; base += 64) {
                        const int32_t s = base + lane;
                        const uint32_t q = s < count_s ? (uint32_t)sQ[s] : 0u;
                        const bool mine = (q >> wave) & 1u;
                        const unsigned long long bm = __ballot(mine);
                        if (mine) {
                            const int32_t p = nw + __popcll(bm & lt);
                            myL[H16 ? h16_slot(p) : p] = (uint16_t)s;
                        }
                        nw += __popcll(bm);
                        if constexpr (FULL) {
                            const bool isf = q == kCoverAll;
                            const unsigned long long fm = __ballot(isf);
                            const int32_t rk = nfull + __popcll(fm & lt);
                            const bool minef = isf && ((rk >> 2) & 3) == wave;
                            const bool mineq = !isf && ((q >> (4 + wave)) & 1u);
                            const unsigned long long bf = __ballot(minef), bq = __ballot(mineq);
                            if (minef) sF[wave][nf + __popcll(bf & lt)] = (uint16_t)s;
                            if (mineq) sQL[wave][nq + __popcll(bq & lt)] = (uint16_t)s;
                            nf += __popcll(bf);
                            nq += __popcll(bq);
                            nfull += __popcll(fm);
                        }
                    }
                    // pad to a whole number of pairs of groups (FP32 operands) or of
                    // 32-point groups (two-term FP16)
                    if (lane < ((kLPad - (nw & (kLPad - 1))) & (kLPad - 1))) {
                        const int32_t p = nw + lane;
                        myL[H16 ? h16_slot(p) : p] = (uint16_t)kPad;
                    }
                    const int32_t npairs = H16 ? 0 : (nw + 7) >> 3;
                    if constexpr (H16) {
                        for (int32_t base = 0; base < nw; base += 32) group16(base, min(32, nw - base));
                    }
                    uint16_t* const myF = FULL ? sF[wave] : myL;
                    uint16_t* const myQ = FULL ? sQL[wave] : myL;
                    if constexpr (FULL) {
                        if (lane < ((8 - (nf & 7)) & 7)) myF[nf + lane] = (uint16_t)kPad;
                        if (lane < ((8 - (nq & 7)) & 7)) myQ[nq + lane] = (uint16_t)kPad;
                    }

                    // ---- matrix-core accumulation, two groups per iteration ---------
                    if (npairs > 0) {
                        int s = myL[kq];
                        float2 ax = sX[s], ay = sY[s], at = sT[s];
                        float4 ab = ADAPT ? sB[s] : float4{};
                        uint32_t ai = EXACT ? sI[s] : 0u;
                        for (int32_t pr = 0; pr < npairs; ++pr) {
                            s = myL[8 * pr + 4 + kq];
                            const float2 bx = sX[s], by = sY[s], bt = sT[s];
                            const float4 bbw = ADAPT ? sB[s] : float4{};
                            const uint32_t bi = EXACT ? sI[s] : 0u;
                            group(ax, ay, at, ab, ai);
                            if (pr + 1 < npairs) {
                                s = myL[8 * pr + 8 + kq];
                                ax = sX[s];
                                ay = sY[s];
                                at = sT[s];
                                if constexpr (ADAPT) ab = sB[s];
                                if constexpr (EXACT) ai = sI[s];
                            }
                            group(bx, by, bt, bbw, bi);
                        }
                    }
                    if constexpr (FULL) {
                        const int32_t nfp = (nf + 7) >> 3;
                        if (nfp > 0) {
                            int s = myF[kq];
                            float2 ax = sX[s], ay = sY[s], at = sT[s];
                            for (int32_t pr = 0; pr < nfp; ++pr) {
                                s = myF[8 * pr + 4 + kq];
                                const float2 bx = sX[s], by = sY[s], bt = sT[s];
                                group_full(ax, ay, at);
                                if (pr + 1 < nfp) {
                                    s = myF[8 * pr + 8 + kq];
                                    ax = sX[s];
                                    ay = sY[s];
                                    at = sT[s];
                                }
                                group_full(bx, by, bt);
                            }
                        }
                        const int32_t nqp = (nq + 7) >> 3;
                        if (nqp > 0) {
                            int s = myQ[kq];
                            float2 ax = sX[s], ay = sY[s], at = sT[s];
                            for (int32_t pr = 0; pr < nqp; ++pr) {
                                s = myQ[8 * pr + 4 + kq];
                                const float2 bx = sX[s], by = sY[s], bt = sT[s];
                                group_quad(ax, ay, at);
                                if (pr + 1 < nqp) {
                                    s = myQ[8 * pr + 8 + kq];
                                    ax = sX[s];
                                    ay = sY[s];
                                    at = sT[s];
                                }
                                group_quad(bx, by, bt);
                            }
                            // acc -= (sum Kt (a - 1))[T][x] + (sum Kt b)[T][y]: lane
                            // (k, j) of a column group reads row group k's entries of
                            // its x column and of its y column
#pragma unroll
                            for (int g = 0; g < 4; ++g) {
                                const int sx = (lane & 48) | (colx(g) - 4 * gqx);
                                const int sy = (lane & 48) | (8 + coly(g) - 4 * gqy);
#pragma unroll
                                for (int b = 0; b < NB; ++b) {
#pragma unroll
                                    for (int e = 0; e < 4; ++e)
                                        acc[g * NB + b][e] -= __shfl(fq[b][e], sx, 64) + __shfl(fq[b][e], sy, 64);
                                }
                            }
#pragma unroll
                            for (int b = 0; b < NB; ++b) fq[b] = f32x4{0.f, 0.f, 0.f, 0.f};
                        }
                        if (nfull > 0) {
                            // add -(sum Kt (a - 1))[T][X] - (sum Kt b)[T][Y] of the
                            // four waves, in wave order, to this phase's sums
                            __syncthreads();  // the survivor arrays are no longer read
                            float* const W = reinterpret_cast<float*>(sXYT);
                            const int32_t t4 = (lane >> 4) * 4, c16 = (lane & 15) * 16;
#pragma unroll
                            for (int b = 0; b < NB; ++b) {
                                *reinterpret_cast<f32x4*>(W + ((wave * 2 + 0) * NB + b) * 256 + c16 + t4) = fa[b];
                                *reinterpret_cast<f32x4*>(W + ((wave * 2 + 1) * NB + b) * 256 + c16 + t4) = fb[b];
                                fa[b] = f32x4{0.f, 0.f, 0.f, 0.f};
                                fb[b] = f32x4{0.f, 0.f, 0.f, 0.f};
                            }
                            __syncthreads();
                            // sum the four waves' entries, in wave order, into
                            // wave 0's region (each thread reads its entry of
                            // every wave before it writes)
                            if (tid < 128 * NB) {
                                f32x4* const W4 = reinterpret_cast<f32x4*>(W);
                                f32x4 v = W4[tid];
#pragma unroll
                                for (int w = 1; w < kWaves; ++w) v += W4[w * 128 * NB + tid];
                                W4[tid] = v;
                            }
                            __syncthreads();
#pragma unroll
                            for (int g = 0; g < 4; ++g) {
                                const int32_t lx = colx(g), ly = coly(g);
#pragma unroll
                                for (int b = 0; b < NB; ++b) {
                                    const f32x4 sa = *reinterpret_cast<const f32x4*>(W + (0 * NB + b) * 256 + lx * 16 + t4);
                                    const f32x4 sbv = *reinterpret_cast<const f32x4*>(W + (1 * NB + b) * 256 + ly * 16 + t4);
                                    acc[g * NB + b] -= sa + sbv;
                                }
                            }
                            __syncthreads();  // W is the survivor list again
                            if (tid == 0) {
                                sX[kPad] = make_float2(-1.0e6f, 0.f);
                                sY[kPad] = make_float2(-1.0e6f, 0.f);
                                sT[kPad] = make_float2(-1.0e6f, 0.f);
                            }
                        }
                    }
                    if constexpr (MODE == kAccKahanReg) {
                        kahan_fold<CG>(sum, comp, acc);
                    } else if constexpr (MODE == kAccKahanMem) {
                        // the same operations as in registers; a tile that ends in
                        // its first phase (sum = comp = 0) keeps acc as it is
                        const bool last = bb >= cend;
                        if (!(nphase == 0 && last)) {
#pragma unroll
                            for (int k = 0; k < CG; ++k) {
                                const f32x4 s0 = nphase == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : kslot[k];
                                const f32x4 c0 = nphase == 0 ? f32x4{0.f, 0.f, 0.f, 0.f} : kslot[CG + k];
                                f32x4 t, c1;
#pragma unroll
                                for (int e = 0; e < 4; ++e) {
                                    const float y = __fsub_rn(acc[k][e], c0[e]);
                                    t[e] = __fadd_rn(s0[e], y);
                                    c1[e] = __fsub_rn(__fsub_rn(t[e], s0[e]), y);
                                }
                                if (last) {
                                    acc[k] = t;
                                } else {
                                    kslot[k] = t;
                                    kslot[CG + k] = c1;
                                    acc[k] = f32x4{0.f, 0.f, 0.f, 0.f};
                                }
                            }
                        }
                    }
                    ++nphase;
                    __syncthreads();  // the lists are refilled next
                }

                // ---- store: lane holds rows 16 b + 4 (lane / 16) + e of column
                // (lane % 4, (lane / 4) % 4) of each of its column groups -------------
                if constexpr (REG) {
#pragma unroll
                    for (int k = 0; k < CG; ++k) acc[k] = sum[k];
                }
                if (it.slot != kNoSlot) {
                    float* P = partials + (size_t)it.slot * (kTileXY * kTileXY * TT);
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const int32_t lx = colx(g), ly = coly(g);
#pragma unroll
                        for (int b = 0; b < NB; ++b)
                            *reinterpret_cast<f32x4*>(P + (lx * kTileXY + ly) * TT + 16 * b + 4 * (lane >> 4)) =
                                acc[g * NB + b];
                    }
                    continue;
                }
                const bool mass = (D.flags & kInstMass) != 0;
                const int32_t gxI = D.gx, gyI = D.gy, gtI = D.gt;
                const float cnorm = D.cnorm;
                float* __restrict__ out = D.out;
                double msum = 0.0;
                const bool vec = (gtI & 3) == 0;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int32_t X = X0 + colx(g);
                    const int32_t Y = Y0 + coly(g);
                    if (X >= gxI || Y >= gyI) continue;
                    float* col = out + ((size_t)X * gyI + Y) * gtI;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const int32_t T = T0 + 16 * b + 4 * (lane >> 4);
                        const f32x4 v = acc[g * NB + b] * cnorm;
                        if (vec && T + 3 < gtI) {
                            *reinterpret_cast<__attribute__((address_space(1))) f32x4*>(as_global(col) + T) = v;
                            msum += (double)v[0] + (double)v[1] + (double)v[2] + (double)v[3];
                        } else {
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                if (T + e < gtI) {
                                    as_global(col)[T + e] = v[e];
                                    msum += (double)v[e];
                                }
                            }
                        }
                    }
                }
                if (mass) {
#pragma unroll
                    for (int d = 32; d >= 1; d >>= 1) msum += __shfl_xor(msum, d, 64);
                    if (lane == 0) as_global(D.tile_part)[(size_t)tile * kWaves + wave] = msum;
                }
            }
        }
    }
}

// Split tiles: add the parts' partial sums in part order, scale, store, and
// write the tile's mass partials.  Thread k owns column (k / 16, k % 16).
template <int TT, bool KAHAN>
__global__ __launch_bounds__(kThreads) void k_reduce_split(const InstDev* __restrict__ descs,
                                                           int32_t count,
                                                           const uint32_t* __restrict__ top,
                                                           const uint32_t* __restrict__ sc,
                                                           const float* __restrict__ partials) {
    const uint32_t nsplit = sc[kScSplit];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int32_t lx = tid / kTileXY, ly = tid % kTileXY;
    for (uint32_t k = blockIdx.x; k < nsplit; k += gridDim.x) {
        const uint32_t tile_g = top[4 * k], parts = top[4 * k + 1], slot0 = top[4 * k + 2];
        const int32_t inst = find_inst(descs, count, tile_g);
        const InstDev& D = descs[inst];
        const int32_t tile = (int32_t)(tile_g - (uint32_t)D.tile_base);
        const int32_t tx = tile % D.ntx;
        const int32_t rest = tile / D.ntx;
        const int32_t ty = rest % D.nty;
        const int32_t tt = rest / D.nty;
        const int32_t X = tx * kTileXY + lx, Y = ty * kTileXY + ly, T0 = tt * TT;
        const bool col_ok = X < D.gx && Y < D.gy;
        const int32_t gtI = D.gt;
        float* col = D.out + ((size_t)(col_ok ? X : 0) * D.gy + (col_ok ? Y : 0)) * gtI;
        double msum = 0.0;
#pragma unroll
        for (int r = 0; r < TT; r += 4) {
            f32x4 s = f32x4{0.f, 0.f, 0.f, 0.f}, c = f32x4{0.f, 0.f, 0.f, 0.f};
            // every part's values in flight at once, then added in part order
            f32x4 pv[kMaxParts];
#pragma unroll
            for (int p = 0; p < kMaxParts; ++p)
                pv[p] = (uint32_t)p < parts ? *reinterpret_cast<const f32x4*>(
                                                  partials + ((size_t)(slot0 + p) * (kTileXY * kTileXY) + tid) * TT + r)
                                            : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int p = 0; p < kMaxParts; ++p) {
                if ((uint32_t)p >= parts) break;
                const f32x4 v = pv[p];
                if constexpr (KAHAN) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const float y = __fsub_rn(v[e], c[e]);
                        const float t = __fadd_rn(s[e], y);
                        c[e] = __fsub_rn(__fsub_rn(t, s[e]), y);
                        s[e] = t;
                    }
                } else {
                    s += v;
                }
            }
            const f32x4 o = s * D.cnorm;
            if (col_ok) {
                if ((gtI & 3) == 0 && T0 + r + 3 < gtI) {
                    *reinterpret_cast<__attribute__((address_space(1))) f32x4*>(as_global(col) + T0 + r) = o;
#pragma unroll
                    for (int e = 0; e < 4; ++e) msum += (double)o[e];
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (T0 + r + e < gtI) {
                            as_global(col)[T0 + r + e] = o[e];
                            msum += (double)o[e];
                        }
                    }
                }
            }
        }
        if (D.flags & kInstMass) {
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) msum += __shfl_xor(msum, d, 64);
            if (lane == 0) as_global(D.tile_part)[(size_t)tile * kWaves + wave] = msum;
        }
    }
}

// Workgroups of the persistent gather: compute units x resident workgroups
// per compute unit, cached per device (memory-mode Kahan at most
// kMemKahanGroups, the slots of its scratch).
template <int TT, int MODE, bool FULL, bool ADAPT, int KF, bool H16>
int resident_groups() {
    static_assert(!FULL || TT <= 32, "the full-cover sums of 64-row tiles do not fit the survivor LDS");
    static std::atomic<int> cache[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v > 0) return v;
    int ncu = 0, occ = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_gather_items<TT, MODE, FULL, ADAPT, KF, H16>,
                                                     kThreads, 0) != hipSuccess)
        occ = 0;
    v = (ncu > 0 ? ncu : 256) * (occ > 0 ? occ : 1);
    if (MODE == kAccKahanMem && v > kMemKahanGroups) v = kMemKahanGroups;  // (and below kahan_slots(T))
    cache[dev].store(v, std::memory_order_relaxed);
    return v;
}

template <int TT, int MODE, bool FULL, bool ADAPT, int KF, bool H16>
void launch_items_t(const InstDev* d, int32_t count, const WorkItem* items, const uint32_t* bits,
                    const uint32_t* sc, uint32_t* ctr, float* partials, float* kscratch, int64_t T,
                    hipStream_t s) {
    int64_t g = resident_groups<TT, MODE, FULL, ADAPT, KF, H16>();
    const int64_t most = max_items(T);  // (the Kahan scratch holds kahan_slots(T) workgroups)
    if (g > most) g = most;
    if (g < 1) g = 1;
    hipLaunchKernelGGL((k_gather_items<TT, MODE, FULL, ADAPT, KF, H16>), dim3((uint32_t)g), dim3(kThreads), 0,
                       s, d, count, (int32_t)T, items, bits, sc, ctr, partials, kscratch);
}

// f.template operator()<TT, MODE, FULL, ADAPT, KF, H16>() for one (tile
// rows, mode) of the Epanechnikov pair: per-point bandwidths never take the
// full-cover path, nor do 64-row tiles; two-term FP16 operands are the
// kernels without either of them, 16 or 32 rows, plain or scratch-form
// Kahan (the caller maps the register form to the scratch form).
template <int TT, int MODE, typename F>
void dispatch_variant(bool full, bool adapt, bool h16, F& f) {
    if (adapt) {
        f.template operator()<TT, MODE, false, true, kKernelEpan, false>();
    } else if constexpr (TT <= 32) {
        if (full) f.template operator()<TT, MODE, true, false, kKernelEpan, false>();
        else if constexpr (MODE != kAccKahanReg) {
            if (h16) f.template operator()<TT, MODE, false, false, kKernelEpan, true>();
            else f.template operator()<TT, MODE, false, false, kKernelEpan, false>();
        } else {
            f.template operator()<TT, MODE, false, false, kKernelEpan, false>();
        }
    } else {
        f.template operator()<TT, MODE, false, false, kKernelEpan, false>();
    }
}

// The other pairs: 16- or 32-row tiles, plain or compensated (scratch form;
// the register form performs the same operations), one bandwidth pair.
template <int KF, bool H, typename F>
void dispatch_pair_form(int tile_t, int mode, F& f) {
    const bool kahan = mode != kAccPlain;
    if (tile_t == 16) {
        kahan ? f.template operator()<16, kAccKahanMem, false, false, KF, H>()
              : f.template operator()<16, kAccPlain, false, false, KF, H>();
    } else {
        kahan ? f.template operator()<32, kAccKahanMem, false, false, KF, H>()
              : f.template operator()<32, kAccPlain, false, false, KF, H>();
    }
}
template <int KF, typename F>
void dispatch_pair(int tile_t, int mode, bool h16, F& f) {
    if (h16) dispatch_pair_form<KF, true>(tile_t, mode, f);
    else dispatch_pair_form<KF, false>(tile_t, mode, f);
}

// The kernel variant of (tile_t, mode, full, adapt, kernel pair, operand
// form); 64-row tiles are plain.
template <typename F>
void dispatch(int tile_t, int mode, bool full, bool adapt, int kf, bool h16, F&& f) {
    if (kf == kKernelQuartic) return dispatch_pair<kKernelQuartic>(tile_t, mode, h16, f);
    if (kf == kKernelGauss) return dispatch_pair<kKernelGauss>(tile_t, mode, h16, f);
    if (kf == kKernelPrinted) return dispatch_pair<kKernelPrinted>(tile_t, mode, h16, f);
    if (tile_t == 16) {
        if (mode == kAccKahanReg) dispatch_variant<16, kAccKahanReg>(full, adapt, h16, f);
        else if (mode == kAccKahanMem) dispatch_variant<16, kAccKahanMem>(full, adapt, h16, f);
        else dispatch_variant<16, kAccPlain>(full, adapt, h16, f);
    } else if (tile_t == 32) {
        if (mode == kAccKahanReg) dispatch_variant<32, kAccKahanReg>(full, adapt, h16, f);
        else if (mode == kAccKahanMem) dispatch_variant<32, kAccKahanMem>(full, adapt, h16, f);
        else dispatch_variant<32, kAccPlain>(full, adapt, h16, f);
    } else {
        dispatch_variant<64, kAccPlain>(full, adapt, h16, f);
    }
}

template <int TT, bool K>
void launch_reduce_t(const InstDev* d, int32_t count, const uint32_t* top, const uint32_t* sc,
                     const float* partials, hipStream_t s) {
    hipLaunchKernelGGL((k_reduce_split<TT, K>), dim3(256), dim3(kThreads), 0, s, d, count, top, sc,
                       partials);
}

}  // namespace

hipError_t launch_gather_items(const InstDev* d_desc, int32_t count, const WorkItem* d_items,
                               const uint32_t* d_bits, const uint32_t* d_scalars,
                               uint32_t* d_counters, float* d_partials, float* d_kscratch, int64_t T,
                               int tile_t, int mode, bool full, bool adapt, int kf, bool h16,
                               hipStream_t s) {
    dispatch(tile_t, mode, full, adapt, kf, h16, [&]<int TT, int M, bool F, bool A, int K, bool H>() {
        launch_items_t<TT, M, F, A, K, H>(d_desc, count, d_items, d_bits, d_scalars, d_counters, d_partials,
                                          d_kscratch, T, s);
    });
    return hipGetLastError();
}

void prepare_gather(int tile_t, int mode, bool full, bool adapt, int kf, bool h16) {
    dispatch(tile_t, mode, full, adapt, kf, h16,
             []<int TT, int M, bool F, bool A, int K, bool H>() { (void)resident_groups<TT, M, F, A, K, H>(); });
}

hipError_t launch_reduce_split(const InstDev* d_desc, int32_t count, const uint32_t* d_top,
                               const uint32_t* d_scalars, const float* d_partials, int tile_t,
                               bool kahan, hipStream_t s) {
    if (tile_t == 16) {
        kahan ? launch_reduce_t<16, true>(d_desc, count, d_top, d_scalars, d_partials, s)
              : launch_reduce_t<16, false>(d_desc, count, d_top, d_scalars, d_partials, s);
    } else if (tile_t == 32) {
        kahan ? launch_reduce_t<32, true>(d_desc, count, d_top, d_scalars, d_partials, s)
              : launch_reduce_t<32, false>(d_desc, count, d_top, d_scalars, d_partials, s);
    } else {
        launch_reduce_t<64, false>(d_desc, count, d_top, d_scalars, d_partials, s);
    }
    return hipGetLastError();
}

}  // namespace stkde
