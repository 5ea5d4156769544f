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
// every workgroup leaves after one failed fetch per counter; in the
// single-variant kernel a queue that fits the grid of workgroups is handed
// out without counters.  One launch serves any number of instances (grids
// with their own bandwidths and windows over their own binned sets).
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
//           scaled by the normalisation (2/pi)(3/4)/(n hs^2 ht) (32-row tiles
//           of the single-variant kernel without the full-cover path:
//           non-temporal stores); a part of a split tile writes its unscaled
//           sums to a partial slot instead, and the split reduction adds the
//           parts in part order.
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
// The LDS of one gather variant (one member of a union in the kernel that
// serves several variants).
template <int TT, int MODE, bool FULL, bool ADAPT, int KF, bool H16>
struct GatherLds {
    static constexpr int kCap = H16 ? kCapH16 : kCapF32;
    static constexpr int kLPad = H16 ? 32 : 8;  // wave lists are padded to this many entries
    static constexpr bool EXACT = KF == kKernelGauss || KF == kKernelPrinted;
    // survivor list: tile-local coordinates as (head, tail) pairs and the
    // quadrants its footprint box meets; entry kCap is a point far outside
    // every tile (one block, so that the full-cover partial sums can reuse it)
    float2 sXYT[3 * (kCap + 1)];
    uint8_t sQ[kCap];
    // per-point bandwidth terms of the survivors (ADAPT only)
    float4 sB[ADAPT ? kCap + 1 : 1];
    // record index of each survivor (pairs with exact support tests only)
    uint32_t sI[EXACT ? kCap + 1 : 1];
    // per-wave lists of survivor indices meeting the wave's quadrant, padded to
    // kLPad (two-term FP16 kernels: in h16_slot order)
    alignas(16) uint16_t sL[kWaves][kCap + kLPad];
    // full-cover kernels: each wave's share of the tile-cover survivors and its
    // quadrant-cover survivors (one scan fills all three lists)
    uint16_t sF[FULL ? kWaves : 1][FULL ? kCap / 4 + 8 : 1];
    uint16_t sQL[FULL ? kWaves : 1][FULL ? kCap + 8 : 1];
    int32_t sRB[kMaxRanges];
    int32_t sRP[kMaxRanges + 1];
    int32_t sWC[kWaves];

    // The padding survivor (one thread; read only after later barriers).
    __device__ void put_pad() {
        sXYT[kCap] = make_float2(-1.0e6f, 0.f);
        sXYT[2 * kCap + 1] = make_float2(-1.0e6f, 0.f);
        sXYT[3 * kCap + 2] = make_float2(-1.0e6f, 0.f);
        if constexpr (ADAPT) sB[kCap] = make_float4(1.0f, 1.0f, 0.0f, 0.0f);
        if constexpr (EXACT) sI[kCap] = 0u;  // never read: the pad is far from every boundary
    }
};

// One work item of the gather (see the header): a tile, or one part of a
// split tile.  taken: the tile is the heaviest-first queue's (the item came
// from the spatial queue and is skipped after the set-up).  q, pend, pnext,
// k, c: the fetch state of the calling loop (spatial queue: the next
// position of counter c, index k, is taken during a short tile's set-up).
template <int TT, int MODE, bool FULL, bool ADAPT, int KF, bool H16>
__device__ __attribute__((always_inline)) inline void gather_item(
    GatherLds<TT, MODE, FULL, ADAPT, KF, H16>& S, const InstDev* __restrict__ descs, int32_t count,
    const WorkItem it, const uint32_t taken, const int q, bool& pend, uint32_t& pnext, const uint32_t k,
    uint32_t* c, float* __restrict__ partials, float* __restrict__ kscratch, const int32_t kstride,
    const int32_t pstride) {
    static_assert(!(FULL && ADAPT), "the full-cover path assumes one bandwidth pair");
    static_assert(KF == kKernelEpan || (!FULL && !ADAPT), "other pairs: no full-cover path, one pair");
    static_assert(!H16 || (!ADAPT && TT <= 32 && MODE != kAccKahanReg),
                  "two-term FP16 operands: one bandwidth pair, 16/32 rows, no register-form Kahan");
    using Lds = GatherLds<TT, MODE, FULL, ADAPT, KF, H16>;
    constexpr int kCap = Lds::kCap;
    constexpr int kLPad = Lds::kLPad;
    constexpr int NB = TT / 16;  // 16-row blocks per tile
    constexpr int CG = 4 * NB;   // accumulator blocks per wave
    constexpr bool EXACT = Lds::EXACT;
    // Kahan with the running (sum, compensation) in memory: this thread's
    // slot of kscratch (kstride f32x4 per thread, at least 2 CG), sum of
    // block k at [k], compensation at [CG + k]
    f32x4* __restrict__ kslot =
        MODE == kAccKahanMem
            ? reinterpret_cast<f32x4*>(kscratch) + ((size_t)blockIdx.x * kThreads + threadIdx.x) * kstride
            : nullptr;
    constexpr int kPad = kCap;  // index of the padding survivor
    float2* const sXYT = S.sXYT;
    float2* const sX = sXYT;
    float2* const sY = sXYT + (kCap + 1);
    float2* const sT = sXYT + 2 * (kCap + 1);
    uint8_t* const sQ = S.sQ;
    float4* const sB = S.sB;
    uint32_t* const sI = S.sI;
    auto& sL = S.sL;
    auto& sF = S.sF;
    auto& sQL = S.sQL;
    int32_t* const sRB = S.sRB;
    int32_t* const sRP = S.sRP;
    int32_t* const sWC = S.sWC;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
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

#define GATHER_NEXT_ITEM return
#define GATHER_STORE_NT false
#include "gather_item.inc"
#undef GATHER_STORE_NT
#undef GATHER_NEXT_ITEM
}

// The persistent gather of one variant: items first from the heaviest-first
// queue, then from the spatial queue (see the header).
template <int TT, int MODE, bool FULL, bool ADAPT, int KF, bool H16>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(
    (MODE == kAccKahanReg || FULL || ADAPT || TT == 64 || H16) ? 4 : 6, 8))) void k_gather_items(
    const InstDev* __restrict__ descs, int32_t count, int32_t ntiles_total,
    const WorkItem* __restrict__ items, const uint32_t* __restrict__ bits,
    const uint32_t* __restrict__ sc, uint32_t* __restrict__ ctr, float* __restrict__ partials,
    float* __restrict__ kscratch) {
    static_assert(!(FULL && ADAPT), "the full-cover path assumes one bandwidth pair");
    static_assert(KF == kKernelEpan || (!FULL && !ADAPT), "other pairs: no full-cover path, one pair");
    static_assert(!H16 || (!ADAPT && TT <= 32 && MODE != kAccKahanReg),
                  "two-term FP16 operands: one bandwidth pair, 16/32 rows, no register-form Kahan");
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
        // an empty queue is skipped without reading its counters (the spatial
        // queue is empty when the heaviest-first queue took every tile)
        const uint32_t qlen = q == 0 ? sc[kScHeavyItems] : (sc[kScHeavyTiles] >= T ? 0u : T);
        // queues of at most one item per workgroup are not fetched from: the
        // heaviest-first queue's item b goes to workgroup b, and when both
        // queues together fit the grid, the spatial queue's item j to
        // workgroup (heavy items) + j, one that holds no heavy item (every
        // workgroup is resident, so each item starts at once, as with the
        // counters, and no workgroup walks them)
        const uint32_t sbase = q == 0 ? 0u : sc[kScHeavyItems];
        const bool dyn = sbase + qlen > gridDim.x;
        for (uint32_t lane_off = 0; qlen > 0 && lane_off < (dyn ? (uint32_t)kFetchLanes : 1u); ++lane_off) {
            const uint32_t k = (home + lane_off) % kFetchLanes;
            uint32_t* c = ctr + (q * kFetchLanes + k) * kCtrStride;
            // spatial queue: after the set-up of a tile that takes one phase, the
            // next position of this counter is taken at once, so that the
            // atomic's latency is hidden behind the tile's work (taking it
            // early for longer tiles costs more in balance than it saves; a
            // queue not fetched from ignores that position)
            bool pend = false, first = true;
            uint32_t pnext = 0;
            for (;;) {
                if (tid == 0) {
                    uint32_t v;
                    if (!dyn) {
                        v = first && blockIdx.x >= sbase ? blockIdx.x - sbase : 0xffffffffu;
                    } else if (pend) {
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
                first = false;
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
                constexpr int32_t pstride = kTileXY * kTileXY * TT;  // floats per partial slot
#define GATHER_NEXT_ITEM continue
#define GATHER_STORE_NT true
#include "gather_item.inc"
#undef GATHER_STORE_NT
#undef GATHER_NEXT_ITEM
            }
        }
    }
}

// A gather variant as a type (the parameters of k_gather_items).
template <int TT_, int MODE_, bool FULL_, bool ADAPT_, int KF_, bool H16_>
struct GVar {
    static constexpr int TT = TT_, MODE = MODE_, KF = KF_;
    static constexpr bool FULL = FULL_, ADAPT = ADAPT_, H16 = H16_;
    using Lds = GatherLds<TT_, MODE_, FULL_, ADAPT_, KF_, H16_>;
};

template <class... Vs>
constexpr size_t max_lds_bytes() {
    size_t m = 0;
    ((m = sizeof(typename Vs::Lds) > m ? sizeof(typename Vs::Lds) : m), ...);
    return m;
}
template <class... Vs>
constexpr int max_rows() {
    int m = 0;
    ((m = Vs::TT > m ? Vs::TT : m), ...);
    return m;
}

// The persistent gather over grids of several variants in one launch (a
// batch whose grids differ in tile rows, accumulation mode or operand form):
// the same queues and fetch loop as k_gather_items, and each item runs the
// item code of its grid's variant (InstDev::variant indexes Vs), so every grid
// gets the operations, and the bits, of a launch of its own variant.  The
// variants' LDS is one block; a workgroup re-places the padding survivor when
// its variant changes.  Memory-form Kahan slots and split-tile partial slots
// are spaced for the largest variant.
template <class... Vs>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_gather_multi(
    const InstDev* __restrict__ descs, int32_t count, int32_t ntiles_total,
    const WorkItem* __restrict__ items, const uint32_t* __restrict__ bits,
    const uint32_t* __restrict__ sc, uint32_t* __restrict__ ctr, float* __restrict__ partials,
    float* __restrict__ kscratch) {
    __shared__ __align__(16) uint8_t lds[max_lds_bytes<Vs...>()];
    __shared__ uint32_t sIdx;
    constexpr int kRowsMax = max_rows<Vs...>();
    const int tid = threadIdx.x;
    int32_t held = -1;  // the variant whose padding survivor the LDS holds

    const uint32_t T = (uint32_t)ntiles_total;
    const uint32_t home = blockIdx.x % kFetchLanes;
    for (int q = 0; q < 2; ++q) {
        // an empty queue is skipped without reading its counters (the spatial
        // queue is empty when the heaviest-first queue took every tile)
        const uint32_t qlen = q == 0 ? sc[kScHeavyItems] : (sc[kScHeavyTiles] >= T ? 0u : T);
        // (every queue is fetched from here: the static hand-out of short
        // queues, as in k_gather_items, measured 20 % slower in this kernel,
        // whose register allocation spills)
        for (uint32_t lane_off = 0; qlen > 0 && lane_off < (uint32_t)kFetchLanes; ++lane_off) {
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
                const int32_t var = descs[find_inst(descs, count, it.tile)].variant;  // uniform
                if (var != held) {
                    held = var;
                    int32_t vi = 0;
                    ((var == vi++ && tid == 0 ? (reinterpret_cast<typename Vs::Lds*>(lds)->put_pad(), 0) : 0), ...);
                }
                int32_t vi = 0;
                ((var == vi++ ? (gather_item<Vs::TT, Vs::MODE, Vs::FULL, Vs::ADAPT, Vs::KF, Vs::H16>(
                                     *reinterpret_cast<typename Vs::Lds*>(lds), descs, count, it, taken, q, pend,
                                     pnext, k, c, partials, kscratch, 2 * 4 * (kRowsMax / 16),
                                     kTileXY * kTileXY * kRowsMax),
                                 0)
                              : 0),
                 ...);
            }
        }
    }
}

// The kernel of a variant list, as a type.
template <class... Vs>
struct k_gather_multi_t {
    static auto kernel() { return k_gather_multi<Vs...>; }
};

// One split tile: add its parts' partial sums (slots slot0 .. slot0 + parts - 1,
// pstride floats apart) in part order, scale, store, and write the tile's mass
// partials.  Thread k owns column (k / 16, k % 16).
template <int TT, bool KAHAN>
__device__ __attribute__((always_inline)) inline void reduce_split_tile(const InstDev& D, uint32_t tile_g,
                                                                        uint32_t parts, uint32_t slot0,
                                                                        const float* __restrict__ partials,
                                                                        int32_t pstride) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int32_t lx = tid / kTileXY, ly = tid % kTileXY;
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
                                              partials + (size_t)(slot0 + p) * pstride + (size_t)tid * TT + r)
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

// Split tiles of a pass with one tile height.
template <int TT, bool KAHAN>
__global__ __launch_bounds__(kThreads) void k_reduce_split(const InstDev* __restrict__ descs,
                                                           int32_t count,
                                                           const uint32_t* __restrict__ top,
                                                           const uint32_t* __restrict__ sc,
                                                           const float* __restrict__ partials) {
    const uint32_t nsplit = sc[kScSplit];
    for (uint32_t k = blockIdx.x; k < nsplit; k += gridDim.x) {
        const uint32_t tile_g = top[4 * k], parts = top[4 * k + 1], slot0 = top[4 * k + 2];
        reduce_split_tile<TT, KAHAN>(descs[find_inst(descs, count, tile_g)], tile_g, parts, slot0, partials,
                                     kTileXY * kTileXY * TT);
    }
}

// Split tiles of a pass whose grids have 16- or 32-row tiles (a batch in one
// launch): each tile reduced by the code of its grid's height, the partial
// slots 16 x 16 x 32 floats apart.
template <bool KAHAN>
__global__ __launch_bounds__(kThreads) void k_reduce_split_multi(const InstDev* __restrict__ descs,
                                                                 int32_t count,
                                                                 const uint32_t* __restrict__ top,
                                                                 const uint32_t* __restrict__ sc,
                                                                 const float* __restrict__ partials) {
    const uint32_t nsplit = sc[kScSplit];
    for (uint32_t k = blockIdx.x; k < nsplit; k += gridDim.x) {
        const uint32_t tile_g = top[4 * k], parts = top[4 * k + 1], slot0 = top[4 * k + 2];
        const InstDev& D = descs[find_inst(descs, count, tile_g)];
        if (D.tile_t == 16)
            reduce_split_tile<16, KAHAN>(D, tile_g, parts, slot0, partials, kTileXY * kTileXY * 32);
        else
            reduce_split_tile<32, KAHAN>(D, tile_g, parts, slot0, partials, kTileXY * kTileXY * 32);
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
        if (full) {
            if constexpr (MODE != kAccKahanReg) {
                if (h16) f.template operator()<TT, MODE, true, false, kKernelEpan, true>();
                else f.template operator()<TT, MODE, true, false, kKernelEpan, false>();
            } else {
                f.template operator()<TT, MODE, true, false, kKernelEpan, false>();
            }
        } else if constexpr (MODE != kAccKahanReg) {
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

// The variant lists of the multi-variant gather, in multi_variant order:
// full-cover FP32 operands 16, 32 rows; two-term FP16 operands 16, 32 rows.
// Compensated sums keep their pair in scratch in every variant here: the
// register form of the full-cover variants (the form a grid of theirs takes
// alone; the same operations, the same bits) made the kernel spill about 127
// VGPRs at its 128-register bound (batch sweep 3.73 -> 3.52 ms without).
using MultiKahan = k_gather_multi_t<GVar<16, kAccKahanMem, true, false, kKernelEpan, false>,
                                    GVar<32, kAccKahanMem, true, false, kKernelEpan, false>,
                                    GVar<16, kAccKahanMem, false, false, kKernelEpan, true>,
                                    GVar<32, kAccKahanMem, false, false, kKernelEpan, true>>;
using MultiPlain = k_gather_multi_t<GVar<16, kAccPlain, true, false, kKernelEpan, false>,
                                    GVar<32, kAccPlain, true, false, kKernelEpan, false>,
                                    GVar<16, kAccPlain, false, false, kKernelEpan, true>,
                                    GVar<32, kAccPlain, false, false, kKernelEpan, true>>;

// Workgroups of a multi-variant gather, as resident_groups (its compensated
// form holds memory-form Kahan slots: at most kMemKahanGroups).
template <class M>
int resident_multi() {
    static std::atomic<int> cache[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v > 0) return v;
    int ncu = 0, occ = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) ncu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, M::kernel(), kThreads, 0) != hipSuccess) occ = 0;
    v = (ncu > 0 ? ncu : 256) * (occ > 0 ? occ : 1);
    if (v > kMemKahanGroups) v = kMemKahanGroups;
    cache[dev].store(v, std::memory_order_relaxed);
    return v;
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

hipError_t launch_gather_multi(const InstDev* d_desc, int32_t count, const WorkItem* d_items,
                               const uint32_t* d_bits, const uint32_t* d_scalars, uint32_t* d_counters,
                               float* d_partials, float* d_kscratch, int64_t T, bool kahan, hipStream_t s) {
    auto run = [&]<class M>() {
        int64_t g = resident_multi<M>();
        const int64_t most = max_items(T);  // (the Kahan scratch holds kahan_slots(T) workgroups)
        if (g > most) g = most;
        if (g < 1) g = 1;
        hipLaunchKernelGGL(M::kernel(), dim3((uint32_t)g), dim3(kThreads), 0, s, d_desc, count, (int32_t)T, d_items,
                           d_bits, d_scalars, d_counters, d_partials, d_kscratch);
    };
    if (kahan) run.template operator()<MultiKahan>();
    else run.template operator()<MultiPlain>();
    return hipGetLastError();
}

void prepare_gather_multi(bool kahan) {
    if (kahan) (void)resident_multi<MultiKahan>();
    else (void)resident_multi<MultiPlain>();
}

hipError_t launch_reduce_split_multi(const InstDev* d_desc, int32_t count, const uint32_t* d_top,
                                     const uint32_t* d_scalars, const float* d_partials, bool kahan,
                                     hipStream_t s) {
    if (kahan)
        hipLaunchKernelGGL((k_reduce_split_multi<true>), dim3(256), dim3(kThreads), 0, s, d_desc, count, d_top,
                           d_scalars, d_partials);
    else
        hipLaunchKernelGGL((k_reduce_split_multi<false>), dim3(256), dim3(kThreads), 0, s, d_desc, count, d_top,
                           d_scalars, d_partials);
    return hipGetLastError();
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
