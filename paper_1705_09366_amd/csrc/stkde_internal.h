// stkde_internal.h -- layouts and launch interfaces shared by the library's
// HIP sources (binning, work lists, gather, statistics) and its host entry
// points.
//
// Units: every quantity below is in voxel units unless named otherwise.  A
// point's voxel-space coordinate is xr = (x - x0)/sres (likewise y, and t with
// tres); the voxel bandwidths are hv = hs/sres and tv = ht/tres, and the
// integer loop bounds Hs = ceil(hv), Ht = ceil(tv) of Sec. 2.1.
//
// Two geometries meet in every computation:
//  * a *binned set*: points transformed into the voxel space of a base grid,
//    sorted into bins and stored as 32-byte records, with the largest
//    bandwidths the set will be used with (they clip the footprint boxes);
//  * an *instance*: one density grid -- the base grid or a voxel-aligned
//    window of it -- with its own bandwidths, at most the set's.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace stkde {

// A 256-thread workgroup owns a 16 x 16 x TT tile of voxels; each of its four
// waves owns an 8 x 8 quadrant of columns, i.e. four 4 x 4 column groups,
// times TT/16 blocks of 16 rows, as FP32 matrix-core accumulators.
constexpr int kTileXY = 16;
constexpr int kWaves = 4;
constexpr int kThreads = 256;
// Bin rows (t, y) a tile may read; the plan picks bin sizes to respect it.
constexpr int kMaxRanges = 64;

// Per-point record in sorted (binned) order, 32 bytes.  Each voxel-space
// coordinate is split into an FP32 head and an FP16 tail (c = head + tail to
// ~2^-35 relative), so that tile-local offsets keep FP64-class accuracy where
// it matters (near the point) although every kernel below works in FP32.
struct alignas(16) PointRec {
    float xh, yh, th;
    uint32_t xb;       // footprint columns in x: lo | hi << 16, clipped to the base grid
    uint32_t yb;       // footprint columns in y: lo | hi << 16
    uint32_t tb;       // footprint rows in t: lo | hi << 16
    uint32_t xl_yl;    // tails of x and y as two FP16 (x in the low half)
    uint32_t tl;       // tail of t as FP16 in the low half
};
static_assert(sizeof(PointRec) == 32, "record layout");

// Binning geometry of a point set.
// Keys of the points that are never visited sort after every bin: culled
// (footprint off the grid) ncell + 0, invalid bandwidth pair ncell + 1,
// non-finite coordinate ncell + 2.  Their bin offsets give their counts.
constexpr int32_t kKeyCulled = 0, kKeyBadBw = 1, kKeyNonFinite = 2, kKeySentinels = 3;

struct SetGeom {
    int32_t gx, gy, gt;       // base grid
    int32_t cx, cxy, ct;      // bin edge in x, in y, and in t (voxels)
    int32_t ncx, ncy, nct;    // bins per axis
    int32_t ncell;            // ncx * ncy * nct
    double x0, y0, t0;
    double sres, tres;
    double hv, tv;            // largest voxel bandwidths (footprint boxes)
};

// Geometry of one density grid (an instance).
struct InstGeom {
    int32_t gx, gy, gt;       // instance grid
    int32_t ox, oy, ot;       // its voxel (0,0,0) in the base grid of its set
    int32_t Hs, Ht;           // ceil(hv), ceil(tv), capped by the grid extent
    int32_t tile_t;           // rows per tile (16 or 32)
    int32_t ntx, nty, ntt;    // tiles per axis
    int32_t ntiles;
    double x0, y0, t0, sres, tres;
    double hs, ht;            // domain bandwidths (normalisation)
    double hv, tv;            // voxel bandwidths
    double Hs_d, Ht_d;        // ceil(hv), ceil(tv) uncapped (loop bounds of the statistics)
    float inv_hv2, inv_tv2;   // 1/hv^2, 1/tv^2 (FP32)
    int32_t kernel;           // kKernel*: the kernel pair
};

// Per-instance descriptor the device work list refers to (pass scratch copy).
struct alignas(16) InstDev {
    const uint32_t* cell_start;          // set: bin offsets
    const PointRec* recs;                // set: records in bin order
    const float4* bw;                    // set: per record (1/hv_i^2, 1/tv_i^2, weight, 0) when
                                         // its points carry their own bandwidths, else null
    const double* x64;                   // set: per record its FP64 voxel coordinates (xr, yr, tr)
                                         // for the exact support tests of the pairs that are not
                                         // zero on their boundary, else null
    float* out;                          // instance grid, [X][Y][T], T fastest
    double* stats;                       // optional 8 doubles, null for none
    double* tile_part;                   // pass scratch: ntiles * kWaves FP64 mass partials
    double mass_scale;                   // sres^2 tres
    int32_t gx, gy, gt;                  // instance grid
    int32_t ox, oy, ot;                  // its voxel (0,0,0) in the set's base grid
    int32_t Hs, Ht;                      // instance loop bounds
    int32_t cx, cxy, ct, ncx, ncy, nct;  // set bins (edges in x, y, t; bins per axis)
    int32_t ntx, nty, ntiles, tile_base; // instance tiles; first global tile index
    uint32_t flags;                      // kInstMass, kInstFull
    float inv_hv2, inv_tv2, cnorm;
    float inv_hv, inv_tv;                // 1/hv, 1/tv (the pair as printed is odd in u, v, w)
    double hv64, tv64;                   // hv, tv in FP64 (exact support tests)
    uint32_t split_share;                // split tiles above total cost / split_share
    int32_t tile_t;                      // rows per tile
    int32_t variant;                     // gather variant (index in a multi-variant pass), else 0
};
// Kernel pairs (the public STKDE_KERNEL_* values).
constexpr int kKernelEpan = 0;
constexpr int kKernelQuartic = 1;
constexpr int kKernelGauss = 2;
constexpr int kKernelPrinted = 3;
constexpr uint32_t kInstMass = 1u;
constexpr uint32_t kInstFull = 2u;  // use the full-cover path (in a kernel that has it)

// One unit of gather work: a tile, a range of its candidate sequence and
// where the result goes (the grid, or a partial slot of a split tile).
struct alignas(16) WorkItem {
    uint32_t tile;            // global tile index (instances concatenated)
    uint32_t cbeg, cend;      // candidate range; cend = kAll for "to the end"
    uint32_t slot;            // partial slot, kNoSlot = store to the grid
};
constexpr uint32_t kAll = 0xffffffffu;
constexpr uint32_t kNoSlot = 0xffffffffu;

// Keys per thread of a radix block: 8 (blocks of 2048 keys), or 2 (512) for
// sets of at most kSmallSort points, whose few blocks would otherwise each
// take eight dependent rounds.
constexpr int kSortItems = 8;
constexpr int kSortItemsSmall = 2;
constexpr int64_t kSmallSort = 65536;
inline int sort_items(int64_t n) { return n <= kSmallSort ? kSortItemsSmall : kSortItems; }
constexpr int kStatBlock = 256;                       // points per statistics block
constexpr int kTopTiles = 1024;                       // most tiles in the heaviest-first queue
constexpr int kMaxParts = 8;                          // parts of one split tile
constexpr int kPartSlots = 1024;                      // partial tiles of one pass
constexpr uint32_t kSplitFloor = 2048;                // never split below this many candidates
constexpr uint32_t kBalanceItems = 2048;              // default split share of an instance's cost
constexpr int kMassChunks = 64;
constexpr int64_t kMassChunkMin = 2048;  // tile partials per mass chunk, at least
// Accumulation modes of the gather: plain FP32; Kahan with the running
// (sum, compensation) pair in registers; the same pair kept in a per-workgroup
// scratch slot, touched only when a tile takes more than one phase (fewer
// registers, so more resident workgroups).  The two Kahan modes perform the
// same operations in the same order and give identical bits.
constexpr int kAccPlain = 0;
constexpr int kAccKahanReg = 1;
constexpr int kAccKahanMem = 2;
constexpr int kMemKahanGroups = 1536;  // workgroups (scratch slots) in memory mode
// Work items of a pass over T tiles: every tile once, the heavy ones (at
// most kTopTiles) in up to kMaxParts parts; the persistent gather never runs
// more workgroups than that, and a pass never needs more partial slots than
// its heavy tiles' parts.
inline int64_t max_items(int64_t T) { return T + (int64_t)(kMaxParts - 1) * (T < kTopTiles ? T : kTopTiles); }
inline int64_t part_slots(int64_t T) {
    const int64_t m = (int64_t)kMaxParts * (T < kTopTiles ? T : kTopTiles);
    return m < kPartSlots ? m : kPartSlots;
}
inline int64_t kahan_slots(int64_t T) { return max_items(T) < kMemKahanGroups ? max_items(T) : kMemKahanGroups; }
// Full-cover path of the gather: a point whose disc covers the whole 16 x 16
// columns of a tile adds Kt (1 - a(x) - b(y)) there, which two 16 x 16
// products (sum of Kt (a - 1) over x, sum of Kt b over y) give for all the
// tile's columns at once.  Used from this voxel bandwidth on (below it few
// discs can cover a tile).
constexpr double kFullMinHv = 14.0;                       // first-level chunks of an instance's mass sum
constexpr int kDescChunk = 16;                        // descriptors written per launch
// Cost class of a tile: the FP32 bit pattern of its candidate count without
// the low 20 bits (exponent and 3 mantissa bits), monotone in the count.
constexpr int kCostClasses = 2048;

// Queue positions are handed out by kFetchLanes interleaved counters:
// counter k gives positions k, k + kFetchLanes, k + 2 kFetchLanes, ...  A
// workgroup draws from counter (its index mod kFetchLanes) and then from the
// others, so the positions in flight stay compact while no single address
// takes every workgroup's atomic (same-address atomics serialise; one
// counter per queue measured ~12 ns per fetch times the number of
// workgroups).
constexpr int kFetchLanes = 16;
// Counters sit 256 bytes apart: atomics to one cache line serialise like
// atomics to one address.
constexpr int kCtrStride = 64;  // u32

// Scalars of a pass (u32 offsets into PassLayout::scalars).
constexpr int kScHeavyItems = 0;  // items in the heaviest-first queue
constexpr int kScSplit = 1;       // split tiles
constexpr int kScHeavyTiles = 2;  // tiles in the heaviest-first queue
constexpr int kScPlanDone = 3;    // workgroups of the queue planning that have finished
constexpr int kScCount = 8;
// Counters (u32 offsets into PassLayout::counters): queue q, lane k at
// (q * kFetchLanes + k) * kCtrStride.
constexpr int kCtrWords = 2 * kFetchLanes * kCtrStride;

// ---- set memory (caller-owned, persistent) --------------------------------
struct SetLayout {
    size_t cell_start;   // (ncell + kKeySentinels + 1) u32
    size_t recs;         // n PointRec
    size_t bw;           // n float4 (per-point bandwidths; 0 bytes without)
    size_t x64;          // n x 3 FP64 voxel coordinates (exact support tests; 0 bytes without)
    size_t total;
};
SetLayout layout_set(const SetGeom& s, int64_t n, bool adaptive = false, bool exact = false);

// ---- scratch of the binning radix sort --------------------------------------
struct SortLayout {
    size_t keys0, vals0, keys1, vals1, hist, totals;
    // a sort of one pass (keys of at most 11 bits): keys0, then the records,
    // bandwidth terms and FP64 voxel coordinates of the valid points in input
    // order (no value or second key array)
    size_t prec, pbw, px64;
    size_t total;
    int32_t nblk;    // radix blocks of kThreads * items keys
    int32_t items;   // sort_items(n)
    bool one_pass;   // the geometry's keys take one pass
    bool adaptive;   // room for per-point bandwidth terms
    bool exact;      // room for FP64 voxel coordinates
};
SortLayout layout_sort(const SetGeom& g, int64_t n, bool adaptive = false, bool exact = false);

// ---- scratch of one gather pass over `count` instances ---------------------
struct PassLayout {
    size_t desc;         // count InstDev
    size_t inst_cost;    // count u64: candidates summed over the instance's tiles
    size_t inst_split;   // count u32: tiles of the instance computed in parts
    size_t mass_done;    // count u32: mass workgroups of the instance that have finished
    size_t cost;         // T u32: candidates per tile
    size_t hist;         // kCostClasses u32: tiles per cost class
    size_t cursor;       // kCostClasses u32: heavy tiles placed per class
    size_t demand;       // kCostClasses u32: partial slots the class's heavy tiles would take
    size_t bits;         // ceil(T / 32) u32: spatial-queue positions taken by the heavy queue
    size_t scalars;      // kScCount u32
    size_t counters;     // kCtrWords u32: the queues' fetch counters
    size_t heavy;        // kTopTiles u64 (cost << 32 | tile) of the heavy tiles, by class
    size_t top;          // kTopTiles x 4 u32 split tiles: tile, parts, slot0, candidates
    size_t items;        // kTopTiles * kMaxParts WorkItem (the heaviest-first queue)
    size_t partials;     // part_slots(T) x 16 x 16 x tile_t FP32
    size_t kscratch;     // Kahan plans: kahan_slots(T) x kThreads x 2 x (4 tile_t/16) f32x4
    size_t tile_part;    // sum over instances of ntiles * kWaves FP64
    size_t mass_mid;     // count * kMassChunks FP64
    size_t total;
    int64_t T;           // total tiles
};
PassLayout layout_pass(const InstGeom* inst, int32_t count, int tile_t, bool kahan);

// Global-memory view of a device pointer.  Pointers the kernels read from
// descriptors are generic to the compiler, and generic (flat) accesses count
// against both the vector-memory and the LDS wait counters: every LDS wait
// would also wait for them (the records in flight, the grid stores).
template <typename T>
__device__ inline __attribute__((address_space(1))) T* as_global(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}

// Instance holding global tile `tile` (descriptors ordered by tile_base).
__device__ inline int32_t find_inst(const InstDev* __restrict__ d, int32_t count, uint32_t tile) {
    int32_t lo = 0, hi = count - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if ((uint32_t)d[mid].tile_base <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ inline int32_t floordiv_i(int32_t a, int32_t b) {
    const int32_t q = a / b;
    return (a % b != 0 && a < 0) ? q - 1 : q;
}

__device__ inline int32_t clamp_i32(int32_t v, int32_t lo, int32_t hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

// Bins a tile may draw points from: a point reaches column X only if floor(xr)
// lies in [X - Hs, X + Hs] (rows likewise with Ht); one voxel of margin on each
// side absorbs rounding of the footprint bounds.  (bx0, by0, bt0) is the tile
// origin in the set's base grid.  The plan keeps
// (cy1 - cy0 + 1) * (ct1 - ct0 + 1) <= kMaxRanges.
struct TileBins {
    int32_t cx0, cx1, cy0, cy1, ct0, ct1;
};
__device__ inline TileBins tile_bins(const InstDev& D, int32_t bx0, int32_t by0, int32_t bt0,
                                     int32_t rows) {
    TileBins b;
    b.cx0 = clamp_i32(floordiv_i(bx0 - D.Hs - 1, D.cx), 0, D.ncx - 1);
    b.cx1 = clamp_i32(floordiv_i(bx0 + kTileXY - 1 + D.Hs + 1, D.cx), 0, D.ncx - 1);
    b.cy0 = clamp_i32(floordiv_i(by0 - D.Hs - 1, D.cxy), 0, D.ncy - 1);
    b.cy1 = clamp_i32(floordiv_i(by0 + kTileXY - 1 + D.Hs + 1, D.cxy), 0, D.ncy - 1);
    b.ct0 = clamp_i32(floordiv_i(bt0 - D.Ht - 1, D.ct), 0, D.nct - 1);
    b.ct1 = clamp_i32(floordiv_i(bt0 + rows - 1 + D.Ht + 1, D.ct), 0, D.nct - 1);
    return b;
}

// The spatial queue visits an instance's tiles with t fastest, then y, then
// x (consecutive tiles share bins and write neighbouring runs of each
// column); global tile index = tile_base + (tt * nty + ty) * ntx + tx.
__device__ inline uint32_t spatial_tile(const InstDev& D, uint32_t k) {
    const uint32_t local = k - (uint32_t)D.tile_base;
    const uint32_t ntt = (uint32_t)D.ntiles / ((uint32_t)D.ntx * (uint32_t)D.nty);
    const uint32_t tt = local % ntt, r = local / ntt;
    const uint32_t ty = r % (uint32_t)D.nty, tx = r / (uint32_t)D.nty;
    return (uint32_t)D.tile_base + (tt * (uint32_t)D.nty + ty) * (uint32_t)D.ntx + tx;
}
// Inverse of spatial_tile: the queue position of global tile j.
__device__ inline uint32_t spatial_pos(const InstDev& D, uint32_t j) {
    const uint32_t local = j - (uint32_t)D.tile_base;
    const uint32_t ntt = (uint32_t)D.ntiles / ((uint32_t)D.ntx * (uint32_t)D.nty);
    const uint32_t tx = local % (uint32_t)D.ntx, r = local / (uint32_t)D.ntx;
    const uint32_t ty = r % (uint32_t)D.nty, tt = r / (uint32_t)D.nty;
    return (uint32_t)D.tile_base + (tx * (uint32_t)D.nty + ty) * ntt + tt;
}

// ---- an instance's statistics ------------------------------------------------
// d_stats of instance D from its grid sum v and its count of split tiles:
// [0] grid mass (v * sres^2 tres, or 0 without the mass flag), [1], [2], [7]
// = 0, [3], [4], [5] = the set's non-finite, culled and invalid-bandwidth
// counts (the offsets of their keys), [6] = tiles computed in parts.
__device__ inline void write_stats(const InstDev& D, double v, uint32_t nsplit) {
    auto* st = as_global(D.stats);
    st[0] = (D.flags & kInstMass) ? v * D.mass_scale : 0.0;
    st[1] = 0.0;
    st[2] = 0.0;
    const auto* cs = as_global(D.cell_start + (size_t)D.ncx * D.ncy * D.nct);
    st[3] = (double)(cs[kKeyNonFinite + 1] - cs[kKeyNonFinite]);
    st[4] = (double)(cs[kKeyCulled + 1] - cs[kKeyCulled]);
    st[5] = (double)(cs[kKeyBadBw + 1] - cs[kKeyBadBw]);
    st[6] = (double)nsplit;
    st[7] = 0.0;
}

// ---- launchers (asynchronous on s; return the launch error) ---------------
// Bin n points into set memory `set` using radix scratch `sort`.  d_hst
// (n x 2 FP64 per-point bandwidths in domain units, or null) makes each
// point's footprint and record terms its own; a pair that is not finite and
// positive, or exceeds the set's bandwidths, drops the point (counted).
hipError_t launch_bin(const SetGeom& g, const double* d_xyt, int32_t n, uint8_t* set,
                      const SetLayout& sl, uint8_t* sort, const SortLayout& so, hipStream_t s,
                      const double* d_hst = nullptr, bool exact = false);
// Work list, gather, split reduction, mass and statistics over `count`
// instances.  The descriptors' tile_part and tile_base fields are filled in
// here; every other field is the caller's.
// ev_before / ev_after (may be null) are recorded on s right before and
// right after the gather kernel.
// full: use the gather's full-cover path (tile_t <= 32); adapt: the
// instances' sets carry per-point bandwidths (never with full); kf: the
// kernel pair (other than Epanechnikov: neither full nor adapt, tile_t <= 32);
// h16: two-term FP16 matrix-core operands (Epanechnikov, neither full nor
// adapt, tile_t <= 32, mode not kAccKahanReg; ignored elsewhere).
// multi: a pass over grids of several gather variants in one launch
// (launch_gather_multi; tile_t and the layout pl are then those of 32-row
// tiles, the spacing of its slots; mode gives plain or compensated; full,
// adapt, kf and h16 are per grid, in each descriptor's variant).
hipError_t launch_pass(InstDev* descs, int32_t count, uint8_t* pass, const PassLayout& pl,
                       int tile_t, int mode, bool full, bool adapt, int kf, bool h16, hipStream_t s,
                       hipEvent_t ev_before = nullptr, hipEvent_t ev_after = nullptr, bool multi = false);
// The gather proper (called by launch_pass).
hipError_t launch_gather_items(const InstDev* d_desc, int32_t count, const WorkItem* d_items,
                               const uint32_t* d_bits, const uint32_t* d_scalars,
                               uint32_t* d_counters, float* d_partials, float* d_kscratch, int64_t T,
                               int tile_t, int mode, bool full, bool adapt, int kf, bool h16,
                               hipStream_t s);
// Query (and cache) the gather's launch size for the current device ahead of a
// stream capture.
void prepare_gather(int tile_t, int mode, bool full, bool adapt, int kf, bool h16);
// The multi-variant gather of a batch (Epanechnikov pair, one bandwidth pair
// per grid): plain or compensated; each grid's InstDev::variant is
// multi_variant(its tile rows, its operand form) -- the full-cover FP32
// kernel (register-form Kahan when compensated) or the two-term FP16 kernel
// (scratch-form Kahan), 16 or 32 rows; those variants give every grid the
// bits of its own pass.  Split-tile partial slots are 16 x 16 x 32 floats.
inline int32_t multi_variant(int tile_t, bool h16) { return (h16 ? 2 : 0) + (tile_t == 32 ? 1 : 0); }
hipError_t launch_gather_multi(const InstDev* d_desc, int32_t count, const WorkItem* d_items,
                               const uint32_t* d_bits, const uint32_t* d_scalars, uint32_t* d_counters,
                               float* d_partials, float* d_kscratch, int64_t T, bool kahan, hipStream_t s);
void prepare_gather_multi(bool kahan);
hipError_t launch_reduce_split_multi(const InstDev* d_desc, int32_t count, const uint32_t* d_top,
                                     const uint32_t* d_scalars, const float* d_partials, bool kahan,
                                     hipStream_t s);
hipError_t launch_reduce_split(const InstDev* d_desc, int32_t count, const uint32_t* d_top,
                               const uint32_t* d_scalars, const float* d_partials, int tile_t,
                               bool kahan, hipStream_t s);
// d_stats[1], [2] from per-point FP64 sums of one instance (part: nblk x 4
// doubles); d_hst as for launch_bin (null: the instance's bandwidths).
hipError_t launch_point_stats(const InstGeom& g, int64_t n_norm, const double* d_xyt, int32_t n,
                              double* d_stats, double* part, int32_t nblk, hipStream_t s,
                              const double* d_hst = nullptr);

// Baselines over a binned set on its own base grid (no window): a zero fill
// then a point-parallel atomic scatter, or a voxel-parallel gather over bins.
hipError_t launch_ablation_scatter(const SetGeom& sg, const InstGeom& ig, const uint8_t* set,
                                   const SetLayout& sl, float cnorm, float* d_out, hipStream_t s);
hipError_t launch_ablation_voxel(const SetGeom& sg, const InstGeom& ig, const uint8_t* set,
                                 const SetLayout& sl, float cnorm, float* d_out, hipStream_t s);

}  // namespace stkde
