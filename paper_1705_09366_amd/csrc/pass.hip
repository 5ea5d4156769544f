// pass.hip -- one gather pass over a list of instances: the tile work list
// (candidate cost per tile, heaviest-first order, splitting of the costliest
// tiles), the gather, the reduction of split tiles, and the per-instance
// FP64 mass and statistics.
//
// Load balance follows Sec. 5.2.  Greedy list scheduling finishes within
// (total work - longest task)/P + longest task (Graham's bound quoted there),
// so two things matter: the order and the longest task.  The cost of a tile
// is the number of points it must examine (the points of its neighbouring
// bins); the costliest tiles are queued first, in non-increasing cost (the
// order of PB-SYM-PD-SCHED), and a tile whose cost exceeds a fixed share of
// its instance's total is cut into contiguous candidate ranges whose partial
// grids are added afterwards in part order (the replication of the critical
// path of PB-SYM-PD-REP, with its extra initialisation and reduction).
// Everything here is deterministic: the queues only change which workgroup
// computes an item, never what it computes.
#include "stkde_internal.h"

namespace stkde {
namespace {

struct DescChunk {
    InstDev d[kDescChunk];
};
static_assert(sizeof(DescChunk) <= 4096, "descriptors must fit the kernel-argument space");

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// Descriptors arrive as kernel arguments, so that a captured pass carries
// them in its graph; the first chunk also clears the pass counters.
__global__ __launch_bounds__(256) void k_put_desc(DescChunk c, int32_t first, int32_t m,
                                                  InstDev* __restrict__ dst,
                                                  unsigned long long* __restrict__ inst_cost,
                                                  uint32_t* __restrict__ inst_split,
                                                  uint32_t* __restrict__ mass_done,
                                                  uint32_t* __restrict__ hist,
                                                  uint32_t* __restrict__ cursor,
                                                  uint32_t* __restrict__ demand,
                                                  uint32_t* __restrict__ sc, int32_t clear) {
    const int tid = threadIdx.x;
    if (tid < m) {
        dst[first + tid] = c.d[tid];
        inst_cost[first + tid] = 0ull;
        inst_split[first + tid] = 0u;
        mass_done[first + tid] = 0u;
    }
    if (clear) {
        for (int k = tid; k < kCostClasses; k += 256) {
            hist[k] = 0u;
            cursor[k] = 0u;
            demand[k] = 0u;
        }
        if (tid < kScCount) sc[tid] = 0u;
    }
}

__device__ inline uint32_t cost_class(uint32_t c) { return __float_as_uint((float)c) >> 20; }

// Candidates of global tile j of instance D (the points of the bins the
// gather reads for it): bin rows (t, y) in batches of 16, each batch's 32
// offsets loaded together; (ct, cy) walks the rows with y fastest.
__device__ inline uint32_t tile_candidates(const InstDev& D, uint32_t j, int32_t rows) {
    const int32_t tile = (int32_t)(j - (uint32_t)D.tile_base);
    const int32_t tx = tile % D.ntx;
    const int32_t rest = tile / D.ntx;
    const int32_t ty = rest % D.nty;
    const int32_t tt = rest / D.nty;
    const TileBins b = tile_bins(D, tx * kTileXY + D.ox, ty * kTileXY + D.oy, tt * rows + D.ot, rows);
    const int32_t nyr = b.cy1 - b.cy0 + 1;
    const int32_t nrows = nyr * (b.ct1 - b.ct0 + 1);
    int32_t ct = b.ct0, cy = b.cy0;
    uint32_t c = 0;
    for (int32_t r0 = 0; r0 < nrows; r0 += 16) {
        uint32_t hi[16], lo[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            hi[u] = lo[u] = 0u;
            if (r0 + u < nrows) {
                const int32_t row = (ct * D.ncy + cy) * D.ncx;
                hi[u] = as_global(D.cell_start)[row + b.cx1 + 1];
                lo[u] = as_global(D.cell_start)[row + b.cx0];
                if (cy == b.cy1) {
                    cy = b.cy0;
                    ++ct;
                } else {
                    ++cy;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) c += hi[u] - lo[u];
    }
    return c;
}

// Candidates per tile, the cost class histogram, and per-instance totals.
__global__ __launch_bounds__(256) void k_tile_cost(const InstDev* __restrict__ descs, int32_t count,
                                                   uint32_t T, uint32_t* __restrict__ cost,
                                                   uint32_t* __restrict__ hist,
                                                   unsigned long long* __restrict__ inst_cost,
                                                   uint32_t* __restrict__ bits) {
    __shared__ uint32_t h[kCostClasses];
    const int tid = threadIdx.x, lane = tid & 63;
    for (int k = tid; k < kCostClasses; k += 256) h[k] = 0u;
    __syncthreads();
    const uint32_t j = blockIdx.x * 256u + (uint32_t)tid;
    const bool valid = j < T;
    if (valid && (j & 31u) == 0) bits[j >> 5] = 0u;
    uint32_t c = 0;
    int32_t inst = 0;
    if (valid) {
        inst = find_inst(descs, count, j);
        c = tile_candidates(descs[inst], j, descs[inst].tile_t);
        cost[j] = c;
        atomicAdd(&h[cost_class(c)], 1u);
    }
    // per-instance totals: one atomic per wave unless the wave spans instances
    const int32_t i0 = __shfl(inst, 0, 64);
    if (__ballot(valid && inst != i0) == 0ull) {
        unsigned long long v = c;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
        if (lane == 0 && v) atomicAdd(&inst_cost[i0], v);
    } else if (valid && c) {
        atomicAdd(&inst_cost[inst], (unsigned long long)c);
    }
    __syncthreads();
    for (int k = tid; k < kCostClasses; k += 256)
        if (h[k]) atomicAdd(&hist[k], h[k]);
}

// Exclusive prefix sum over a 256-thread workgroup; *total gets the sum.
__device__ inline uint32_t block_scan256(uint32_t v, uint32_t* ws, uint32_t* total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    __syncthreads();  // the previous scan's readers are done with ws
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t x = ws[k];
        pre += k < w ? x : 0u;
        tot += x;
    }
    *total = tot;
    return pre + inc - v;
}

// Split threshold of a tile of instance D: max(kSplitFloor, total cost /
// split share); its parts: min(kMaxParts, ceil(cost / threshold)).
__device__ inline uint32_t split_parts(const InstDev& D, unsigned long long inst_total, uint32_t c) {
    const unsigned long long ss = D.split_share;
    const unsigned long long share = (inst_total + ss - 1) / ss;
    const uint32_t thr = share > kSplitFloor ? (share > 0xffffffffull ? 0xffffffffu : (uint32_t)share)
                                             : kSplitFloor;
    if (c <= thr) return 1u;
    const uint32_t want = (uint32_t)(((unsigned long long)c + thr - 1) / thr);
    return want < (uint32_t)kMaxParts ? want : (uint32_t)kMaxParts;
}

// The heaviest-first queue, in one launch.
//
// Every workgroup derives from the cost-class histogram the threshold class
// (the smallest class c >= class(1) whose suffix count, tiles of class >= c,
// is at most kTopTiles) and the number of heavy tiles in the classes above
// each class; it places its heavy tiles (those of the threshold class and
// above) into heavy[] grouped by class, costliest class first (in any order
// within a class), flags them in the spatial queue's bitmask, and adds the
// partial slots each would take if split to its class's demand.
//
// The last workgroup to finish then plans the queue: tiles are split (into
// split_parts parts) in the costliest classes whose summed demand fits the
// partial slots, every tile of a class or none, so that which tiles are cut
// depends only on the costs, not on the order of heavy[]; it writes the work
// items and split records in heavy[] order, and clears the queues' counters.
__global__ __launch_bounds__(256) void k_collect_plan(const InstDev* __restrict__ descs, int32_t count,
                                                      uint32_t T, const uint32_t* __restrict__ cost,
                                                      const uint32_t* __restrict__ hist,
                                                      const unsigned long long* __restrict__ inst_cost,
                                                      uint32_t* __restrict__ inst_split,
                                                      uint32_t* __restrict__ cursor,
                                                      uint32_t* __restrict__ demand,
                                                      unsigned long long* __restrict__ heavy,
                                                      WorkItem* __restrict__ items,
                                                      uint32_t* __restrict__ top,
                                                      uint32_t* __restrict__ bits,
                                                      uint32_t* __restrict__ sc,
                                                      uint32_t* __restrict__ ctr, uint32_t nslots,
                                                      uint32_t* __restrict__ done) {
    constexpr int kPer = kCostClasses / 256;  // classes per thread, highest first
    static_assert(kPer * 256 == kCostClasses, "whole classes per thread");
    __shared__ uint32_t above[kCostClasses];  // heavy tiles in the classes above c
    // this workgroup's heavy tiles per class (its base in heavy[] once
    // reserved) and their slot demand: one global atomic per class present,
    // not one per tile (same-address atomics serialise)
    __shared__ uint32_t lcnt[kCostClasses];
    __shared__ uint32_t ldem[kCostClasses];
    __shared__ uint32_t ws[4];
    __shared__ uint32_t s_cls, s_last;
    // one workgroup (up to 2048 tiles): heavy[] and the demand stay in LDS,
    // without the global atomics and the hand-over to a last workgroup
    __shared__ unsigned long long sheavy[kTopTiles];
    const bool one = gridDim.x == 1;
    const int tid = threadIdx.x;
    for (int k = tid; k < kCostClasses; k += 256) {
        lcnt[k] = 0u;
        ldem[k] = 0u;
    }
    // the costs are loaded first, so that their loads overlap the threshold's
    constexpr int kU = 8;  // loads in flight per thread
    const uint32_t j0 = blockIdx.x * (256u * kU) + tid;
    uint32_t cv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const uint32_t j = j0 + 256u * u;
        cv[u] = j < T ? cost[j] : 0u;
    }
    // suffix counts over the classes, thread tid holding classes
    // kCostClasses - 1 - (kPer tid + u), highest first
    if (tid == 0) s_cls = kCostClasses;
    uint32_t h[kPer], sum = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        h[u] = hist[kCostClasses - 1 - (kPer * tid + u)];
        sum += h[u];
    }
    uint32_t tot;
    uint32_t run = block_scan256(sum, ws, &tot);  // tiles in the classes above this thread's
    const uint32_t cmin = cost_class(1u);
    uint32_t best = kCostClasses;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const uint32_t c = kCostClasses - 1 - (kPer * tid + u);
        above[c] = run;
        run += h[u];
        if (c >= cmin && run <= (uint32_t)kTopTiles) best = c;
    }
    if (best < kCostClasses) atomicMin(&s_cls, best);
    __syncthreads();
    const uint32_t cls = s_cls;
    uint32_t rank[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const uint32_t c = cv[u], j = j0 + 256u * u;
        rank[u] = 0xffffffffu;
        if (c != 0u && cost_class(c) >= cls) {
            const uint32_t k = cost_class(c);
            rank[u] = atomicAdd(&lcnt[k], 1u);
            const int32_t inst = find_inst(descs, count, j);
            const uint32_t parts = split_parts(descs[inst], inst_cost[inst], c);
            if (parts > 1) atomicAdd(&ldem[k], parts);
            const uint32_t sp = spatial_pos(descs[inst], j);
            atomicOr(&bits[sp >> 5], 1u << (sp & 31u));
        }
    }
    __syncthreads();
    // reserve each class's run in heavy[]; lcnt becomes the run's base
    for (int k = tid; k < kCostClasses; k += 256) {
        if (one) {
            lcnt[k] = above[k];
        } else {
            if (lcnt[k]) lcnt[k] = above[k] + atomicAdd(&cursor[k], lcnt[k]);  // < kTopTiles by the choice of cls
            if (ldem[k]) atomicAdd(&demand[k], ldem[k]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const uint32_t c = cv[u], j = j0 + 256u * u;
        if (rank[u] != 0xffffffffu) {
            const uint32_t at = lcnt[cost_class(c)] + rank[u];
            const unsigned long long v = ((unsigned long long)c << 32) | j;
            if (one) sheavy[at] = v;
            else heavy[at] = v;
        }
    }
    // the last workgroup plans the queue
    if (!one) {
        __threadfence();
        __syncthreads();
        if (tid == 0) s_last = atomicAdd(done, 1u) == gridDim.x - 1 ? 1u : 0u;
        __syncthreads();
        if (!s_last) return;
        __threadfence();
    } else {
        __syncthreads();
    }
    const uint32_t nh = (cls < (uint32_t)kCostClasses) ? above[cls] + hist[cls] : 0u;
    // split classes: the costliest classes whose demand fits the slots
    uint32_t dm[kPer], dsum = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const uint32_t k = kCostClasses - 1 - (kPer * tid + u);
        dm[u] = one ? ldem[k] : __hip_atomic_load(&demand[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        dsum += dm[u];
    }
    uint32_t dtot;
    uint32_t drun = block_scan256(dsum, ws, &dtot);
    uint32_t cut = kCostClasses;  // lowest class that may split
    if (tid == 0) s_cls = kCostClasses;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        drun += dm[u];
        if (drun <= nslots) cut = kCostClasses - 1 - (kPer * tid + u);
    }
    if (cut < kCostClasses) atomicMin(&s_cls, cut);
    __syncthreads();
    const uint32_t split_cls = s_cls;
    // heavy[] in order, four entries per thread
    constexpr int kE = kTopTiles / 256;
    uint32_t tl[kE], cc[kE], np[kE];
    int32_t ins[kE];
    uint32_t n_items = 0, n_slots = 0, n_split = 0;
#pragma unroll
    for (int e = 0; e < kE; ++e) {
        const uint32_t k = (uint32_t)(kE * tid + e);
        tl[e] = cc[e] = 0u;
        np[e] = 0u;
        ins[e] = 0;
        if (k < nh) {
            const unsigned long long v =
                one ? sheavy[k] : __hip_atomic_load(&heavy[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            tl[e] = (uint32_t)v;
            cc[e] = (uint32_t)(v >> 32);
            ins[e] = find_inst(descs, count, tl[e]);
            np[e] = cost_class(cc[e]) >= split_cls ? split_parts(descs[ins[e]], inst_cost[ins[e]], cc[e]) : 1u;
            n_items += np[e];
            n_slots += np[e] > 1 ? np[e] : 0u;
            n_split += np[e] > 1 ? 1u : 0u;
        }
    }
    uint32_t tot_items, tot_slots, tot_split;
    uint32_t ipos = block_scan256(n_items, ws, &tot_items);
    uint32_t spos0 = block_scan256(n_slots, ws, &tot_slots);
    uint32_t kpos = block_scan256(n_split, ws, &tot_split);
#pragma unroll
    for (int e = 0; e < kE; ++e) {
        const uint32_t k = (uint32_t)(kE * tid + e);
        if (k >= nh) continue;
        const uint32_t parts = np[e], c = cc[e], tile = tl[e];
        for (uint32_t p = 0; p < parts; ++p) {
            const uint32_t b = (uint32_t)(((unsigned long long)c * p) / parts);
            const uint32_t en = p + 1 == parts ? kAll : (uint32_t)(((unsigned long long)c * (p + 1)) / parts);
            items[ipos + p] = WorkItem{tile, b, en, parts > 1 ? spos0 + p : kNoSlot};
        }
        ipos += parts;
        if (parts > 1) {
            atomicAdd(&inst_split[ins[e]], 1u);
            top[4 * kpos + 0] = tile;
            top[4 * kpos + 1] = parts;
            top[4 * kpos + 2] = spos0;
            top[4 * kpos + 3] = c;
            spos0 += parts;
            ++kpos;
        }
    }
    for (int k = tid; k < kCtrWords; k += 256) ctr[k] = 0u;  // both queues' counters
    if (tid == 0) {
        sc[kScHeavyItems] = tot_items;
        sc[kScSplit] = tot_split;
        sc[kScHeavyTiles] = nh;
        if (!one) *done = 0u;
    }
}

// The whole planning of a pass of at most 256 tiles and kDescChunk grids, in
// one workgroup, tile j on thread j: the descriptors arrive as arguments (this
// kernel stores them for the later ones and clears the pass counters), the
// tile costs as k_tile_cost counts them.  With so few tiles the work list of
// k_collect_plan reduces to: every tile with candidates is heavy (at most
// 256 <= kTopTiles of them), and it is cut into split_parts parts when the
// costliest classes' slot demand fits the partial slots -- every candidate
// of a class whose suffix demand (over the classes at and above it) is at
// most nslots -- the same tiles and parts; the items follow in tile order,
// which changes only which workgroup computes an item.
__global__ __launch_bounds__(256) void k_plan_small(DescChunk dc, int32_t count, uint32_t T,
                                                    InstDev* __restrict__ gdesc,
                                                    uint32_t* __restrict__ inst_split,
                                                    uint32_t* __restrict__ mass_done,
                                                    WorkItem* __restrict__ items,
                                                    uint32_t* __restrict__ top,
                                                    uint32_t* __restrict__ bits,
                                                    uint32_t* __restrict__ sc,
                                                    uint32_t* __restrict__ ctr, uint32_t nslots) {
    __shared__ InstDev sdesc[kDescChunk];
    __shared__ unsigned long long sic[kDescChunk];
    __shared__ uint32_t ssplit[kDescChunk];
    __shared__ uint32_t sbits[256 / 32];
    __shared__ uint32_t scls[256], sdem[256];
    __shared__ uint32_t ws[4];
    const int tid = threadIdx.x;
    if (tid < count) {
        sdesc[tid] = dc.d[tid];
        gdesc[tid] = dc.d[tid];
        sic[tid] = 0ull;
        ssplit[tid] = 0u;
        mass_done[tid] = 0u;
    }
    if (tid < 256 / 32) sbits[tid] = 0u;
    __syncthreads();
    const uint32_t j = (uint32_t)tid;
    const bool valid = j < T;
    int32_t inst = 0;
    uint32_t c = 0;
    if (valid) {
        inst = find_inst(sdesc, count, j);
        c = tile_candidates(sdesc[inst], j, sdesc[inst].tile_t);
        if (c) atomicAdd(&sic[inst], (unsigned long long)c);
    }
    __syncthreads();
    const bool heavy = valid && c != 0u;
    uint32_t parts = heavy ? split_parts(sdesc[inst], sic[inst], c) : 0u;
    if (heavy) {
        const uint32_t sp = spatial_pos(sdesc[inst], j);
        atomicOr(&sbits[sp >> 5], 1u << (sp & 31u));
    }
    // the cut: a tile that would split does when the demand of its class and
    // the costlier ones fits the slots (computed tile by tile only when the
    // whole demand does not fit)
    const uint32_t dem = parts > 1 ? parts : 0u;
    uint32_t dtot;
    (void)block_scan256(dem, ws, &dtot);
    if (dtot > nslots) {
        const uint32_t k = heavy ? cost_class(c) : 0u;
        scls[tid] = k;
        sdem[tid] = dem;
        __syncthreads();
        uint32_t suffix = 0;
        for (int u = 0; u < 256; ++u) suffix += scls[u] >= k ? sdem[u] : 0u;
        if (dem && suffix > nslots) parts = 1u;
    }
    uint32_t tot_items, tot_slots, tot_split, tot_heavy;
    const uint32_t ipos = block_scan256(parts, ws, &tot_items);
    const uint32_t spos = block_scan256(parts > 1 ? parts : 0u, ws, &tot_slots);
    const uint32_t kpos = block_scan256(parts > 1 ? 1u : 0u, ws, &tot_split);
    (void)block_scan256(heavy ? 1u : 0u, ws, &tot_heavy);
    for (uint32_t p = 0; p < parts; ++p) {
        const uint32_t b = (uint32_t)(((unsigned long long)c * p) / parts);
        const uint32_t en = p + 1 == parts ? kAll : (uint32_t)(((unsigned long long)c * (p + 1)) / parts);
        items[ipos + p] = WorkItem{j, b, en, parts > 1 ? spos + p : kNoSlot};
    }
    if (parts > 1) {
        atomicAdd(&ssplit[inst], 1u);
        top[4 * kpos + 0] = j;
        top[4 * kpos + 1] = parts;
        top[4 * kpos + 2] = spos;
        top[4 * kpos + 3] = c;
    }
    for (int k = tid; k < kCtrWords; k += 256) ctr[k] = 0u;  // both queues' counters
    __syncthreads();
    if (tid < (int)((T + 31) / 32)) bits[tid] = sbits[tid];
    if (tid < count) inst_split[tid] = ssplit[tid];
    if (tid < kScCount)
        sc[tid] = tid == kScHeavyItems ? tot_items
                : tid == kScSplit     ? tot_split
                : tid == kScHeavyTiles ? tot_heavy
                                       : 0u;
}

// Each instance's FP64 grid sum in a fixed order: the instance's tile
// partials are cut into nch = min(kMassChunks, ceil(partials / 2048))
// chunks; workgroup (chunk, inst) sums its chunk (strided per-thread sums,
// then a tree) into mid[inst][chunk], and the last of the instance's nch
// workgroups to finish adds the chunks (a butterfly over 64 lanes, zero past
// nch) and writes the instance's statistics (write_stats).  An instance of
// one chunk (at most 512 tiles) writes them at once, without the hand-over.
__global__ __launch_bounds__(256) void k_mass(const InstDev* __restrict__ descs, double* __restrict__ mid,
                                              const uint32_t* __restrict__ inst_split,
                                              uint32_t* __restrict__ mass_done) {
    static_assert(kMassChunks == 64, "one wave adds an instance's chunks");
    __shared__ double sh[256];
    __shared__ uint32_t s_last;
    const int inst = blockIdx.y, ch = blockIdx.x, tid = threadIdx.x;
    const InstDev& D = descs[inst];
    if (!D.stats) return;  // nothing to report (every workgroup of the instance leaves)
    const int64_t cnt = (D.flags & kInstMass) ? (int64_t)D.ntiles * kWaves : 0;
    const int64_t nch64 = (cnt + kMassChunkMin - 1) / kMassChunkMin;
    const int nch = nch64 < 1 ? 1 : (nch64 > kMassChunks ? kMassChunks : (int)nch64);
    if (ch >= nch) return;
    double s = 0.0;
    {
        const int64_t chunk = (cnt + nch - 1) / nch;
        const int64_t beg = (int64_t)ch * chunk;
        const int64_t end = beg + chunk < cnt ? beg + chunk : cnt;
        for (int64_t i = beg + tid; i < end; i += 256) s += as_global(D.tile_part)[i];
    }
    sh[tid] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (tid < w) sh[tid] += sh[tid + w];
        __syncthreads();
    }
    if (nch == 1) {
        if (tid == 0) write_stats(D, sh[0], inst_split[inst]);
        return;
    }
    if (tid == 0) {
        __hip_atomic_store(&mid[(size_t)inst * kMassChunks + ch], sh[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        s_last = atomicAdd(&mass_done[inst], 1u) == (uint32_t)nch - 1 ? 1u : 0u;
    }
    __syncthreads();
    if (!s_last || tid >= 64) return;
    __threadfence();
    const int lane = tid;
    double v = lane < nch ? __hip_atomic_load(&mid[(size_t)inst * kMassChunks + lane], __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT)
                          : 0.0;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0) {
        write_stats(D, v, inst_split[inst]);
        mass_done[inst] = 0u;
    }
}

}  // namespace

PassLayout layout_pass(const InstGeom* inst, int32_t count, int tile_t, bool kahan) {
    PassLayout l{};
    int64_t T = 0, parts = 0;
    for (int32_t i = 0; i < count; ++i) {
        T += inst[i].ntiles;
        parts += (int64_t)inst[i].ntiles * kWaves;
    }
    size_t o = 0;
    l.T = T;
    l.desc = o; o = al256(o + (size_t)count * sizeof(InstDev));
    l.inst_cost = o; o = al256(o + (size_t)count * 8);
    l.inst_split = o; o = al256(o + (size_t)count * 4);
    l.mass_done = o; o = al256(o + (size_t)count * 4);
    l.cost = o; o = al256(o + (size_t)T * 4);
    l.hist = o; o = al256(o + (size_t)kCostClasses * 4);
    l.cursor = o; o = al256(o + (size_t)kCostClasses * 4);
    l.demand = o; o = al256(o + (size_t)kCostClasses * 4);
    l.bits = o; o = al256(o + ((size_t)T + 31) / 32 * 4);
    l.scalars = o; o = al256(o + (size_t)kScCount * 4);
    l.counters = o; o = al256(o + (size_t)kCtrWords * 4);
    l.heavy = o; o = al256(o + (size_t)kTopTiles * 8);
    l.top = o; o = al256(o + (size_t)kTopTiles * 16);
    l.items = o; o = al256(o + (size_t)kTopTiles * kMaxParts * sizeof(WorkItem));
    l.partials = o; o = al256(o + (size_t)part_slots(T) * kTileXY * kTileXY * tile_t * 4);
    l.kscratch = o;
    // per thread: (sum, compensation) of 4 column groups x tile_t/16 row blocks, f32x4 each
    if (kahan) o = al256(o + (size_t)kahan_slots(T) * kThreads * 2 * (4 * (tile_t / 16)) * 16);
    l.tile_part = o; o = al256(o + (size_t)parts * 8);
    l.mass_mid = o; o = al256(o + (size_t)count * kMassChunks * 8);
    l.total = o;
    return l;
}

hipError_t launch_pass(InstDev* descs, int32_t count, uint8_t* pass, const PassLayout& pl,
                       int tile_t, int mode, bool full, bool adapt, int kf, bool h16, hipStream_t s,
                       hipEvent_t ev_before, hipEvent_t ev_after, bool multi) {
    const bool kahan = mode != kAccPlain;
    InstDev* d_desc = reinterpret_cast<InstDev*>(pass + pl.desc);
    auto* inst_cost = reinterpret_cast<unsigned long long*>(pass + pl.inst_cost);
    auto* inst_split = reinterpret_cast<uint32_t*>(pass + pl.inst_split);
    auto* mass_done = reinterpret_cast<uint32_t*>(pass + pl.mass_done);
    auto* cost = reinterpret_cast<uint32_t*>(pass + pl.cost);
    auto* hist = reinterpret_cast<uint32_t*>(pass + pl.hist);
    auto* cursor = reinterpret_cast<uint32_t*>(pass + pl.cursor);
    auto* demand = reinterpret_cast<uint32_t*>(pass + pl.demand);
    auto* bits = reinterpret_cast<uint32_t*>(pass + pl.bits);
    auto* sc = reinterpret_cast<uint32_t*>(pass + pl.scalars);
    auto* ctr = reinterpret_cast<uint32_t*>(pass + pl.counters);
    auto* top = reinterpret_cast<uint32_t*>(pass + pl.top);
    auto* items = reinterpret_cast<WorkItem*>(pass + pl.items);
    auto* partials = reinterpret_cast<float*>(pass + pl.partials);
    auto* kscratch = reinterpret_cast<float*>(pass + pl.kscratch);
    auto* tile_part = reinterpret_cast<double*>(pass + pl.tile_part);
    auto* mid = reinterpret_cast<double*>(pass + pl.mass_mid);
    auto* heavy = reinterpret_cast<unsigned long long*>(pass + pl.heavy);

    bool any_stats = false;
    int64_t tb = 0;
    for (int32_t i = 0; i < count; ++i) {
        descs[i].tile_base = (int32_t)tb;
        descs[i].tile_part = tile_part + tb * kWaves;
        tb += descs[i].ntiles;
        any_stats = any_stats || descs[i].stats != nullptr;
    }
    const uint32_t T = (uint32_t)pl.T;
    if (T <= 256u && count <= kDescChunk) {
        // a pass of at most 256 tiles is planned by one workgroup in one launch
        DescChunk dc{};
        for (int32_t k = 0; k < count; ++k) dc.d[k] = descs[k];
        hipLaunchKernelGGL(k_plan_small, dim3(1), dim3(256), 0, s, dc, count, T, d_desc, inst_split, mass_done,
                           items, top, bits, sc, ctr, (uint32_t)part_slots(pl.T));
    } else {
        for (int32_t first = 0; first < count; first += kDescChunk) {
            DescChunk c{};
            const int32_t m = count - first < kDescChunk ? count - first : kDescChunk;
            for (int32_t k = 0; k < m; ++k) c.d[k] = descs[first + k];
            hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(256), 0, s, c, first, m, d_desc, inst_cost,
                               inst_split, mass_done, hist, cursor, demand, sc, first == 0 ? 1 : 0);
        }
        hipLaunchKernelGGL(k_tile_cost, dim3((T + 255) / 256), dim3(256), 0, s, (const InstDev*)d_desc,
                           count, T, cost, hist, inst_cost, bits);
        hipLaunchKernelGGL(k_collect_plan, dim3((T + 2047) / 2048), dim3(256), 0, s, (const InstDev*)d_desc,
                           count, T, (const uint32_t*)cost, (const uint32_t*)hist,
                           (const unsigned long long*)inst_cost, inst_split, cursor, demand, heavy, items, top,
                           bits, sc, ctr, (uint32_t)part_slots(pl.T), sc + kScPlanDone);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev_before && (e = hipEventRecord(ev_before, s)) != hipSuccess) return e;
    e = multi ? launch_gather_multi(d_desc, count, items, bits, sc, ctr, partials, kscratch, pl.T, kahan, s)
              : launch_gather_items(d_desc, count, items, bits, sc, ctr, partials, kscratch, pl.T, tile_t, mode,
                                    full, adapt, kf, h16, s);
    if (e != hipSuccess) return e;
    if (ev_after && (e = hipEventRecord(ev_after, s)) != hipSuccess) return e;
    e = multi ? launch_reduce_split_multi(d_desc, count, top, sc, partials, kahan, s)
              : launch_reduce_split(d_desc, count, top, sc, partials, tile_t, kahan, s);
    if (e != hipSuccess) return e;
    if (any_stats)
        hipLaunchKernelGGL(k_mass, dim3(kMassChunks, (uint32_t)count), dim3(256), 0, s, (const InstDev*)d_desc,
                           mid, (const uint32_t*)inst_split, mass_done);
    return hipGetLastError();
}

}  // namespace stkde
