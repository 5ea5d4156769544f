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
                                                  uint32_t* __restrict__ hist,
                                                  uint32_t* __restrict__ sc, int32_t clear) {
    const int tid = threadIdx.x;
    if (tid < m) {
        dst[first + tid] = c.d[tid];
        inst_cost[first + tid] = 0ull;
        inst_split[first + tid] = 0u;
    }
    if (clear) {
        for (int k = tid; k < kCostClasses; k += 256) hist[k] = 0u;
        if (tid < kScCount) sc[tid] = 0u;
    }
}

__device__ inline uint32_t cost_class(uint32_t c) { return __float_as_uint((float)c) >> 20; }

// Candidates per tile (the points of the bins the gather reads), the cost
// class histogram, and per-instance totals.
__global__ __launch_bounds__(256) void k_tile_cost(const InstDev* __restrict__ descs, int32_t count,
                                                   uint32_t T, int32_t rows,
                                                   uint32_t* __restrict__ cost,
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
        const InstDev& D = descs[inst];
        const int32_t tile = (int32_t)(j - (uint32_t)D.tile_base);
        const int32_t tx = tile % D.ntx;
        const int32_t rest = tile / D.ntx;
        const int32_t ty = rest % D.nty;
        const int32_t tt = rest / D.nty;
        const TileBins b = tile_bins(D, tx * kTileXY + D.ox, ty * kTileXY + D.oy, tt * rows + D.ot, rows);
        // bin rows (t, y) in batches of 16, each batch's 32 offsets loaded
        // together; (ct, cy) walks the rows with y fastest
        const int32_t nyr = b.cy1 - b.cy0 + 1;
        const int32_t nrows = nyr * (b.ct1 - b.ct0 + 1);
        int32_t ct = b.ct0, cy = b.cy0;
        for (int32_t r0 = 0; r0 < nrows; r0 += 16) {
            uint32_t hi[16], lo[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                hi[u] = lo[u] = 0u;
                if (r0 + u < nrows) {
                    const int32_t row = (ct * D.ncy + cy) * D.ncx;
                    hi[u] = D.cell_start[row + b.cx1 + 1];
                    lo[u] = D.cell_start[row + b.cx0];
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

// Exclusive prefix sum over a 1024-thread workgroup; *total gets the sum.
__device__ inline uint32_t block_scan(uint32_t v, uint32_t* ws, uint32_t* total) {
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
    for (int k = 0; k < 16; ++k) {
        const uint32_t x = ws[k];
        pre += k < w ? x : 0u;
        tot += x;
    }
    *total = tot;
    return pre + inc - v;
}

// Threshold class of the heaviest-first queue: the smallest class c >=
// class(1) whose suffix count (tiles of class >= c) is at most kTopTiles.
// Every workgroup of k_collect_heavy derives it from the histogram alone.
__device__ inline uint32_t heavy_class(const uint32_t* __restrict__ hist, uint32_t* ws,
                                       uint32_t* s_cls) {
    const int tid = threadIdx.x;
    constexpr int kPer = kCostClasses / 256;  // classes per thread, highest first
    static_assert(kPer * 256 == kCostClasses, "whole classes per thread");
    if (tid == 0) *s_cls = kCostClasses;
    uint32_t h[kPer], sum = 0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        h[u] = hist[kCostClasses - 1 - (kPer * tid + u)];
        sum += h[u];
    }
    // exclusive scan over the 256 threads (classes above this thread's)
    const int lane = tid & 63, w = tid >> 6;
    uint32_t inc = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t v = __shfl_up(inc, o, 64);
        if (lane >= o) inc += v;
    }
    if (lane == 63) ws[w] = inc;
    __syncthreads();
    uint32_t above = inc - sum;
    for (int k = 0; k < w; ++k) above += ws[k];
    const uint32_t cmin = cost_class(1u);
    uint32_t best = kCostClasses;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const uint32_t c = kCostClasses - 1 - (kPer * tid + u);
        above += h[u];
        if (c >= cmin && above <= (uint32_t)kTopTiles) best = c;
    }
    if (best < kCostClasses) atomicMin(s_cls, best);
    __syncthreads();
    return *s_cls;
}

// Collect the heavy tiles (those of the threshold class and above) into
// heavy[] in any order; k_plan_items sorts them.
__global__ __launch_bounds__(256) void k_collect_heavy(uint32_t T, const uint32_t* __restrict__ cost,
                                                       const uint32_t* __restrict__ hist,
                                                       unsigned long long* __restrict__ heavy,
                                                       uint32_t* __restrict__ sc) {
    __shared__ uint32_t ws[4];
    __shared__ uint32_t s_cls;
    // the costs are loaded first, so that their loads overlap the threshold's
    constexpr int kU = 8;  // loads in flight per thread
    const uint32_t j0 = blockIdx.x * (256u * kU) + threadIdx.x;
    uint32_t cv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        const uint32_t j = j0 + 256u * u;
        cv[u] = j < T ? cost[j] : 0u;
    }
    const uint32_t cls = heavy_class(hist, ws, &s_cls);
#pragma unroll
    for (int u = 0; u < kU; ++u) {
        if (cv[u] != 0u && cost_class(cv[u]) >= cls) {
            const uint32_t pos = atomicAdd(&sc[kScHeavyFound], 1u);  // < kTopTiles by the choice of cls
            heavy[pos] = ((unsigned long long)(~cv[u]) << 32) | (j0 + 256u * u);
        }
    }
}

// The heaviest-first queue (one workgroup of 1024 threads):
//  1. the heavy tiles (k_collect_heavy) are sorted by cost, descending
//     (ties by tile), and flagged in the spatial queue's bitmask;
//  2. a taken tile whose cost exceeds max(kSplitFloor, its instance's total
//     cost / its split share) is cut into up to kMaxParts equal candidate
//     ranges, while partial slots last (costliest first); inst_split counts
//     the tiles of each instance that are cut.
__global__ __launch_bounds__(1024) void k_plan_items(const InstDev* __restrict__ descs, int32_t count,
                                                     const unsigned long long* __restrict__ heavy,
                                                     const unsigned long long* __restrict__ inst_cost,
                                                     uint32_t* __restrict__ inst_split,
                                                     WorkItem* __restrict__ items,
                                                     uint32_t* __restrict__ top,
                                                     uint32_t* __restrict__ bits,
                                                     uint32_t* __restrict__ sc,
                                                     uint32_t* __restrict__ ctr, uint32_t nslots) {
    __shared__ unsigned long long keys[kTopTiles];
    __shared__ uint32_t ws[16];
    const int tid = threadIdx.x;
    const uint32_t nh = sc[kScHeavyFound];  // <= kTopTiles
    // bitonic sort of the heavy keys, ascending: cost descending, then tile.
    // One key per thread; exchanges with partners in the same wave go through
    // lane shuffles, the others through LDS.
    unsigned long long key = (uint32_t)tid < nh ? heavy[tid] : ~0ull;
    if (nh > 1) {
        for (int k = 2; k <= kTopTiles; k <<= 1) {
            for (int jj = k >> 1; jj > 0; jj >>= 1) {
                unsigned long long other;
                if (jj >= 64) {
                    __syncthreads();  // every thread has read the previous exchange
                    keys[tid] = key;
                    __syncthreads();
                    other = keys[tid ^ jj];
                } else {
                    const uint32_t lo = __shfl_xor((uint32_t)key, jj, 64);
                    const uint32_t hi = __shfl_xor((uint32_t)(key >> 32), jj, 64);
                    other = ((unsigned long long)hi << 32) | lo;
                }
                // the lower index of a pair keeps the smaller key in an
                // ascending run, the larger one in a descending run
                const bool up = (tid & k) == 0;
                const bool lower = (tid & jj) == 0;
                const bool keep_small = (up == lower);
                key = keep_small ? (key < other ? key : other) : (key < other ? other : key);
            }
        }
    }
    __syncthreads();
    keys[tid] = key;
    __syncthreads();

    // ---- 2. splitting
    uint32_t tile = 0, c = 0, parts = 1;
    int32_t inst = 0;
    if ((uint32_t)tid < nh) {
        const unsigned long long k = keys[tid];
        tile = (uint32_t)k;
        c = ~(uint32_t)(k >> 32);
        inst = find_inst(descs, count, tile);
        const unsigned long long ss = descs[inst].split_share;
        const unsigned long long share = (inst_cost[inst] + ss - 1) / ss;
        const uint32_t thr = share > kSplitFloor ? (share > 0xffffffffull ? 0xffffffffu : (uint32_t)share)
                                                 : kSplitFloor;
        if (c > thr) {
            const uint32_t want = (uint32_t)(((unsigned long long)c + thr - 1) / thr);
            parts = want < (uint32_t)kMaxParts ? want : (uint32_t)kMaxParts;
        }
        const uint32_t pos = spatial_pos(descs[inst], tile);
        atomicOr(&bits[pos >> 5], 1u << (pos & 31u));
    }
    uint32_t need = parts > 1 ? parts : 0u;
    uint32_t tot_need;
    const uint32_t pre_need = block_scan(need, ws, &tot_need);
    if (pre_need + need > nslots) {
        parts = 1;
        need = 0;
    }
    uint32_t nslot_used, nitems_h, nsplit;
    const uint32_t slot0 = block_scan(need, ws, &nslot_used);
    const uint32_t ipos = block_scan((uint32_t)tid < nh ? parts : 0u, ws, &nitems_h);
    const uint32_t spos = block_scan(parts > 1 ? 1u : 0u, ws, &nsplit);
    if ((uint32_t)tid < nh) {
        for (uint32_t p = 0; p < parts; ++p) {
            const uint32_t b = (uint32_t)(((unsigned long long)c * p) / parts);
            const uint32_t e = p + 1 == parts ? kAll : (uint32_t)(((unsigned long long)c * (p + 1)) / parts);
            items[ipos + p] = WorkItem{tile, b, e, parts > 1 ? slot0 + p : kNoSlot};
        }
        if (parts > 1) {
            atomicAdd(&inst_split[inst], 1u);
            top[4 * spos + 0] = tile;
            top[4 * spos + 1] = parts;
            top[4 * spos + 2] = slot0;
            top[4 * spos + 3] = c;
        }
    }
    for (int k = tid; k < kCtrWords; k += 1024) ctr[k] = 0u;  // both queues' counters
    if (tid == 0) {
        sc[kScHeavyItems] = nitems_h;
        sc[kScSplit] = nsplit;
        sc[kScHeavyTiles] = nh;
    }
}

// First level of each instance's FP64 grid sum: chunk blockIdx.x of the
// tile partials of instance blockIdx.y, strided per-thread sums, then a tree.
__global__ __launch_bounds__(256) void k_mass_chunks(const InstDev* __restrict__ descs,
                                                     double* __restrict__ mid) {
    __shared__ double sh[256];
    const int inst = blockIdx.y, ch = blockIdx.x, tid = threadIdx.x;
    const InstDev& D = descs[inst];
    double s = 0.0;
    if (D.flags & kInstMass) {
        const int64_t cnt = (int64_t)D.ntiles * kWaves;
        const int64_t chunk = (cnt + kMassChunks - 1) / kMassChunks;
        const int64_t beg = (int64_t)ch * chunk;
        const int64_t end = beg + chunk < cnt ? beg + chunk : cnt;
        for (int64_t i = beg + tid; i < end; i += 256) s += D.tile_part[i];
    }
    sh[tid] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (tid < w) sh[tid] += sh[tid + w];
        __syncthreads();
    }
    if (tid == 0) mid[(size_t)inst * kMassChunks + ch] = sh[0];
}

// Per instance: stats[0] = grid mass (sum * sres^2 tres, or 0 without the
// mass flag), [1], [2], [7] = 0, [3], [4], [5] = the set's non-finite,
// culled and invalid-bandwidth counts, [6] = tiles computed in parts.
__global__ __launch_bounds__(64) void k_finalize(const InstDev* __restrict__ descs,
                                                 const double* __restrict__ mid,
                                                 const uint32_t* __restrict__ inst_split) {
    static_assert(kMassChunks == 64, "one wave per instance");
    const InstDev& D = descs[blockIdx.x];
    double* st = D.stats;
    if (!st) return;
    const int lane = threadIdx.x;
    double v = mid[(size_t)blockIdx.x * kMassChunks + lane];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    if (lane == 0) {
        st[0] = (D.flags & kInstMass) ? v * D.mass_scale : 0.0;
        st[1] = 0.0;
        st[2] = 0.0;
        // the set's points that are never visited, from the offsets of their keys
        const uint32_t* cs = D.cell_start + (size_t)D.ncx * D.ncy * D.nct;
        st[3] = (double)(cs[kKeyNonFinite + 1] - cs[kKeyNonFinite]);
        st[4] = (double)(cs[kKeyCulled + 1] - cs[kKeyCulled]);
        st[5] = (double)(cs[kKeyBadBw + 1] - cs[kKeyBadBw]);
        st[6] = (double)inst_split[blockIdx.x];
        st[7] = 0.0;
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
    l.cost = o; o = al256(o + (size_t)T * 4);
    l.hist = o; o = al256(o + (size_t)kCostClasses * 4);
    l.bits = o; o = al256(o + ((size_t)T + 31) / 32 * 4);
    l.scalars = o; o = al256(o + (size_t)kScCount * 4);
    l.counters = o; o = al256(o + (size_t)kCtrWords * 4);
    l.heavy = o; o = al256(o + (size_t)kTopTiles * 8);
    l.top = o; o = al256(o + (size_t)kTopTiles * 16);
    l.items = o; o = al256(o + (size_t)kTopTiles * kMaxParts * sizeof(WorkItem));
    l.partials = o; o = al256(o + (size_t)kPartSlots * kTileXY * kTileXY * tile_t * 4);
    l.kscratch = o;
    // per thread: (sum, compensation) of 4 column groups x tile_t/16 row blocks, f32x4 each
    if (kahan) o = al256(o + (size_t)kMemKahanGroups * kThreads * 2 * (4 * (tile_t / 16)) * 16);
    l.tile_part = o; o = al256(o + (size_t)parts * 8);
    l.mass_mid = o; o = al256(o + (size_t)count * kMassChunks * 8);
    l.total = o;
    return l;
}

hipError_t launch_pass(InstDev* descs, int32_t count, uint8_t* pass, const PassLayout& pl,
                       int tile_t, int mode, bool full, bool adapt, int kf, bool h16, hipStream_t s,
                       hipEvent_t ev_before, hipEvent_t ev_after) {
    const bool kahan = mode != kAccPlain;
    InstDev* d_desc = reinterpret_cast<InstDev*>(pass + pl.desc);
    auto* inst_cost = reinterpret_cast<unsigned long long*>(pass + pl.inst_cost);
    auto* inst_split = reinterpret_cast<uint32_t*>(pass + pl.inst_split);
    auto* cost = reinterpret_cast<uint32_t*>(pass + pl.cost);
    auto* hist = reinterpret_cast<uint32_t*>(pass + pl.hist);
    auto* bits = reinterpret_cast<uint32_t*>(pass + pl.bits);
    auto* sc = reinterpret_cast<uint32_t*>(pass + pl.scalars);
    auto* ctr = reinterpret_cast<uint32_t*>(pass + pl.counters);
    auto* top = reinterpret_cast<uint32_t*>(pass + pl.top);
    auto* items = reinterpret_cast<WorkItem*>(pass + pl.items);
    auto* partials = reinterpret_cast<float*>(pass + pl.partials);
    auto* kscratch = reinterpret_cast<float*>(pass + pl.kscratch);
    auto* tile_part = reinterpret_cast<double*>(pass + pl.tile_part);
    auto* mid = reinterpret_cast<double*>(pass + pl.mass_mid);

    int64_t tb = 0;
    for (int32_t i = 0; i < count; ++i) {
        descs[i].tile_base = (int32_t)tb;
        descs[i].tile_part = tile_part + tb * kWaves;
        tb += descs[i].ntiles;
    }
    for (int32_t first = 0; first < count; first += kDescChunk) {
        DescChunk c{};
        const int32_t m = count - first < kDescChunk ? count - first : kDescChunk;
        for (int32_t k = 0; k < m; ++k) c.d[k] = descs[first + k];
        hipLaunchKernelGGL(k_put_desc, dim3(1), dim3(256), 0, s, c, first, m, d_desc, inst_cost,
                           inst_split, hist, sc, first == 0 ? 1 : 0);
    }
    const uint32_t T = (uint32_t)pl.T;
    hipLaunchKernelGGL(k_tile_cost, dim3((T + 255) / 256), dim3(256), 0, s, (const InstDev*)d_desc,
                       count, T, tile_t, cost, hist, inst_cost, bits);
    auto* heavy = reinterpret_cast<unsigned long long*>(pass + pl.heavy);
    hipLaunchKernelGGL(k_collect_heavy, dim3((T + 2047) / 2048), dim3(256), 0, s, T, (const uint32_t*)cost,
                       (const uint32_t*)hist, heavy, sc);
    hipLaunchKernelGGL(k_plan_items, dim3(1), dim3(1024), 0, s, (const InstDev*)d_desc, count,
                       (const unsigned long long*)heavy, (const unsigned long long*)inst_cost, inst_split,
                       items, top,
                       bits, sc, ctr, (uint32_t)kPartSlots);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (ev_before && (e = hipEventRecord(ev_before, s)) != hipSuccess) return e;
    e = launch_gather_items(d_desc, count, items, bits, sc, ctr, partials, kscratch, pl.T, tile_t, mode,
                            full, adapt, kf, h16, s);
    if (e != hipSuccess) return e;
    if (ev_after && (e = hipEventRecord(ev_after, s)) != hipSuccess) return e;
    e = launch_reduce_split(d_desc, count, top, sc, partials, tile_t, kahan, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mass_chunks, dim3(kMassChunks, (uint32_t)count), dim3(256), 0, s,
                       (const InstDev*)d_desc, mid);
    hipLaunchKernelGGL(k_finalize, dim3((uint32_t)count), dim3(64), 0, s, (const InstDev*)d_desc,
                       (const double*)mid, (const uint32_t*)inst_split);
    return hipGetLastError();
}

}  // namespace stkde
