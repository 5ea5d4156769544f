// bin.hip -- binning of points into space-time bins on the device.
//
// Stages (all deterministic):
//   1. transform: FP64 point -> voxel coordinates, support footprint clipped
//      to the grid, bin key (bins narrow in x, bandwidth-sized in y and t).
//      Points whose footprint misses the grid, with an invalid bandwidth
//      pair or with a non-finite coordinate get keys ncell + 0, 1, 2, which
//      sort after every bin and are never visited.
//   2. stable LSD radix sort of (key, index) with 8- to 11-bit digits, 1-3
//      passes.
//      This is the device form of the per-subdomain point lists that the
//      paper's domain decompositions build on the host (Sec. 4.2, Sec. 5.1).
//   3. bin offsets, cell_start[c] = first sorted position with key >= c, and
//      (same kernel) per sorted point the 32-byte PointRec (voxel-space
//      coordinates as FP32 head + FP16 tail, and the clipped footprint box).
// The bin offsets and records form the *binned set*, which stays
// valid for any number of later density computations on the base grid or a
// window of it with bandwidths up to the set's; the sort buffers are scratch.
#include <utility>

#include "stkde_internal.h"

namespace stkde {
namespace {

struct Footprint {
    double xr, yr, tr;
    int32_t xlo, xhi, ylo, yhi, tlo, thi;
    int32_t fx, fy, ft;  // floor of the voxel coordinate, clamped to [-1, G]
    bool finite, inside;
};

__device__ inline int32_t clamp_i(int32_t v, int32_t lo, int32_t hi) {
    return v < lo ? lo : (v > hi ? hi : v);
}

__device__ inline int32_t floordiv(int32_t a, int32_t b) {
    int32_t q = a / b;
    return (a % b != 0 && (a < 0)) ? q - 1 : q;
}

// Voxel-space footprint of one point with voxel bandwidths hv, tv (the
// set's, or the point's own).  Column X is inside the disc when
// |X + 1/2 - xr| < hv; row T is inside the window when |T + 1/2 - tr| <= tv.
// The integer ranges below are those sets up to rows where the kernel value
// is zero to rounding, clipped to the grid.
__device__ inline Footprint footprint(const SetGeom& g, double x, double y, double t, double hv,
                                      double tv) {
    Footprint f;
    f.finite = isfinite(x) && isfinite(y) && isfinite(t);
    f.inside = false;
    f.xr = (x - g.x0) / g.sres;
    f.yr = (y - g.y0) / g.sres;
    f.tr = (t - g.t0) / g.tres;
    f.xlo = f.xhi = f.ylo = f.yhi = f.tlo = f.thi = 0;
    f.fx = f.fy = f.ft = 0;
    if (!f.finite) return f;
    // reject far-away points before any conversion to integers
    if (f.xr + hv < -1.0 || f.xr - hv > (double)g.gx + 1.0) return f;
    if (f.yr + hv < -1.0 || f.yr - hv > (double)g.gy + 1.0) return f;
    if (f.tr + tv < -1.0 || f.tr - tv > (double)g.gt + 1.0) return f;
    const double xlo = floor(f.xr - hv - 0.5) + 1.0, xhi = ceil(f.xr + hv - 0.5) - 1.0;
    const double ylo = floor(f.yr - hv - 0.5) + 1.0, yhi = ceil(f.yr + hv - 0.5) - 1.0;
    const double tlo = ceil(f.tr - tv - 0.5), thi = floor(f.tr + tv - 0.5);
    f.xlo = (int32_t)fmax(xlo, 0.0);
    f.xhi = (int32_t)fmin(xhi, (double)(g.gx - 1));
    f.ylo = (int32_t)fmax(ylo, 0.0);
    f.yhi = (int32_t)fmin(yhi, (double)(g.gy - 1));
    f.tlo = (int32_t)fmax(tlo, 0.0);
    f.thi = (int32_t)fmin(thi, (double)(g.gt - 1));
    f.inside = f.xlo <= f.xhi && f.ylo <= f.yhi && f.tlo <= f.thi;
    f.fx = (int32_t)fmin(fmax(floor(f.xr), -1.0), (double)g.gx);
    f.fy = (int32_t)fmin(fmax(floor(f.yr), -1.0), (double)g.gy);
    f.ft = (int32_t)fmin(fmax(floor(f.tr), -1.0), (double)g.gt);
    return f;
}

__device__ inline uint32_t bin_key(const SetGeom& g, const Footprint& f) {
    const int32_t cx = clamp_i(floordiv(f.fx, g.cx), 0, g.ncx - 1);
    const int32_t cy = clamp_i(floordiv(f.fy, g.cxy), 0, g.ncy - 1);
    const int32_t ct = clamp_i(floordiv(f.ft, g.ct), 0, g.nct - 1);
    return (uint32_t)((ct * g.ncy + cy) * g.ncx + cx);
}

// A point's voxel bandwidths: the set's, or its own pair (hs_i / sres,
// ht_i / tres) when it carries one; false for a pair that is not finite and
// positive or exceeds the set's (bins and tiles are sized by the set's).
__device__ inline bool point_bandwidths(const SetGeom& g, const double* __restrict__ hst, int64_t i,
                                        double* hv, double* tv) {
    if (!hst) {
        *hv = g.hv;
        *tv = g.tv;
        return true;
    }
    const double hs = hst[2 * (size_t)i], ht = hst[2 * (size_t)i + 1];
    *hv = hs / g.sres;
    *tv = ht / g.tres;
    return isfinite(hs) && isfinite(ht) && hs > 0.0 && ht > 0.0 && *hv <= g.hv && *tv <= g.tv;
}

// Key of point i (an index into the bins, or one of the sentinel keys past
// them), with its footprint and voxel bandwidths: those of the record when
// the key is below ncell.
__device__ inline uint32_t point_key(const SetGeom& g, const double* __restrict__ hst, int64_t i, double x,
                                     double y, double t, Footprint& f, double& hv, double& tv) {
    const bool bw_ok = point_bandwidths(g, hst, i, &hv, &tv);
    f = footprint(g, x, y, t, bw_ok ? hv : g.hv, bw_ok ? tv : g.tv);
    if (!f.finite) return (uint32_t)(g.ncell + kKeyNonFinite);
    if (!bw_ok) return (uint32_t)(g.ncell + kKeyBadBw);
    if (!f.inside) return (uint32_t)(g.ncell + kKeyCulled);
    return bin_key(g, f);
}

// FP16 bit pattern of the tail v - head (|tail| <= half an FP32 ulp of v).
__device__ inline uint32_t pack_tail(double v, float head) {
    const _Float16 h = (_Float16)(float)(v - (double)head);
    return (uint32_t)__builtin_bit_cast(uint16_t, h);
}

// The 32-byte record of a valid point (footprint f, voxel bandwidths hv, tv)
// at index `at` of recs; with per-point bandwidths (bw) its terms (1/hv_i^2,
// 1/tv_i^2, (hv^2 tv) / (hv_i^2 tv_i)): the weight carries the point's own
// normalisation relative to the set's, which the store applies; with x64 its
// FP64 voxel coordinates.
__device__ inline void store_record(const SetGeom& g, const Footprint& f, double hv, double tv, int64_t at,
                                    PointRec* __restrict__ recs, float4* __restrict__ bw,
                                    double* __restrict__ x64) {
    if (bw)
        bw[at] = make_float4((float)(1.0 / (hv * hv)), (float)(1.0 / (tv * tv)),
                             (float)((g.hv * g.hv * g.tv) / (hv * hv * tv)), 0.0f);
    if (x64) {
        x64[3 * at] = f.xr;
        x64[3 * at + 1] = f.yr;
        x64[3 * at + 2] = f.tr;
    }
    PointRec r;
    r.xh = (float)f.xr;
    r.yh = (float)f.yr;
    r.th = (float)f.tr;
    r.xb = (uint32_t)f.xlo | ((uint32_t)f.xhi << 16);
    r.yb = (uint32_t)f.ylo | ((uint32_t)f.yhi << 16);
    r.tb = (uint32_t)f.tlo | ((uint32_t)f.thi << 16);
    r.xl_yl = pack_tail(f.xr, r.xh) | (pack_tail(f.yr, r.yh) << 16);
    r.tl = pack_tail(f.tr, r.th);
    recs[at] = r;
}

// Bin offsets at sorted position s, called by every lane of a wave: the
// cells (lo, hi] start at s, where lo is the key before s (-1 at s = 0) and
// hi the key at s (ncell + kKeySentinels at s = n), so each cell is written
// once, by the position that starts it; runs of empty bins can be long, so
// runs of more than two cells are written by the whole wave, 64 cells a step.
__device__ inline void put_cell_starts(uint32_t* __restrict__ cell_start, uint32_t s, int32_t lo, int32_t hi,
                                       int lane) {
    const bool wide = hi - lo > 2;
    if (!wide) {
        for (int32_t c = lo + 1; c <= hi; ++c) cell_start[c] = s;
    }
    for (unsigned long long m = __ballot(wide); m != 0ull; m &= m - 1ull) {
        const int src = __builtin_ctzll(m);
        const int32_t wlo = __shfl(lo, src, 64), whi = __shfl(hi, src, 64);
        const uint32_t ws = (uint32_t)__shfl((int32_t)s, src, 64);
        for (int32_t c = wlo + 1 + lane; c <= whi; c += 64) cell_start[c] = ws;
    }
}

constexpr int kMaxDigitBits = 11;
constexpr int kMaxBuckets = 1 << kMaxDigitBits;

// A sort of one pass (keys of at most kMaxDigitBits bits, the digit being
// the whole key) places the records itself: the transform writes each valid
// point's record (and bandwidth terms, FP64 voxel coordinates) at its input
// index in scratch (prec, pbw, px64), the scatter moves them to their sorted
// positions in the set (recs, bw, x64), and the bin offsets are the
// exclusive scan of the digit totals, which the scatter's first block writes
// to cell_start.  No key or value array is written.
struct RecMove {
    PointRec* prec;
    float4* pbw;
    double* px64;
    PointRec* recs;
    float4* bw;
    double* x64;
    uint32_t* cell_start;
};

// Keys of one radix block's points (kThreads * ITEMS of them) and the block's
// histogram of the first digit (the low dbits bits), hist[d * nblk + block]:
// two points per thread (the histogram does not depend on which thread counts
// a point).
template <int ITEMS, bool MOVE>
__global__ __launch_bounds__(kThreads * ITEMS / 2) void k_transform(SetGeom g, const double* __restrict__ xyt,
                                                                    const double* __restrict__ hst, int32_t n,
                                                                    uint32_t* __restrict__ keys,
                                                                    uint32_t* __restrict__ vals, int nbuck,
                                                                    uint32_t* __restrict__ hist, int32_t nblk,
                                                                    RecMove mv) {
    constexpr int kTransformThreads = kThreads * ITEMS / 2;
    constexpr int kTransformItems = 2;
    __shared__ uint32_t cnt[kMaxBuckets];
    const int tid = threadIdx.x;
    const int32_t base = blockIdx.x * (kThreads * ITEMS);
    // every coordinate of this thread is loaded before the first footprint,
    // so that the loads are in flight together
    double px[kTransformItems], py[kTransformItems], pt[kTransformItems];
#pragma unroll
    for (int it = 0; it < kTransformItems; ++it) {
        const int32_t i = base + it * kTransformThreads + tid;
        const int32_t ic = i < n ? i : n - 1;
        px[it] = xyt[3 * (size_t)ic];
        py[it] = xyt[3 * (size_t)ic + 1];
        pt[it] = xyt[3 * (size_t)ic + 2];
    }
    for (int d = tid; d < nbuck; d += kTransformThreads) cnt[d] = 0;
    __syncthreads();
    const uint32_t mask = (uint32_t)nbuck - 1u;
#pragma unroll
    for (int it = 0; it < kTransformItems; ++it) {
        const int32_t i = base + it * kTransformThreads + tid;
        if (i < n) {
            double hv, tv;
            Footprint f;
            const uint32_t key = point_key(g, hst, i, px[it], py[it], pt[it], f, hv, tv);
            keys[i] = key;
            if constexpr (MOVE) {
                if (key < (uint32_t)g.ncell) store_record(g, f, hv, tv, i, mv.prec, mv.pbw, mv.px64);
            } else {
                vals[i] = (uint32_t)i;
            }
            atomicAdd(&cnt[key & mask], 1u);
        }
    }
    __syncthreads();
    for (int d = tid; d < nbuck; d += kTransformThreads) hist[(size_t)d * nblk + blockIdx.x] = cnt[d];
}

// ---- stable LSD radix sort, digits of 6 to 11 bits --------------------------
//
// A key of b bits is sorted in ceil(b / 11) passes of equal digits (18-bit
// keys: two 9-bit passes; 12- to 14-bit keys: two passes of 6 or 7 bits, fewer
// buckets than threads).  The first pass's histogram comes with the keys.

// Per-block digit histogram.  hist is digit-major: hist[d * nblk + b].
template <int ITEMS>
__global__ __launch_bounds__(kThreads) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                         int32_t n, int shift, int nbuck,
                                                         uint32_t* __restrict__ hist,
                                                         int32_t nblk) {
    __shared__ uint32_t cnt[kMaxBuckets];
    // every key of this thread is loaded before the first count, so that the
    // loads are in flight together
    const int32_t base = blockIdx.x * (kThreads * ITEMS);
    uint32_t kr[ITEMS];
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int32_t i = base + it * kThreads + threadIdx.x;
        kr[it] = i < n ? keys[i] : 0u;
    }
    for (int d = threadIdx.x; d < nbuck; d += kThreads) cnt[d] = 0;
    __syncthreads();
    const uint32_t mask = (uint32_t)nbuck - 1u;
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const int32_t i = base + it * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(kr[it] >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < nbuck; d += kThreads) hist[(size_t)d * nblk + blockIdx.x] = cnt[d];
}

// One workgroup per digit d: hist[d][b] <- keys with digit d in blocks before
// b (an exclusive scan of the row), totals[d] <- the row's sum.  The keys of
// smaller digits are added by the scatter.
__global__ __launch_bounds__(kThreads) void k_radix_rowscan(uint32_t* __restrict__ hist, int32_t nblk,
                                                            uint32_t* __restrict__ totals) {
    __shared__ uint32_t wsum[kWaves];
    __shared__ uint32_t carry_s;
    const int d = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) carry_s = 0u;
    uint32_t* row = hist + (size_t)d * nblk;
    for (int32_t base = 0; base < nblk; base += kThreads) {
        const int32_t i = base + tid;
        const uint32_t v = i < nblk ? row[i] : 0u;
        uint32_t inc = v;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(inc, o, 64);
            if (lane >= o) inc += u;
        }
        __syncthreads();  // carry_s and wsum of the previous round are consumed
        if (lane == 63) wsum[wv] = inc;
        __syncthreads();
        uint32_t pre = carry_s;
        for (int w = 0; w < wv; ++w) pre += wsum[w];
        if (i < nblk) row[i] = pre + inc - v;
        __syncthreads();
        if (tid == 0) carry_s += wsum[0] + wsum[1] + wsum[2] + wsum[3];
    }
    __syncthreads();
    if (tid == 0) totals[d] = carry_s;
}

// Stable scatter.  Keys of a block are processed in index order: round r
// covers indices base + r*256 + [0, 256), waves in order, lanes in order.
// The rank of a key among equal digits is (keys of that digit in earlier
// rounds) + (in earlier waves of this round) + (in earlier lanes).
// MOVE (a sort of one pass): values are the input indices, and instead of
// keys and values the records are written (RecMove).
template <int ITEMS, bool MOVE>
__global__ __launch_bounds__(kThreads) void k_radix_scatter(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, int32_t n, int shift,
    int dbits, const uint32_t* __restrict__ hist, const uint32_t* __restrict__ totals, int32_t nblk,
    uint32_t* __restrict__ kout, uint32_t* __restrict__ vout, uint32_t ncell, RecMove mv) {
    __shared__ uint32_t off[kMaxBuckets];
    __shared__ uint32_t wcnt[kWaves][kMaxBuckets];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nbuck = 1 << dbits;
    const uint32_t mask = (uint32_t)nbuck - 1u;
    // every key and value of this thread is loaded up front, so that the
    // loads are in flight together rather than one round at a time
    const int32_t base = blockIdx.x * (kThreads * ITEMS);
    uint32_t kr[ITEMS], vr[ITEMS];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int32_t i = base + r * kThreads + tid;
        kr[r] = i < n ? kin[i] : 0u;
        vr[r] = MOVE ? (uint32_t)i : (i < n ? vin[i] : 0u);
    }
    // off[d] = keys of the smaller digits (an exclusive scan of the digit
    // totals; thread tid holds digits per * tid + [0, per) below nbuck, per
    // >= 1 also for digits of fewer than 8 bits) + this block's offset within
    // digit d
    {
        const int per = (nbuck + kThreads - 1) / kThreads;
        uint32_t tv[kMaxBuckets / kThreads], ts = 0;
#pragma unroll
        for (int k = 0; k < kMaxBuckets / kThreads; ++k) {
            const int d = per * tid + k;
            tv[k] = (k < per && d < nbuck) ? totals[d] : 0u;
            ts += tv[k];
        }
        uint32_t inc = ts;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t u = __shfl_up(inc, o, 64);
            if (lane >= o) inc += u;
        }
        if (lane == 63) wcnt[0][wv] = inc;
        __syncthreads();
        uint32_t run = inc - ts;
        for (int w = 0; w < wv; ++w) run += wcnt[0][w];
#pragma unroll
        for (int k = 0; k < kMaxBuckets / kThreads; ++k) {
            const int d = per * tid + k;
            if (k < per && d < nbuck) {
                off[d] = run + hist[(size_t)d * nblk + blockIdx.x];
                // bin offsets: cell_start[c] = keys below c, c <= ncell + kKeySentinels
                if (MOVE && blockIdx.x == 0 && d <= (int)ncell + kKeySentinels) mv.cell_start[d] = run;
                run += tv[k];
            }
        }
        if (MOVE && blockIdx.x == 0 && tid == 0 && (int)ncell + kKeySentinels == nbuck) mv.cell_start[nbuck] = (uint32_t)n;
        __syncthreads();  // wcnt[0] is cleared next
    }
    for (int d = tid; d < nbuck; d += kThreads) {
#pragma unroll
        for (int w = 0; w < kWaves; ++w) wcnt[w][d] = 0;
    }
    __syncthreads();
    const unsigned long long lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const int32_t i = base + r * kThreads + tid;
        const bool valid = i < n;
        const uint32_t key = kr[r], val = vr[r];
        const uint32_t d = valid ? (key >> shift) & mask : 0u;
        // the record moves with a valid point's key; loaded before the rank
        // is known, so that the load overlaps the ranking
        const bool mrec = MOVE && valid && key < ncell;
        uint4 ra = make_uint4(0u, 0u, 0u, 0u), rb = ra;
        if (mrec) {
            const uint4* src = reinterpret_cast<const uint4*>(mv.prec + val);
            ra = src[0];
            rb = src[1];
        }
        unsigned long long peers = __ballot(valid);
        for (int b = 0; b < dbits; ++b) {
            const unsigned long long bb = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(peers & lt_mask);
        const bool lead = valid && rank == 0;  // one lane per (wave, digit) present
        const uint32_t cnt = (uint32_t)__popcll(peers);
        if (lead) wcnt[wv][d] = cnt;
        __syncthreads();
        if (valid) {
            uint32_t pos = off[d] + rank;
            for (int w = 0; w < wv; ++w) pos += wcnt[w][d];
            if constexpr (MOVE) {
                if (mrec) {
                    uint4* dst = reinterpret_cast<uint4*>(mv.recs + pos);
                    dst[0] = ra;
                    dst[1] = rb;
                    if (mv.bw) mv.bw[pos] = mv.pbw[val];
                    if (mv.x64) {
                        mv.x64[3 * (size_t)pos] = mv.px64[3 * (size_t)val];
                        mv.x64[3 * (size_t)pos + 1] = mv.px64[3 * (size_t)val + 1];
                        mv.x64[3 * (size_t)pos + 2] = mv.px64[3 * (size_t)val + 2];
                    }
                }
            } else {
                kout[pos] = key;
                vout[pos] = val;
            }
        }
        __syncthreads();  // off and wcnt of this round are read
        // only the digits present move: each leader adds its wave's count and
        // clears its own entry (the next round's entries of other waves are
        // other rows; its own wave's come after this in program order, and
        // they are read only after the next round's first barrier)
        if (lead) {
            atomicAdd(&off[d], cnt);
            wcnt[wv][d] = 0;
        }
    }
}

// Per sorted position s in [0, n]:
//  - bin offsets: cell_start[c] = lower_bound(sorted keys, c) for c in
//    [0, ncell + kKeySentinels]; s is the lower bound of the cells in
//    (key[s - 1], key[s]] (key[-1] = -1, key[n] = ncell + kKeySentinels),
//    so each cell is written once, by the position that starts it (the
//    offsets past ncell count the points that are never visited);
//  - for a valid point (key below ncell): its record (store_record).
// vals is a permutation of [0, n), so the point's coordinates are loaded
// before its validity is known and the loads are in flight together.
__global__ __launch_bounds__(kThreads) void k_offsets_records(
    SetGeom g, const double* __restrict__ xyt, const double* __restrict__ hst,
    const uint32_t* __restrict__ keys, const uint32_t* __restrict__ vals, int32_t n,
    uint32_t* __restrict__ cell_start,
    PointRec* __restrict__ recs, float4* __restrict__ bw, double* __restrict__ x64) {
    const int64_t s = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool act = s <= n;  // every lane stays for the wave's shared cell writes
    // clamped positions, so that every load is unconditional (n > 0)
    const int64_t sp = s > 0 ? (s <= n ? s - 1 : (int64_t)n - 1) : 0, sc = s < n ? s : (int64_t)n - 1;
    uint32_t kp = 0, kc = 0, i = 0;
    double x = 0.0, y = 0.0, t = 0.0;
    if (n > 0) {
        kp = keys[sp];
        kc = keys[sc];
        i = vals[sc];
        x = xyt[3 * (size_t)i];
        y = xyt[3 * (size_t)i + 1];
        t = xyt[3 * (size_t)i + 2];
    }
    const int32_t lo = !act ? 0 : (s == 0 ? -1 : (int32_t)kp);
    const int32_t hi = !act ? 0 : (s == n ? g.ncell + kKeySentinels : (int32_t)kc);
    put_cell_starts(cell_start, (uint32_t)s, lo, hi, lane);
    if (!act || s == n || kc >= (uint32_t)g.ncell) return;
    double hv, tv;
    (void)point_bandwidths(g, hst, i, &hv, &tv);  // valid: invalid pairs sort past the bins
    const Footprint f = footprint(g, x, y, t, hv, tv);
    store_record(g, f, hv, tv, s, recs, bw, x64);
}

inline int bits_for(uint32_t v) {
    int b = 0;
    while (b < 32 && (v >> b) != 0u) ++b;
    return b;
}

}  // namespace

namespace {
size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }
}  // namespace

SetLayout layout_set(const SetGeom& g, int64_t n, bool adaptive, bool exact) {
    SetLayout l{};
    size_t o = 0;
    l.cell_start = o; o = al256(o + ((size_t)g.ncell + kKeySentinels + 1) * 4);
    l.recs = o; o = al256(o + (size_t)n * sizeof(PointRec));
    l.bw = o; o = al256(o + (adaptive ? (size_t)n * sizeof(float4) : 0));
    l.x64 = o; o = al256(o + (exact ? (size_t)n * 3 * sizeof(double) : 0));
    l.total = o;
    return l;
}

namespace {
// Passes and digit bits of the binning sort: keys are at most ncell + 2
// (non-finite points), sorted in ceil(bits / 11) passes of equal digits
// (one pass of 8 bits for keys of up to 8).
struct SortPlan {
    int passes, dbits;
};
SortPlan sort_plan(const SetGeom& g) {
    const int bits = bits_for((uint32_t)(g.ncell + kKeySentinels - 1));
    const int passes = bits <= 8 ? 1 : (bits + kMaxDigitBits - 1) / kMaxDigitBits;
    return SortPlan{passes, bits <= 8 ? 8 : (bits + passes - 1) / passes};
}
}  // namespace

SortLayout layout_sort(const SetGeom& g, int64_t n, bool adaptive, bool exact) {
    SortLayout l{};
    size_t o = 0;
    const size_t nn = (size_t)n;
    l.items = sort_items(n);
    const int64_t tile = (int64_t)kThreads * l.items;
    l.nblk = (int32_t)((n + tile - 1) / tile);
    l.one_pass = sort_plan(g).passes == 1;
    l.adaptive = adaptive;
    l.exact = exact;
    l.keys0 = o; o = al256(o + nn * 4);
    if (l.one_pass) {
        l.prec = o; o = al256(o + nn * sizeof(PointRec));
        l.pbw = o; o = al256(o + (adaptive ? nn * sizeof(float4) : 0));
        l.px64 = o; o = al256(o + (exact ? nn * 3 * sizeof(double) : 0));
    } else {
        l.vals0 = o; o = al256(o + nn * 4);
        l.keys1 = o; o = al256(o + nn * 4);
        l.vals1 = o; o = al256(o + nn * 4);
    }
    l.hist = o; o = al256(o + (size_t)kMaxBuckets * l.nblk * 4);
    l.totals = o; o = al256(o + 3 * (size_t)kMaxBuckets * 4);
    l.total = o;
    return l;
}

hipError_t launch_bin(const SetGeom& g, const double* d_xyt, int32_t n, uint8_t* set,
                      const SetLayout& sl, uint8_t* sort, const SortLayout& so, hipStream_t s,
                      const double* d_hst, bool exact) {
    uint32_t* k0 = reinterpret_cast<uint32_t*>(sort + so.keys0);
    uint32_t* v0 = reinterpret_cast<uint32_t*>(sort + so.vals0);
    uint32_t* k1 = reinterpret_cast<uint32_t*>(sort + so.keys1);
    uint32_t* v1 = reinterpret_cast<uint32_t*>(sort + so.vals1);
    uint32_t* hist = reinterpret_cast<uint32_t*>(sort + so.hist);
    uint32_t* totals = reinterpret_cast<uint32_t*>(sort + so.totals);
    uint32_t* cs = reinterpret_cast<uint32_t*>(set + sl.cell_start);

    const SortPlan sp = sort_plan(g);
    // a layout made for another geometry, or without room for the payload
    if (sp.passes == 1 && (!so.one_pass || (d_hst && !so.adaptive) || (exact && !so.exact)))
        return hipErrorInvalidValue;
    const int nbuck = 1 << sp.dbits;
    PointRec* recs = reinterpret_cast<PointRec*>(set + sl.recs);
    float4* bw = d_hst ? reinterpret_cast<float4*>(set + sl.bw) : nullptr;
    double* x64 = exact ? reinterpret_cast<double*>(set + sl.x64) : nullptr;
    RecMove mv{};
    if (sp.passes == 1)
        mv = RecMove{reinterpret_cast<PointRec*>(sort + so.prec), d_hst ? reinterpret_cast<float4*>(sort + so.pbw) : nullptr,
                     exact ? reinterpret_cast<double*>(sort + so.px64) : nullptr, recs, bw, x64, cs};
    auto run_sort = [&]<int ITEMS, bool MOVE>() {
        hipLaunchKernelGGL((k_transform<ITEMS, MOVE>), dim3(so.nblk), dim3(kThreads * ITEMS / 2), 0, s, g, d_xyt,
                           d_hst, n, k0, v0, nbuck, hist, so.nblk, mv);
        for (int p = 0; p < sp.passes; ++p) {
            if (p > 0)
                hipLaunchKernelGGL((k_radix_hist<ITEMS>), dim3(so.nblk), dim3(kThreads), 0, s, k0, n, sp.dbits * p,
                                   nbuck, hist, so.nblk);
            uint32_t* tot = totals + kMaxBuckets * p;
            hipLaunchKernelGGL(k_radix_rowscan, dim3(nbuck), dim3(kThreads), 0, s, hist, so.nblk, tot);
            hipLaunchKernelGGL((k_radix_scatter<ITEMS, MOVE>), dim3(so.nblk), dim3(kThreads), 0, s, k0, v0, n,
                               sp.dbits * p, sp.dbits, hist, tot, so.nblk, k1, v1, (uint32_t)g.ncell, mv);
            std::swap(k0, k1);
            std::swap(v0, v1);
        }
    };
    if (sp.passes == 1) {
        // the scatter places the records and writes the bin offsets
        if (so.items == kSortItemsSmall) run_sort.template operator()<kSortItemsSmall, true>();
        else run_sort.template operator()<kSortItems, true>();
        return hipGetLastError();
    }
    if (so.items == kSortItemsSmall) run_sort.template operator()<kSortItemsSmall, false>();
    else run_sort.template operator()<kSortItems, false>();
    hipLaunchKernelGGL(k_offsets_records, dim3((uint32_t)(((int64_t)n + kThreads) / kThreads)), dim3(kThreads), 0,
                       s, g, d_xyt, d_hst, k0, v0, n, cs, recs, bw, x64);
    return hipGetLastError();
}

}  // namespace stkde
