// stkde_internal.h -- layouts and launch interfaces shared by the library's
// HIP sources (binning, gather, statistics) and its host entry points.
//
// Units: every quantity below is in voxel units unless named otherwise.  A
// point's voxel-space coordinate is xr = (x - x0)/sres (likewise y, and t with
// tres); the voxel bandwidths are hv = hs/sres and tv = ht/tres, and the
// integer loop bounds Hs = ceil(hv), Ht = ceil(tv) of Sec. 2.1.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace stkde {

// A 256-thread workgroup owns a 16 x 16 x TT tile of voxels; each of its four
// waves owns an 8 x 8 quadrant of columns, i.e. four 4 x 4 column groups,
// times TT/16 blocks of 16 rows, as FP32 matrix-core accumulators.
constexpr int kPatch = 8;
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
    uint32_t xb;       // footprint columns in x: lo | hi << 16, clipped to the grid
    uint32_t yb;       // footprint columns in y: lo | hi << 16
    uint32_t tb;       // footprint rows in t: lo | hi << 16
    uint32_t xl_yl;    // tails of x and y as two FP16 (x in the low half)
    uint32_t tl;       // tail of t as FP16 in the low half
};
static_assert(sizeof(PointRec) == 32, "record layout");

// Geometry of one plan, in the form the kernels consume.
struct Geometry {
    int32_t gx, gy, gt;
    int32_t Hs, Ht;           // ceil(hv), ceil(tv)
    int32_t cxy, ct;          // bin edge in x/y and in t (voxels)
    int32_t ncx, ncy, nct;    // bins per axis
    int32_t ncell;            // ncx * ncy * nct
    int32_t key_bits;         // bits of the largest key (ncell, used for culled points)
    int32_t tile_t;           // time rows per lane (16 or 32)
    int32_t ntx, nty, ntt;    // tiles per axis
    int32_t ntiles;
    int32_t max_ranges;       // most (t, y) bin rows one tile reads
    double x0, y0, t0;
    double inv_sres, inv_tres;  // used as multipliers only where exact (see binning)
    double sres, tres;
    double hv, tv;            // voxel bandwidths
    double Hs_d, Ht_d;        // ceil(hv), ceil(tv) uncapped (loop bounds of the statistics)
    double hs, ht;            // domain bandwidths
    float inv_hv2;            // 1/hv^2 (FP32)
    float inv_tv2;            // 1/tv^2 (FP32)
};

// Workspace carve-up (byte offsets from d_ws, each 256-byte aligned).
struct Workspace {
    size_t keys0, vals0, keys1, vals1;
    size_t hist;         // radix digit counts, 256 * nblk_sort u32
    size_t cell_start;   // (ncell + 1) u32
    size_t recs;         // n PointRec
    size_t tile_part;    // ntiles * kWaves double (grid mass partials)
    size_t pt_part;      // nblk_pts * 4 double (per-point statistics partials)
    size_t counters;     // 4 x u64 (non-finite, culled), then 3 x 256 u32 digit totals
    size_t mass_part;    // kMassBlocks double (first level of the grid-mass sum)
    size_t total;
    int32_t nblk_sort;
    int32_t nblk_pts;
};

constexpr int kSortItems = 8;                         // keys per thread per block
constexpr int kSortTile = kThreads * kSortItems;      // keys per block
constexpr int kStatBlock = 256;                       // points per statistics block
constexpr int kMassBlocks = 256;                      // workgroups of the grid-mass sum

Workspace layout_workspace(const Geometry& g, int64_t n);

// Stage launchers (all asynchronous on `s`; return the launch error).
hipError_t launch_bin(const Geometry& g, const double* d_xyt, int32_t n, uint8_t* ws,
                      const Workspace& w, hipStream_t s);
hipError_t launch_gather(const Geometry& g, float cnorm, bool kahan, bool mass, float* d_out,
                         uint8_t* ws, const Workspace& w, hipStream_t s);
hipError_t launch_mass_reduce(const Geometry& g, double* d_dst, uint8_t* ws, const Workspace& w,
                              hipStream_t s);
// d_stats[0..7] = 0 except the binning counters in [3], [4]
hipError_t launch_stats(const Geometry& g, const double* d_xyt, int32_t n, bool point_stats,
                        double* d_stats, uint8_t* ws, const Workspace& w, hipStream_t s);
// d_stats[1], [2] from per-point FP64 sums
hipError_t launch_point_stats(const Geometry& g, const double* d_xyt, int32_t n, double* d_stats,
                              uint8_t* ws, const Workspace& w, hipStream_t s);

}  // namespace stkde
