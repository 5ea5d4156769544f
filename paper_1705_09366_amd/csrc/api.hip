// api.hip -- host side of the C ABI declared in include/stkde.h: argument
// validation, plan and set geometry, workspace layouts and the launch
// sequences
//   compute = bin (transform, radix sort, bin offsets, records) into the
//             workspace's set region -> one pass (work list, gather, split
//             reduction, mass) -> optional point statistics;
//   batch   = one pass per (tile_t, Kahan) group over the items' sets, or one
//             pass with one multi-variant gather when they allow it.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <new>
#include <vector>

#include "../../include/stkde.h"
#include "../../include/stkde_ablation.h"
#include "stkde_internal.h"

struct stkde_plan_s {
    stkde_desc desc;
    uint32_t split_share;
    int32_t kahan_mode;  // 0 automatic, else kAccKahanReg / kAccKahanMem
    int32_t operand_form;  // 0 two-term FP16 where the gather has it, 1 FP32
    stkde::InstGeom ig;  // the plan's grid as an instance of its own set
    stkde::SetGeom sg;   // binning of the plan's own points
    // gather timing (stkde_plan_profile): event pairs, filled in order
    std::vector<hipEvent_t> ev;
    int32_t ev_used = 0;
    // one stkde_compute recorded as a HIP graph (stkde_plan_capture)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool capturing = false;  // no profiling events while recording
};

namespace {
void release_events(stkde_plan_s* p) {
    for (hipEvent_t e : p->ev)
        if (e) (void)hipEventDestroy(e);
    p->ev.clear();
    p->ev_used = 0;
}
void release_graph(stkde_plan_s* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}
}  // namespace

struct stkde_set_s {
    stkde_desc base;
    stkde::SetGeom sg;
    int64_t n;
    stkde::SetLayout sl;
    stkde::SortLayout so;
};

struct stkde_batch_s {
    struct Group {
        int tile_t;
        bool kahan;
        int mode;  // accumulation mode of the gather (kAcc*)
        bool full; // full-cover path
        bool h16;  // two-term FP16 operands
        bool multi = false;  // grids of several gather variants in one launch
        std::vector<int32_t> idx;
        std::vector<stkde::InstGeom> geo;
        std::vector<int32_t> variant;  // multi: each grid's gather variant
        stkde::PassLayout pl;
    };
    std::vector<stkde_item> items;
    std::vector<Group> groups;
    size_t ws_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

constexpr int64_t kMaxDim = 65535;
constexpr int32_t kXBin = 8;           // x bin edge in voxels (see make_set_geom)
constexpr int32_t kMaxCells = 1 << 22;  // keys of at most 23 bits: <= 3 radix passes (<= 2 below 2^22 - 2 bins)
constexpr int32_t kMaxBatch = 4096;
constexpr double kSparseCandidates = 384.0;  // half the gather's survivor buffer
constexpr uint32_t kKnownFlags = STKDE_FLAG_KAHAN | STKDE_FLAG_MASS | STKDE_FLAG_POINT_STATS |
                                  STKDE_FLAG_ADAPTIVE | STKDE_FLAG_CORNER | STKDE_KERNEL_MASK;

int kernel_of(const stkde_desc& d) { return (int)((d.flags & STKDE_KERNEL_MASK) >> STKDE_KERNEL_SHIFT); }

// Sampling at lower corners is sampling at centres of the grid whose origin
// sits half a voxel lower: every stage works on that grid.
double origin_shift(const stkde_desc& d, double res) { return (d.flags & STKDE_FLAG_CORNER) ? 0.5 * res : 0.0; }

// Pairs that are not zero on their support boundary test membership near it
// in FP64, from coordinates the binned set then keeps.
bool exact_support(const stkde_desc& d) {
    return kernel_of(d) == STKDE_KERNEL_GAUSSIAN || kernel_of(d) == STKDE_KERNEL_PRINTED;
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

int32_t ceil_div(int64_t a, int64_t b) { return (int32_t)((a + b - 1) / b); }

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

stkde_status check_desc(const stkde_desc* d) {
    if (d->gx < 1 || d->gy < 1 || d->gt < 1) return STKDE_ERR_INVALID_ARG;
    if (d->gx > kMaxDim || d->gy > kMaxDim || d->gt > kMaxDim) return STKDE_ERR_TOO_LARGE;
    if (!finite_pos(d->sres) || !finite_pos(d->tres) || !finite_pos(d->hs) || !finite_pos(d->ht))
        return STKDE_ERR_INVALID_ARG;
    if (!isfinite(d->x0) || !isfinite(d->y0) || !isfinite(d->t0)) return STKDE_ERR_INVALID_ARG;
    if (d->flags & ~kKnownFlags) return STKDE_ERR_INVALID_ARG;
    if (kernel_of(*d) > STKDE_KERNEL_PRINTED) return STKDE_ERR_INVALID_ARG;
    const uint64_t nvox = (uint64_t)d->gx * (uint64_t)d->gy * (uint64_t)d->gt;
    if (nvox > ((uint64_t)1 << 40)) return STKDE_ERR_TOO_LARGE;  // 4 TiB of FP32
    if (!(d->hs / d->sres < 1e9) || !(d->ht / d->tres < 1e9)) return STKDE_ERR_TOO_LARGE;
    return STKDE_OK;
}

stkde_status check_tuning(const stkde_tuning* t) {
    if (!t) return STKDE_OK;
    if (t->tile_t != 0 && t->tile_t != 16 && t->tile_t != 32 && t->tile_t != 64)
        return STKDE_ERR_INVALID_ARG;
    if (t->cell_xy != 0 && (t->cell_xy < 4 || t->cell_xy > 256)) return STKDE_ERR_INVALID_ARG;
    if (t->cell_t != 0 && (t->cell_t < 4 || t->cell_t > 256)) return STKDE_ERR_INVALID_ARG;
    if (t->split_share != 0 && (t->split_share < 64 || t->split_share > 65536))
        return STKDE_ERR_INVALID_ARG;
    if (t->kahan_mode < 0 || t->kahan_mode > 2) return STKDE_ERR_INVALID_ARG;
    if (t->operand_form < 0 || t->operand_form > 1) return STKDE_ERR_INVALID_ARG;
    return STKDE_OK;
}

// Hs = ceil(hv), Ht = ceil(tv) (Sec. 2.1).  A bound beyond the base grid's
// extent changes nothing: points farther out are binned into the edge bins.
int32_t cap_hs(double hv, const stkde_desc& base) {
    return (int32_t)fmin(ceil(hv), (double)(base.gx > base.gy ? base.gx : base.gy) + 2.0);
}
int32_t cap_ht(double tv, const stkde_desc& base) { return (int32_t)fmin(ceil(tv), (double)base.gt + 2.0); }

// most bins an interval of L voxels can touch when bins are c wide
int64_t span(int64_t L, int64_t c) { return (L - 1) / c + 2; }

// bin rows (t, y) one tile of `rows` time rows reads with loop bounds Hs, Ht
int64_t ranges_needed(const stkde::SetGeom& g, int32_t Hs, int32_t Ht, int32_t rows) {
    const int64_t ny = span(stkde::kTileXY + 2 * (int64_t)Hs + 2, g.cxy);
    const int64_t nt = span(rows + 2 * (int64_t)Ht + 2, g.ct);
    return (ny < g.ncy ? ny : g.ncy) * (nt < g.nct ? nt : g.nct);
}

// Bins about as wide as the bandwidth in y and t (the paper's bandwidth-sized
// blocks of points, Sec. 4.2 and Sec. 5.1): a tile then reads a few bin rows.
// Within a row (t, y) a tile reads one contiguous run of x bins, so narrow x
// bins cost no extra ranges and cut the candidates that miss the tile in x:
// x bins are kXBin voxels wide (at most the y edge), widened only to keep the
// bin count within kMaxCells.
void make_set_geom(const stkde_desc& d, int32_t cell_xy, int32_t cell_t, int32_t rows,
                   stkde::SetGeom* out) {
    stkde::SetGeom g{};
    g.gx = (int32_t)d.gx;
    g.gy = (int32_t)d.gy;
    g.gt = (int32_t)d.gt;
    g.x0 = d.x0 - origin_shift(d, d.sres);
    g.y0 = d.y0 - origin_shift(d, d.sres);
    g.t0 = d.t0 - origin_shift(d, d.tres);
    g.sres = d.sres;
    g.tres = d.tres;
    g.hv = d.hs / d.sres;
    g.tv = d.ht / d.tres;
    const int32_t Hs = cap_hs(g.hv, d), Ht = cap_ht(g.tv, d);
    g.cxy = cell_xy ? cell_xy : (int32_t)fmin(256.0, fmax(16.0, 8.0 * ceil(Hs / 8.0)));
    g.ct = cell_t ? cell_t : (int32_t)fmin(256.0, fmax(8.0, 4.0 * ceil(Ht / 4.0)));
    g.cx = g.cxy < kXBin ? g.cxy : kXBin;
    for (;;) {
        g.ncx = ceil_div(d.gx, g.cx);
        g.ncy = ceil_div(d.gy, g.cxy);
        g.nct = ceil_div(d.gt, g.ct);
        const int64_t nc = (int64_t)g.ncx * g.ncy * g.nct;
        const int64_t ny = span(stkde::kTileXY + 2 * (int64_t)Hs + 2, g.cxy);
        const int64_t nt = span(rows + 2 * (int64_t)Ht + 2, g.ct);
        const int64_t ry = ny < g.ncy ? ny : g.ncy, rt = nt < g.nct ? nt : g.nct;
        if (nc <= kMaxCells && ry * rt <= stkde::kMaxRanges) {
            g.ncell = (int32_t)nc;
            break;
        }
        // too many bins: first widen the x bins back towards the y edge; else
        // grow the dimension that contributes more bin rows
        if (nc > kMaxCells && g.cx < g.cxy) {
            g.cx = 2 * g.cx < g.cxy ? 2 * g.cx : g.cxy;
            continue;
        }
        if ((ry >= rt && g.cxy < 65536) || g.ct >= 65536) g.cxy *= 2;
        else g.ct *= 2;
    }
    *out = g;
}

// The grid of `d` as an instance whose set has base grid `base`.
stkde_status make_inst_geom(const stkde_desc& d, const stkde_desc& base, int32_t tile_t,
                            stkde::InstGeom* out) {
    stkde::InstGeom g{};
    g.gx = (int32_t)d.gx;
    g.gy = (int32_t)d.gy;
    g.gt = (int32_t)d.gt;
    g.x0 = d.x0 - origin_shift(d, d.sres);
    g.y0 = d.y0 - origin_shift(d, d.sres);
    g.t0 = d.t0 - origin_shift(d, d.tres);
    g.sres = d.sres;
    g.tres = d.tres;
    g.hs = d.hs;
    g.ht = d.ht;
    g.kernel = kernel_of(d);
    g.hv = d.hs / d.sres;
    g.tv = d.ht / d.tres;
    g.Hs = cap_hs(g.hv, base);
    g.Ht = cap_ht(g.tv, base);
    g.Hs_d = ceil(g.hv);
    g.Ht_d = ceil(g.tv);
    g.inv_hv2 = (float)(1.0 / (g.hv * g.hv));
    g.inv_tv2 = (float)(1.0 / (g.tv * g.tv));
    g.tile_t = tile_t;
    g.ntx = ceil_div(d.gx, stkde::kTileXY);
    g.nty = ceil_div(d.gy, stkde::kTileXY);
    g.ntt = ceil_div(d.gt, tile_t);
    const int64_t nt = (int64_t)g.ntx * g.nty * g.ntt;
    if (nt > 0x7fffffffLL) return STKDE_ERR_TOO_LARGE;
    g.ntiles = (int32_t)nt;
    *out = g;
    return STKDE_OK;
}

// Default rows per tile (measured on gfx950): with short time windows a
// 32-row tile halves the per-tile setup and candidate reads; with long ones
// most points reach most rows of a tile either way, and 16-row tiles give
// the scheduler twice as many, smaller items.
int32_t default_tile_t(double tv) { return ceil(tv) <= 12.0 ? 32 : 16; }

// Compensated accumulation keeps its running pair in memory when tiles are
// expected to finish in one matrix-core phase (the pair is then never
// touched): n points spread over the base grid put about
// n * (16 + 2 Hs + 2)^2 (TT + 2 Ht + 2) / voxels candidates into a tile's bins.
// Either mode gives the same bits; this only picks the faster one.
int acc_mode(bool kahan, int32_t requested, int64_t n, const stkde_desc& base, int32_t Hs, int32_t Ht,
             int32_t rows) {
    if (!kahan) return stkde::kAccPlain;
    if (requested == 1) return stkde::kAccKahanReg;
    if (requested == 2) return stkde::kAccKahanMem;
    const double side = 16.0 + 2.0 * Hs + 2.0;
    const double reach = side * side * (rows + 2.0 * Ht + 2.0);
    const double vox = (double)base.gx * (double)base.gy * (double)base.gt;
    const double est = (double)n * (reach < vox ? reach / vox : 1.0);
    return est <= kSparseCandidates ? stkde::kAccKahanMem : stkde::kAccKahanReg;
}

// The constant factors of the kernel pair times 1/(n hs^2 ht), rounded
// once to FP32 at the store: (2/pi)(3/4) for Epanechnikov, (3/pi)(15/16)
// quartic, 1/(Zs Zt) for the truncated Gaussian (Zs = (pi/2)(1 - e^-2),
// Zt = sqrt(pi/2) erf(sqrt 2)), (pi/2)(3/4) for the pair as printed.
float norm_const(double hs, double ht, int64_t n, int kernel = 0) {
    const double pi = 3.14159265358979323846;
    double c = (2.0 / pi) * 0.75;
    if (kernel == STKDE_KERNEL_QUARTIC) c = (3.0 / pi) * (15.0 / 16.0);
    if (kernel == STKDE_KERNEL_GAUSSIAN) c = 1.0 / ((0.5 * pi * (1.0 - exp(-2.0))) * (sqrt(0.5 * pi) * erf(sqrt(2.0))));
    if (kernel == STKDE_KERNEL_PRINTED) c = (0.5 * pi) * 0.75;
    return (float)(c / ((double)n * hs * hs * ht));
}

// The gather's full-cover path pays off when discs are large against a tile.
bool use_full(double hv, int32_t tile_t) { return tile_t <= 32 && hv >= stkde::kFullMinHv; }

// Two-term FP16 matrix-core operands: the gathers with one bandwidth pair and
// 16- or 32-row tiles have them (every kernel pair), unless the plan's tuning
// asks for FP32 operands -- with the full-cover path only at 16 rows (that
// kernel's 32-row form holds too many registers) and only in a computation of
// its own: a batch keeps FP32 operands on the full-cover path, the kernel its
// one-launch gather holds (with the two-term full-cover kernel that launch
// would run at half the occupancy).
bool use_h16(int kf, bool adapt, bool full, int32_t tile_t, int32_t operand_form, bool batch = false) {
    (void)kf;
    return !adapt && tile_t <= 32 && operand_form == 0 && (!full || (tile_t == 16 && !batch));
}

stkde::InstDev make_dev(const stkde::InstGeom& ig, const stkde::SetGeom& sg, const uint8_t* set_mem,
                        const stkde::SetLayout& sl, int64_t n_norm, int32_t ox, int32_t oy,
                        int32_t ot, float* out, double* stats, bool mass, uint32_t split_share,
                        bool adaptive = false) {
    stkde::InstDev d{};
    d.cell_start = reinterpret_cast<const uint32_t*>(set_mem + sl.cell_start);
    d.recs = reinterpret_cast<const stkde::PointRec*>(set_mem + sl.recs);
    d.bw = adaptive ? reinterpret_cast<const float4*>(set_mem + sl.bw) : nullptr;
    d.out = out;
    d.stats = stats;
    d.tile_part = nullptr;
    d.mass_scale = ig.sres * ig.sres * ig.tres;
    d.gx = ig.gx;
    d.gy = ig.gy;
    d.gt = ig.gt;
    d.ox = ox;
    d.oy = oy;
    d.ot = ot;
    d.Hs = ig.Hs;
    d.Ht = ig.Ht;
    d.cx = sg.cx;
    d.cxy = sg.cxy;
    d.ct = sg.ct;
    d.ncx = sg.ncx;
    d.ncy = sg.ncy;
    d.nct = sg.nct;
    d.ntx = ig.ntx;
    d.nty = ig.nty;
    d.ntiles = ig.ntiles;
    d.tile_base = 0;
    d.tile_t = ig.tile_t;
    d.variant = 0;
    d.flags = (mass && stats) ? stkde::kInstMass : 0u;
    if (!adaptive && ig.kernel == stkde::kKernelEpan && use_full(ig.hv, ig.tile_t)) d.flags |= stkde::kInstFull;
    d.inv_hv2 = ig.inv_hv2;
    d.inv_tv2 = ig.inv_tv2;
    d.inv_hv = (float)(1.0 / ig.hv);
    d.inv_tv = (float)(1.0 / ig.tv);
    d.hv64 = ig.hv;
    d.tv64 = ig.tv;
    d.x64 = (ig.kernel == stkde::kKernelGauss || ig.kernel == stkde::kKernelPrinted)
                ? reinterpret_cast<const double*>(set_mem + sl.x64)
                : nullptr;
    d.cnorm = norm_const(ig.hs, ig.ht, n_norm, ig.kernel);
    d.split_share = split_share;
    return d;
}

// Workspace of stkde_compute: the set region, then one region shared by the
// binning sort, the pass and the point statistics (they run one after the
// other on the stream).
struct ComputeLayout {
    stkde::SetLayout sl;
    stkde::SortLayout so;
    stkde::PassLayout pl;
    size_t shared;  // offset of the shared region
    size_t pstats;  // bytes of the point-statistics partials
    int32_t nblk_pts;
    size_t total;
};

ComputeLayout layout_compute(const stkde_plan_s* p, int64_t n) {
    ComputeLayout c{};
    c.sl = stkde::layout_set(p->sg, n, (p->desc.flags & STKDE_FLAG_ADAPTIVE) != 0, exact_support(p->desc));
    c.so = stkde::layout_sort(p->sg, n, (p->desc.flags & STKDE_FLAG_ADAPTIVE) != 0, exact_support(p->desc));
    c.pl = stkde::layout_pass(&p->ig, 1, p->ig.tile_t, (p->desc.flags & STKDE_FLAG_KAHAN) != 0);
    c.nblk_pts = (int32_t)((n + stkde::kStatBlock - 1) / stkde::kStatBlock);
    c.pstats = al256((size_t)c.nblk_pts * 4 * 8);
    c.shared = al256(c.sl.total);
    size_t u = c.so.total;
    if (c.pl.total > u) u = c.pl.total;
    if (c.pstats > u) u = c.pstats;
    c.total = c.shared + u;
    return c;
}

struct Call {
    ComputeLayout L;
    hipStream_t s;
    uint8_t* ws;
};

stkde_status check_common(stkde_plan_t p, int64_t n, void* d_ws, size_t ws_bytes, void* stream,
                          Call* c) {
    if (!p || n < 1) return STKDE_ERR_INVALID_ARG;
    if (n > 0x7fffffffLL) return STKDE_ERR_TOO_LARGE;
    c->L = layout_compute(p, n);
    if (!d_ws || ws_bytes < c->L.total || ((uintptr_t)d_ws & 255u)) return STKDE_ERR_WORKSPACE;
    c->s = reinterpret_cast<hipStream_t>(stream);
    c->ws = reinterpret_cast<uint8_t*>(d_ws);
    return STKDE_OK;
}

bool same_res(double a, double b) { return fabs(a - b) <= 1e-12 * fabs(b); }

}  // namespace

extern "C" {

const char* stkde_status_string(stkde_status s) {
    switch (s) {
        case STKDE_OK: return "ok";
        case STKDE_ERR_INVALID_ARG: return "invalid argument";
        case STKDE_ERR_TOO_LARGE: return "size too large";
        case STKDE_ERR_WORKSPACE: return "workspace missing or too small";
        case STKDE_ERR_HIP: return "HIP runtime error";
        case STKDE_ERR_UNSUPPORTED: return "unsupported request";
    }
    return "unknown status";
}

int32_t stkde_version(void) { return 200; }

stkde_status stkde_plan(const stkde_desc* d, const stkde_tuning* tun, stkde_plan_t* out) {
    if (!d || !out) return STKDE_ERR_INVALID_ARG;
    stkde_status st = check_desc(d);
    if (st != STKDE_OK) return st;
    st = check_tuning(tun);
    if (st != STKDE_OK) return st;
    int32_t tile_t = tun && tun->tile_t ? tun->tile_t : default_tile_t(d->ht / d->tres);
    // compensated accumulation holds three accumulator sets; with 64-row
    // tiles that would leave one wave per SIMD (the other kernel pairs have
    // 16- and 32-row gathers only)
    if (((d->flags & STKDE_FLAG_KAHAN) || kernel_of(*d) != STKDE_KERNEL_EPANECHNIKOV) && tile_t > 32) tile_t = 32;
    if (kernel_of(*d) != STKDE_KERNEL_EPANECHNIKOV && (d->flags & STKDE_FLAG_ADAPTIVE))
        return STKDE_ERR_UNSUPPORTED;
    stkde_plan_s tmp;
    tmp.desc = *d;
    tmp.split_share = tun && tun->split_share ? (uint32_t)tun->split_share : stkde::kBalanceItems;
    tmp.kahan_mode = tun ? tun->kahan_mode : 0;
    tmp.operand_form = tun ? tun->operand_form : 0;
    make_set_geom(*d, tun ? tun->cell_xy : 0, tun ? tun->cell_t : 0, tile_t, &tmp.sg);
    st = make_inst_geom(*d, *d, tile_t, &tmp.ig);
    if (st != STKDE_OK) return st;
    stkde_plan_s* p = new (std::nothrow) stkde_plan_s(tmp);
    if (!p) return STKDE_ERR_TOO_LARGE;
    *out = p;
    return STKDE_OK;
}

stkde_status stkde_plan_destroy(stkde_plan_t p) {
    if (p) {
        release_events(p);
        release_graph(p);
    }
    delete p;
    return STKDE_OK;
}

stkde_status stkde_plan_profile(stkde_plan_t p, int32_t capacity) {
    if (!p || capacity < 0 || capacity > (1 << 20)) return STKDE_ERR_INVALID_ARG;
    release_events(p);
    for (int32_t k = 0; k < 2 * capacity; ++k) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) {
            release_events(p);
            return STKDE_ERR_HIP;
        }
        p->ev.push_back(e);
    }
    return STKDE_OK;
}

stkde_status stkde_plan_profile_read(stkde_plan_t p, float* ms, int32_t max, int32_t* count) {
    if (!p || !count || (max > 0 && !ms) || max < 0) return STKDE_ERR_INVALID_ARG;
    const int32_t have = p->ev_used / 2;
    const int32_t k = have < max ? have : max;
    for (int32_t i = 0; i < k; ++i) {
        if (hipEventSynchronize(p->ev[(size_t)(2 * i + 1)]) != hipSuccess) return STKDE_ERR_HIP;
        if (hipEventElapsedTime(&ms[i], p->ev[(size_t)(2 * i)], p->ev[(size_t)(2 * i + 1)]) != hipSuccess)
            return STKDE_ERR_HIP;
    }
    *count = k;
    p->ev_used = 0;
    return STKDE_OK;
}

stkde_status stkde_workspace_bytes(stkde_plan_t p, int64_t n, size_t* bytes) {
    if (!p || !bytes || n < 1) return STKDE_ERR_INVALID_ARG;
    if (n > 0x7fffffffLL) return STKDE_ERR_TOO_LARGE;
    *bytes = layout_compute(p, n).total;
    return STKDE_OK;
}

namespace {
bool is_adaptive(stkde_plan_t p) { return (p->desc.flags & STKDE_FLAG_ADAPTIVE) != 0; }

stkde_status bin_impl(stkde_plan_t p, const double* d_xyt, const double* d_hst, int64_t n, void* d_ws,
                      size_t ws_bytes, void* stream) {
    Call c;
    const stkde_status st = check_common(p, n, d_ws, ws_bytes, stream, &c);
    if (st != STKDE_OK) return st;
    if (stkde::launch_bin(p->sg, d_xyt, (int32_t)n, c.ws, c.L.sl, c.ws + c.L.shared, c.L.so, c.s,
                          d_hst, exact_support(p->desc)) != hipSuccess)
        return STKDE_ERR_HIP;
    return STKDE_OK;
}
}  // namespace

stkde_status stkde_bin(stkde_plan_t p, const double* d_xyt, int64_t n, void* d_ws, size_t ws_bytes,
                       void* stream) {
    if (!p || !d_xyt || is_adaptive(p)) return STKDE_ERR_INVALID_ARG;
    return bin_impl(p, d_xyt, nullptr, n, d_ws, ws_bytes, stream);
}

stkde_status stkde_bin_adaptive(stkde_plan_t p, const double* d_xyt, const double* d_hst, int64_t n,
                                void* d_ws, size_t ws_bytes, void* stream) {
    if (!p || !d_xyt || !d_hst || !is_adaptive(p)) return STKDE_ERR_INVALID_ARG;
    return bin_impl(p, d_xyt, d_hst, n, d_ws, ws_bytes, stream);
}

stkde_status stkde_accumulate(stkde_plan_t p, int64_t n, float* d_out, void* d_ws, size_t ws_bytes,
                              double* d_stats, void* stream) {
    if (!d_out) return STKDE_ERR_INVALID_ARG;
    Call c;
    const stkde_status st = check_common(p, n, d_ws, ws_bytes, stream, &c);
    if (st != STKDE_OK) return st;
    const uint32_t fl = p->desc.flags;
    const bool adapt = (fl & STKDE_FLAG_ADAPTIVE) != 0;
    stkde::InstDev d = make_dev(p->ig, p->sg, c.ws, c.L.sl, n, 0, 0, 0, d_out, d_stats,
                                (fl & STKDE_FLAG_MASS) != 0, p->split_share, adapt);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!p->capturing && p->ev_used + 2 <= (int32_t)p->ev.size()) {
        e0 = p->ev[(size_t)p->ev_used];
        e1 = p->ev[(size_t)p->ev_used + 1];
        p->ev_used += 2;
    }
    const int kf = p->ig.kernel;
    int mode = acc_mode((fl & STKDE_FLAG_KAHAN) != 0, p->kahan_mode, n, p->desc, p->ig.Hs, p->ig.Ht,
                        p->ig.tile_t);
    if (kf != stkde::kKernelEpan && mode == stkde::kAccKahanReg) mode = stkde::kAccKahanMem;  // same bits
    const bool full = !adapt && kf == stkde::kKernelEpan && use_full(p->ig.hv, p->ig.tile_t);
    const bool h16 = use_h16(kf, adapt, full, p->ig.tile_t, p->operand_form);
    if (h16 && mode == stkde::kAccKahanReg) mode = stkde::kAccKahanMem;
    if (stkde::launch_pass(&d, 1, c.ws + c.L.shared, c.L.pl, p->ig.tile_t, mode, full, adapt, kf, h16, c.s,
                           e0, e1) != hipSuccess)
        return STKDE_ERR_HIP;
    return STKDE_OK;
}

namespace {
stkde_status compute_impl(stkde_plan_t p, const double* d_xyt, const double* d_hst, int64_t n,
                          float* d_out, void* d_ws, size_t ws_bytes, double* d_stats, void* stream) {
    Call c;
    stkde_status st = check_common(p, n, d_ws, ws_bytes, stream, &c);
    if (st != STKDE_OK) return st;
    st = bin_impl(p, d_xyt, d_hst, n, d_ws, ws_bytes, stream);
    if (st != STKDE_OK) return st;
    st = stkde_accumulate(p, n, d_out, d_ws, ws_bytes, d_stats, stream);
    if (st != STKDE_OK) return st;
    if (d_stats && (p->desc.flags & STKDE_FLAG_POINT_STATS)) {
        double* part = reinterpret_cast<double*>(c.ws + c.L.shared);
        if (stkde::launch_point_stats(p->ig, n, d_xyt, (int32_t)n, d_stats, part, c.L.nblk_pts, c.s,
                                      d_hst) != hipSuccess)
            return STKDE_ERR_HIP;
    }
    return STKDE_OK;
}
}  // namespace

stkde_status stkde_compute(stkde_plan_t p, const double* d_xyt, int64_t n, float* d_out, void* d_ws,
                           size_t ws_bytes, double* d_stats, void* stream) {
    if (!p || !d_xyt || !d_out || is_adaptive(p)) return STKDE_ERR_INVALID_ARG;
    return compute_impl(p, d_xyt, nullptr, n, d_out, d_ws, ws_bytes, d_stats, stream);
}

stkde_status stkde_compute_adaptive(stkde_plan_t p, const double* d_xyt, const double* d_hst, int64_t n,
                                    float* d_out, void* d_ws, size_t ws_bytes, double* d_stats,
                                    void* stream) {
    if (!p || !d_xyt || !d_hst || !d_out || !is_adaptive(p)) return STKDE_ERR_INVALID_ARG;
    return compute_impl(p, d_xyt, d_hst, n, d_out, d_ws, ws_bytes, d_stats, stream);
}

// ---- one computation as a HIP graph ------------------------------------------

stkde_status stkde_plan_capture(stkde_plan_t p, const double* d_xyt, int64_t n, float* d_out, void* d_ws,
                                size_t ws_bytes, double* d_stats) {
    if (!p || !d_xyt || !d_out || is_adaptive(p)) return STKDE_ERR_INVALID_ARG;
    Call c;
    stkde_status st = check_common(p, n, d_ws, ws_bytes, nullptr, &c);
    if (st != STKDE_OK) return st;
    {
        // the gather's launch size is a host query: make it before recording
        const uint32_t fl = p->desc.flags;
        const int kf = p->ig.kernel;
        int mode = acc_mode((fl & STKDE_FLAG_KAHAN) != 0, p->kahan_mode, n, p->desc, p->ig.Hs, p->ig.Ht,
                            p->ig.tile_t);
        if (kf != stkde::kKernelEpan && mode == stkde::kAccKahanReg) mode = stkde::kAccKahanMem;
        const bool full = kf == stkde::kKernelEpan && use_full(p->ig.hv, p->ig.tile_t);
        const bool h16 = use_h16(kf, false, full, p->ig.tile_t, p->operand_form);
        if (h16 && mode == stkde::kAccKahanReg) mode = stkde::kAccKahanMem;
        stkde::prepare_gather(p->ig.tile_t, mode, full, false, kf, h16);
    }
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return STKDE_ERR_HIP;
    hipGraph_t graph = nullptr;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        st = STKDE_ERR_HIP;
    } else {
        p->capturing = true;
        st = compute_impl(p, d_xyt, nullptr, n, d_out, d_ws, ws_bytes, d_stats, cs);
        p->capturing = false;
        // always end the capture, also after a failed launch
        if (hipStreamEndCapture(cs, &graph) != hipSuccess && st == STKDE_OK) st = STKDE_ERR_HIP;
    }
    hipGraphExec_t exec = nullptr;
    if (st == STKDE_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
        st = STKDE_ERR_HIP;
    (void)hipStreamDestroy(cs);
    if (st != STKDE_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return st;
    }
    release_graph(p);
    p->graph = graph;
    p->exec = exec;
    return STKDE_OK;
}

stkde_status stkde_plan_replay(stkde_plan_t p, void* stream) {
    if (!p) return STKDE_ERR_INVALID_ARG;
    if (!p->exec) return STKDE_ERR_UNSUPPORTED;
    if (hipGraphLaunch(p->exec, reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return STKDE_ERR_HIP;
    return STKDE_OK;
}

}  // extern "C"

// ---- one computation in the library's own device scratch -------------------
//
// stkde_compute_noalloc runs stkde_compute with the workspace in `scratch`,
// a file-scope device array that each GPU holds from the library's load
// until the process ends.  In host code `scratch` names a host-side stand-in,
// not device memory: its device address on the current GPU comes from
// hipGetSymbolAddress, taken once per device and kept in scratch_ptr.
static __device__ __align__(256) uint8_t scratch[STKDE_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::atomic<void*> scratch_ptr[kMaxScratchDevices];

// Device address of the current GPU's copy of `scratch` (null on failure).
void* static_scratch() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) return nullptr;
    void* p = scratch_ptr[dev].load(std::memory_order_acquire);
    if (p) return p;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    scratch_ptr[dev].store(p, std::memory_order_release);  // every thread finds the same address
    return p;
}
}  // namespace

extern "C" {

stkde_status stkde_compute_noalloc(stkde_plan_t p, const double* d_xyt, int64_t n, float* d_out,
                                   double* d_stats, void* stream) {
    if (!p || !d_xyt || !d_out || is_adaptive(p) || n < 1) return STKDE_ERR_INVALID_ARG;
    if (n > 0x7fffffffLL) return STKDE_ERR_TOO_LARGE;
    if (layout_compute(p, n).total > (size_t)STKDE_STATIC_SCRATCH_BYTES) return STKDE_ERR_WORKSPACE;
    void* ws = static_scratch();
    if (!ws) return STKDE_ERR_HIP;
    return compute_impl(p, d_xyt, nullptr, n, d_out, ws, (size_t)STKDE_STATIC_SCRATCH_BYTES, d_stats, stream);
}

// ---- binned sets ------------------------------------------------------------

stkde_status stkde_set_plan(const stkde_desc* base, const stkde_tuning* tun, int64_t n,
                            stkde_set_t* out) {
    if (!base || !out || n < 1) return STKDE_ERR_INVALID_ARG;
    if (n > 0x7fffffffLL) return STKDE_ERR_TOO_LARGE;
    stkde_status st = check_desc(base);
    if (st != STKDE_OK) return st;
    if (base->flags != 0) return STKDE_ERR_INVALID_ARG;
    st = check_tuning(tun);
    if (st != STKDE_OK) return st;
    const int32_t rows = tun && tun->tile_t ? tun->tile_t : 32;
    stkde_set_s tmp;
    tmp.base = *base;
    tmp.n = n;
    make_set_geom(*base, tun ? tun->cell_xy : 0, tun ? tun->cell_t : 0, rows, &tmp.sg);
    tmp.sl = stkde::layout_set(tmp.sg, n);
    tmp.so = stkde::layout_sort(tmp.sg, n);
    stkde_set_s* s = new (std::nothrow) stkde_set_s(tmp);
    if (!s) return STKDE_ERR_TOO_LARGE;
    *out = s;
    return STKDE_OK;
}

stkde_status stkde_set_bytes(stkde_set_t s, size_t* set_bytes, size_t* scratch_bytes) {
    if (!s || !set_bytes || !scratch_bytes) return STKDE_ERR_INVALID_ARG;
    *set_bytes = s->sl.total;
    *scratch_bytes = s->so.total;
    return STKDE_OK;
}

stkde_status stkde_set_build(stkde_set_t s, const double* d_xyt, void* d_set, size_t set_bytes,
                             void* d_scratch, size_t scratch_bytes, void* stream) {
    if (!s || !d_xyt) return STKDE_ERR_INVALID_ARG;
    if (!d_set || set_bytes < s->sl.total || ((uintptr_t)d_set & 255u)) return STKDE_ERR_WORKSPACE;
    if (!d_scratch || scratch_bytes < s->so.total || ((uintptr_t)d_scratch & 255u))
        return STKDE_ERR_WORKSPACE;
    if (stkde::launch_bin(s->sg, d_xyt, (int32_t)s->n, reinterpret_cast<uint8_t*>(d_set), s->sl,
                          reinterpret_cast<uint8_t*>(d_scratch), s->so,
                          reinterpret_cast<hipStream_t>(stream)) != hipSuccess)
        return STKDE_ERR_HIP;
    return STKDE_OK;
}

stkde_status stkde_set_destroy(stkde_set_t s) {
    delete s;
    return STKDE_OK;
}

// ---- batches ----------------------------------------------------------------

stkde_status stkde_batch_plan(const stkde_item* items, int32_t count, stkde_batch_t* out) {
    if (!items || !out || count < 1) return STKDE_ERR_INVALID_ARG;
    if (count > kMaxBatch) return STKDE_ERR_TOO_LARGE;
    std::vector<stkde::InstGeom> geo((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        const stkde_item& it = items[i];
        if (!it.plan || !it.set || !it.d_set || !it.d_out) return STKDE_ERR_INVALID_ARG;
        if ((uintptr_t)it.d_set & 255u) return STKDE_ERR_INVALID_ARG;
        const stkde_desc& d = it.plan->desc;
        const stkde_desc& b = it.set->base;
        if (d.flags & (STKDE_FLAG_POINT_STATS | STKDE_FLAG_ADAPTIVE | STKDE_FLAG_CORNER | STKDE_KERNEL_MASK))
            return STKDE_ERR_UNSUPPORTED;
        if (!same_res(d.sres, b.sres) || !same_res(d.tres, b.tres)) return STKDE_ERR_INVALID_ARG;
        if (d.hs > b.hs || d.ht > b.ht) return STKDE_ERR_INVALID_ARG;
        if (it.ox < 0 || it.oy < 0 || it.ot < 0 || it.ox + d.gx > b.gx || it.oy + d.gy > b.gy ||
            it.ot + d.gt > b.gt)
            return STKDE_ERR_INVALID_ARG;
        const double tol_s = 1e-6 * b.sres, tol_t = 1e-6 * b.tres;
        if (fabs(d.x0 - (b.x0 + (double)it.ox * b.sres)) > tol_s ||
            fabs(d.y0 - (b.y0 + (double)it.oy * b.sres)) > tol_s ||
            fabs(d.t0 - (b.t0 + (double)it.ot * b.tres)) > tol_t)
            return STKDE_ERR_INVALID_ARG;
        const stkde_status st = make_inst_geom(d, b, it.plan->ig.tile_t, &geo[(size_t)i]);
        if (st != STKDE_OK) return st;
        if (ranges_needed(it.set->sg, geo[(size_t)i].Hs, geo[(size_t)i].Ht, geo[(size_t)i].tile_t) >
            stkde::kMaxRanges)
            return STKDE_ERR_UNSUPPORTED;
    }
    stkde_batch_s* bt = new (std::nothrow) stkde_batch_s;
    if (!bt) return STKDE_ERR_TOO_LARGE;
    bt->items.assign(items, items + count);
    // one pass per (tile rows, accumulation mode)
    std::vector<int> mode((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        const stkde_item& it = items[i];
        mode[(size_t)i] = acc_mode((it.plan->desc.flags & STKDE_FLAG_KAHAN) != 0, it.plan->kahan_mode,
                                   it.set->n, it.set->base, geo[(size_t)i].Hs, geo[(size_t)i].Ht,
                                   geo[(size_t)i].tile_t);
    }
    // one pass per (tile rows, plain or compensated, operand form); an FP32
    // pass takes the register form of Kahan if any of its grids expects dense
    // tiles (both forms give the same bits) and the kernel with the
    // full-cover path if any of its grids uses it (the path is switched per
    // grid); a grid takes the same kernel as alone
    const int tts[3] = {16, 32, 64};
    for (int kahan = 0; kahan < 2; ++kahan) {
        for (int tt : tts) {
            for (int h16 = 0; h16 < 2; ++h16) {
                stkde_batch_s::Group g;
                g.tile_t = tt;
                g.kahan = kahan != 0;
                g.h16 = h16 != 0;
                g.mode = g.kahan ? stkde::kAccKahanMem : stkde::kAccPlain;
                g.full = false;
                for (int32_t i = 0; i < count; ++i) {
                    const bool fi = use_full(geo[(size_t)i].hv, tt);
                    const bool hi = use_h16(stkde::kKernelEpan, false, fi, tt, items[i].plan->operand_form, true);
                    if ((mode[(size_t)i] != stkde::kAccPlain) == g.kahan && geo[(size_t)i].tile_t == tt &&
                        hi == g.h16) {
                        g.idx.push_back(i);
                        g.geo.push_back(geo[(size_t)i]);
                        if (mode[(size_t)i] == stkde::kAccKahanReg && !g.h16) g.mode = stkde::kAccKahanReg;
                        if (fi) g.full = true;
                    }
                }
                if (g.idx.empty()) continue;
                g.pl = stkde::layout_pass(g.geo.data(), (int32_t)g.geo.size(), tt, g.kahan);
                if (g.pl.T > 0x7fffffffLL) {
                    delete bt;
                    return STKDE_ERR_TOO_LARGE;
                }
                bt->ws_bytes = std::max(bt->ws_bytes, g.pl.total);
                bt->groups.push_back(std::move(g));
            }
        }
    }
    // The passes of a batch that is all plain or all compensated, with 16- and
    // 32-row tiles, run as one pass with one gather launch (the multi-variant
    // gather): each grid keeps its kernel's code -- the full-cover FP32 kernel
    // for the FP32 passes (the path is switched per grid; compensated sums in
    // the scratch form, which gives the bits of the register form), the
    // two-term FP16 kernel for the others -- so each keeps the bits of its own
    // pass.
    if (bt->groups.size() > 1) {
        bool one = true;
        for (const auto& g : bt->groups)
            one = one && g.kahan == bt->groups[0].kahan && (g.tile_t == 16 || g.tile_t == 32);
        if (one) {
            stkde_batch_s::Group m;
            m.kahan = bt->groups[0].kahan;
            m.mode = m.kahan ? stkde::kAccKahanMem : stkde::kAccPlain;
            m.full = false;
            m.h16 = false;
            m.multi = true;
            // the multi-variant gather spaces its Kahan and partial slots for
            // 32-row tiles whatever rows the batch's grids have: so does the layout
            m.tile_t = 32;
            for (const auto& g : bt->groups) {
                for (size_t k = 0; k < g.idx.size(); ++k) {
                    m.idx.push_back(g.idx[k]);
                    m.geo.push_back(g.geo[k]);
                    m.variant.push_back(stkde::multi_variant(g.tile_t, g.h16));
                }
            }
            m.pl = stkde::layout_pass(m.geo.data(), (int32_t)m.geo.size(), m.tile_t, m.kahan);
            if (m.pl.T > 0x7fffffffLL) {
                delete bt;
                return STKDE_ERR_TOO_LARGE;
            }
            bt->groups.clear();
            bt->ws_bytes = m.pl.total;
            bt->groups.push_back(std::move(m));
        }
    }
    *out = bt;
    return STKDE_OK;
}

stkde_status stkde_batch_workspace_bytes(stkde_batch_t b, size_t* bytes) {
    if (!b || !bytes) return STKDE_ERR_INVALID_ARG;
    *bytes = b->ws_bytes;
    return STKDE_OK;
}

stkde_status stkde_batch_passes(stkde_batch_t b, int32_t* passes) {
    if (!b || !passes) return STKDE_ERR_INVALID_ARG;
    *passes = (int32_t)b->groups.size();
    return STKDE_OK;
}

namespace {

stkde_status batch_enqueue(stkde_batch_t b, uint8_t* ws, hipStream_t s) {
    std::vector<stkde::InstDev> devs;
    for (const auto& g : b->groups) {
        devs.clear();
        for (size_t k = 0; k < g.idx.size(); ++k) {
            const stkde_item& it = b->items[(size_t)g.idx[k]];
            devs.push_back(make_dev(g.geo[k], it.set->sg, reinterpret_cast<const uint8_t*>(it.d_set),
                                    it.set->sl, it.set->n, (int32_t)it.ox, (int32_t)it.oy,
                                    (int32_t)it.ot, it.d_out, it.d_stats,
                                    (it.plan->desc.flags & STKDE_FLAG_MASS) != 0,
                                    it.plan->split_share));
            if (g.multi) devs.back().variant = g.variant[k];
        }
        if (stkde::launch_pass(devs.data(), (int32_t)devs.size(), ws, g.pl, g.tile_t, g.mode, g.full, false,
                               stkde::kKernelEpan, g.h16, s, nullptr, nullptr, g.multi) != hipSuccess)
            return STKDE_ERR_HIP;
    }
    return STKDE_OK;
}

}  // namespace

stkde_status stkde_batch_run(stkde_batch_t b, void* d_ws, size_t ws_bytes, void* stream) {
    if (!b) return STKDE_ERR_INVALID_ARG;
    if (!d_ws || ws_bytes < b->ws_bytes || ((uintptr_t)d_ws & 255u)) return STKDE_ERR_WORKSPACE;
    return batch_enqueue(b, reinterpret_cast<uint8_t*>(d_ws), reinterpret_cast<hipStream_t>(stream));
}

stkde_status stkde_batch_capture(stkde_batch_t b, void* d_ws, size_t ws_bytes) {
    if (!b) return STKDE_ERR_INVALID_ARG;
    if (!d_ws || ws_bytes < b->ws_bytes || ((uintptr_t)d_ws & 255u)) return STKDE_ERR_WORKSPACE;
    for (const auto& g : b->groups) {
        if (g.multi) stkde::prepare_gather_multi(g.kahan);
        else stkde::prepare_gather(g.tile_t, g.mode, g.full, false, stkde::kKernelEpan, g.h16);
    }
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return STKDE_ERR_HIP;
    hipGraph_t graph = nullptr;
    stkde_status st = STKDE_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        st = STKDE_ERR_HIP;
    } else {
        st = batch_enqueue(b, reinterpret_cast<uint8_t*>(d_ws), cs);
        // always end the capture, also after a failed launch
        if (hipStreamEndCapture(cs, &graph) != hipSuccess && st == STKDE_OK) st = STKDE_ERR_HIP;
    }
    hipGraphExec_t exec = nullptr;
    if (st == STKDE_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
        st = STKDE_ERR_HIP;
    if (st != STKDE_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cs);
        return st;
    }
    (void)hipStreamDestroy(cs);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->graph = graph;
    b->exec = exec;
    return STKDE_OK;
}

stkde_status stkde_batch_replay(stkde_batch_t b, void* stream) {
    if (!b) return STKDE_ERR_INVALID_ARG;
    if (!b->exec) return STKDE_ERR_UNSUPPORTED;
    if (hipGraphLaunch(b->exec, reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return STKDE_ERR_HIP;
    return STKDE_OK;
}

stkde_status stkde_batch_destroy(stkde_batch_t b) {
    if (!b) return STKDE_OK;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    delete b;
    return STKDE_OK;
}

// ---- baselines (stkde_ablation.h) ------------------------------------------------

stkde_status stkde_ablation_accumulate(stkde_plan_t p, int32_t method, int64_t n, float* d_out,
                                       void* d_ws, size_t ws_bytes, void* stream) {
    if (!d_out || (method != STKDE_ABLATION_SCATTER && method != STKDE_ABLATION_VOXEL))
        return STKDE_ERR_INVALID_ARG;
    Call c;
    const stkde_status st = check_common(p, n, d_ws, ws_bytes, stream, &c);
    if (st != STKDE_OK) return st;
    if (is_adaptive(p) || p->ig.kernel != stkde::kKernelEpan) return STKDE_ERR_UNSUPPORTED;
    // the scatter indexes a footprint box, the voxel gather its grid, in 32 bits
    const stkde::InstGeom& g = p->ig;
    const int64_t box = (int64_t)std::min<int64_t>(g.gx, 2 * (int64_t)g.Hs + 2) *
                        std::min<int64_t>(g.gy, 2 * (int64_t)g.Hs + 2) *
                        std::min<int64_t>(g.gt, 2 * (int64_t)g.Ht + 2);
    const int64_t blocks = ((int64_t)g.gx * g.gy * g.gt + 255) / 256;
    if (box > 0x7fffffffLL || blocks > 0x7fffffffLL) return STKDE_ERR_UNSUPPORTED;
    const float cn = norm_const(p->ig.hs, p->ig.ht, n);
    const hipError_t e =
        method == STKDE_ABLATION_SCATTER
            ? stkde::launch_ablation_scatter(p->sg, p->ig, c.ws, c.L.sl, cn, d_out, c.s)
            : stkde::launch_ablation_voxel(p->sg, p->ig, c.ws, c.L.sl, cn, d_out, c.s);
    return e == hipSuccess ? STKDE_OK : STKDE_ERR_HIP;
}

stkde_status stkde_ablation_compute(stkde_plan_t p, int32_t method, const double* d_xyt, int64_t n,
                                    float* d_out, void* d_ws, size_t ws_bytes, void* stream) {
    if (!p || !d_xyt || !d_out || (method != STKDE_ABLATION_SCATTER && method != STKDE_ABLATION_VOXEL))
        return STKDE_ERR_INVALID_ARG;
    if (is_adaptive(p) || p->ig.kernel != stkde::kKernelEpan) return STKDE_ERR_UNSUPPORTED;
    stkde_status st = stkde_bin(p, d_xyt, n, d_ws, ws_bytes, stream);
    if (st != STKDE_OK) return st;
    return stkde_ablation_accumulate(p, method, n, d_out, d_ws, ws_bytes, stream);
}

}  // extern "C"
