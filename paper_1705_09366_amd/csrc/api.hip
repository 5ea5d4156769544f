// api.hip -- host side of the C ABI declared in include/stkde.h: argument
// validation, plan geometry, workspace layout and the launch sequence
//   bin (transform, radix sort, bin offsets, records) -> gather/store
//   -> optional statistics.
#include <math.h>
#include <stdlib.h>

#include <new>

#include "../../include/stkde.h"
#include "stkde_internal.h"

struct stkde_plan_s {
    stkde_desc desc;
    stkde::Geometry g;
};

namespace {

constexpr int64_t kMaxDim = 65535;
constexpr int32_t kMaxCells = 1 << 22;  // keys of at most 23 bits: <= 3 radix passes
constexpr uint32_t kKnownFlags = STKDE_FLAG_KAHAN | STKDE_FLAG_MASS | STKDE_FLAG_POINT_STATS;

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

int32_t ceil_div(int64_t a, int64_t b) { return (int32_t)((a + b - 1) / b); }

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

int32_t stkde_version(void) { return 100; }

stkde_status stkde_plan(const stkde_desc* d, const stkde_tuning* tun, stkde_plan_t* out) {
    if (!d || !out) return STKDE_ERR_INVALID_ARG;
    if (d->gx < 1 || d->gy < 1 || d->gt < 1) return STKDE_ERR_INVALID_ARG;
    if (d->gx > kMaxDim || d->gy > kMaxDim || d->gt > kMaxDim) return STKDE_ERR_TOO_LARGE;
    if (!finite_pos(d->sres) || !finite_pos(d->tres) || !finite_pos(d->hs) || !finite_pos(d->ht))
        return STKDE_ERR_INVALID_ARG;
    if (!isfinite(d->x0) || !isfinite(d->y0) || !isfinite(d->t0)) return STKDE_ERR_INVALID_ARG;
    if (d->flags & ~kKnownFlags) return STKDE_ERR_INVALID_ARG;
    const uint64_t nvox = (uint64_t)d->gx * (uint64_t)d->gy * (uint64_t)d->gt;
    if (nvox > ((uint64_t)1 << 40)) return STKDE_ERR_TOO_LARGE;  // 4 TiB of FP32

    int32_t tile_t = 0, cell_xy = 0, cell_t = 0;
    if (tun) {
        if (tun->tile_t != 0 && tun->tile_t != 16 && tun->tile_t != 32 && tun->tile_t != 64)
            return STKDE_ERR_INVALID_ARG;
        if (tun->cell_xy != 0 && (tun->cell_xy < 4 || tun->cell_xy > 256))
            return STKDE_ERR_INVALID_ARG;
        if (tun->cell_t != 0 && (tun->cell_t < 4 || tun->cell_t > 256))
            return STKDE_ERR_INVALID_ARG;
        tile_t = tun->tile_t;
        cell_xy = tun->cell_xy;
        cell_t = tun->cell_t;
    }

    stkde::Geometry g{};
    g.gx = (int32_t)d->gx;
    g.gy = (int32_t)d->gy;
    g.gt = (int32_t)d->gt;
    g.x0 = d->x0;
    g.y0 = d->y0;
    g.t0 = d->t0;
    g.sres = d->sres;
    g.tres = d->tres;
    g.inv_sres = 1.0 / d->sres;
    g.inv_tres = 1.0 / d->tres;
    g.hs = d->hs;
    g.ht = d->ht;
    g.hv = d->hs / d->sres;
    g.tv = d->ht / d->tres;
    // Hs = ceil(hs/sres), Ht = ceil(ht/tres) (Sec. 2.1).  Beyond the grid
    // extent a larger bound changes nothing, so cap it there.
    const double hcap = (double)(d->gx > d->gy ? d->gx : d->gy) + 2.0;
    g.Hs = (int32_t)fmin(ceil(g.hv), hcap);
    g.Ht = (int32_t)fmin(ceil(g.tv), (double)d->gt + 2.0);
    if (!(g.hv < 1e9) || !(g.tv < 1e9)) return STKDE_ERR_TOO_LARGE;
    g.Hs_d = ceil(g.hv);
    g.Ht_d = ceil(g.tv);
    g.inv_hv2 = (float)(1.0 / (g.hv * g.hv));
    g.inv_tv2 = (float)(1.0 / (g.tv * g.tv));

    g.tile_t = tile_t ? tile_t : 32;
    // compensated accumulation holds three accumulator sets; with 64-row
    // tiles that would leave one wave per SIMD
    if ((d->flags & STKDE_FLAG_KAHAN) && g.tile_t > 32) g.tile_t = 32;
    // Bins about as wide as the bandwidth (the paper's bandwidth-sized
    // blocks of points, Sec. 4.2 and Sec. 5.1): a tile then reads a few bin
    // rows, and few of the candidates it reads miss it.
    g.cxy = cell_xy ? cell_xy : (int32_t)fmin(256.0, fmax(16.0, 8.0 * ceil(g.Hs / 8.0)));
    g.ct = cell_t ? cell_t : (int32_t)fmin(256.0, fmax(8.0, 4.0 * ceil(g.Ht / 4.0)));
    // most bins an interval of L voxels can touch when bins are c wide
    auto span = [](int64_t L, int64_t c) { return (L - 1) / c + 2; };
    for (;;) {
        g.ncx = ceil_div(d->gx, g.cxy);
        g.ncy = ceil_div(d->gy, g.cxy);
        g.nct = ceil_div(d->gt, g.ct);
        const int64_t nc = (int64_t)g.ncx * g.ncy * g.nct;
        const int64_t ny = span(stkde::kTileXY + 2 * (int64_t)g.Hs + 2, g.cxy);
        const int64_t nt = span(g.tile_t + 2 * (int64_t)g.Ht + 2, g.ct);
        const int64_t ry = ny < g.ncy ? ny : g.ncy, rt = nt < g.nct ? nt : g.nct;
        if (nc <= kMaxCells && ry * rt <= stkde::kMaxRanges) {
            g.ncell = (int32_t)nc;
            g.max_ranges = (int32_t)(ry * rt);
            break;
        }
        // grow the dimension that contributes more bin rows
        if ((ry >= rt && g.cxy < 65536) || g.ct >= 65536) g.cxy *= 2;
        else g.ct *= 2;
    }
    // Keys of at most 16 bits sort in two radix passes instead of three:
    // widen the bins in t (up to twice) when that alone gets there and the
    // range limit still holds.
    if (!cell_t && g.ncell >= 65536 && g.ncell < (1 << 20)) {
        for (int32_t c = g.ct + 1; c <= 2 * g.ct; ++c) {
            const int64_t nct = (d->gt + c - 1) / c;
            const int64_t nc = (int64_t)g.ncx * g.ncy * nct;
            const int64_t nt = span(g.tile_t + 2 * (int64_t)g.Ht + 2, c);
            const int64_t ry = span(stkde::kTileXY + 2 * (int64_t)g.Hs + 2, g.cxy);
            const int64_t rr = (ry < g.ncy ? ry : g.ncy) * (nt < nct ? nt : nct);
            if (nc < 65536 && rr <= stkde::kMaxRanges) {
                g.ct = c;
                g.nct = (int32_t)nct;
                g.ncell = (int32_t)nc;
                g.max_ranges = (int32_t)rr;
                break;
            }
        }
    }
    g.ntx = ceil_div(d->gx, stkde::kTileXY);
    g.nty = ceil_div(d->gy, stkde::kTileXY);
    g.ntt = ceil_div(d->gt, g.tile_t);
    const int64_t nt = (int64_t)g.ntx * g.nty * g.ntt;
    if (nt > 0x7fffffffLL) return STKDE_ERR_TOO_LARGE;
    g.ntiles = (int32_t)nt;

    stkde_plan_s* p = new (std::nothrow) stkde_plan_s;
    if (!p) return STKDE_ERR_TOO_LARGE;
    p->desc = *d;
    p->g = g;
    *out = p;
    return STKDE_OK;
}

stkde_status stkde_plan_destroy(stkde_plan_t p) {
    delete p;
    return STKDE_OK;
}

stkde_status stkde_workspace_bytes(stkde_plan_t p, int64_t n, size_t* bytes) {
    if (!p || !bytes || n < 1) return STKDE_ERR_INVALID_ARG;
    if (n > 0x7fffffffLL) return STKDE_ERR_TOO_LARGE;
    *bytes = stkde::layout_workspace(p->g, n).total;
    return STKDE_OK;
}

namespace {

struct Call {
    stkde::Workspace w;
    hipStream_t s;
    uint8_t* ws;
};

stkde_status check_common(stkde_plan_t p, int64_t n, void* d_ws, size_t ws_bytes, void* stream,
                          Call* c) {
    if (!p || n < 1) return STKDE_ERR_INVALID_ARG;
    if (n > 0x7fffffffLL) return STKDE_ERR_TOO_LARGE;
    c->w = stkde::layout_workspace(p->g, n);
    if (!d_ws || ws_bytes < c->w.total || ((uintptr_t)d_ws & 255u)) return STKDE_ERR_WORKSPACE;
    c->s = reinterpret_cast<hipStream_t>(stream);
    c->ws = reinterpret_cast<uint8_t*>(d_ws);
    return STKDE_OK;
}

// (2/pi) (3/4) / (n hs^2 ht): the constants of both kernels and the
// estimator's normalisation, rounded once to FP32 at the store.
float norm_const(const stkde::Geometry& g, int64_t n) {
    return (float)((2.0 / 3.14159265358979323846) * 0.75 / ((double)n * g.hs * g.hs * g.ht));
}

}  // namespace

stkde_status stkde_bin(stkde_plan_t p, const double* d_xyt, int64_t n, void* d_ws, size_t ws_bytes,
                       void* stream) {
    if (!d_xyt) return STKDE_ERR_INVALID_ARG;
    Call c;
    const stkde_status st = check_common(p, n, d_ws, ws_bytes, stream, &c);
    if (st != STKDE_OK) return st;
    if (stkde::launch_bin(p->g, d_xyt, (int32_t)n, c.ws, c.w, c.s) != hipSuccess) return STKDE_ERR_HIP;
    return STKDE_OK;
}

stkde_status stkde_accumulate(stkde_plan_t p, int64_t n, float* d_out, void* d_ws, size_t ws_bytes,
                              double* d_stats, void* stream) {
    if (!d_out) return STKDE_ERR_INVALID_ARG;
    Call c;
    const stkde_status st = check_common(p, n, d_ws, ws_bytes, stream, &c);
    if (st != STKDE_OK) return st;
    const stkde::Geometry& g = p->g;
    const uint32_t fl = p->desc.flags;
    const bool mass = (fl & STKDE_FLAG_MASS) && d_stats;
    if (stkde::launch_gather(g, norm_const(g, n), (fl & STKDE_FLAG_KAHAN) != 0, mass, d_out, c.ws, c.w,
                             c.s) != hipSuccess)
        return STKDE_ERR_HIP;
    if (d_stats) {
        if (stkde::launch_stats(g, nullptr, (int32_t)n, false, d_stats, c.ws, c.w, c.s) != hipSuccess)
            return STKDE_ERR_HIP;
        if (mass && stkde::launch_mass_reduce(g, d_stats, c.ws, c.w, c.s) != hipSuccess)
            return STKDE_ERR_HIP;
    }
    return STKDE_OK;
}

stkde_status stkde_compute(stkde_plan_t p, const double* d_xyt, int64_t n, float* d_out, void* d_ws,
                           size_t ws_bytes, double* d_stats, void* stream) {
    if (!p || !d_xyt || !d_out) return STKDE_ERR_INVALID_ARG;
    Call c;
    stkde_status st = check_common(p, n, d_ws, ws_bytes, stream, &c);
    if (st != STKDE_OK) return st;
    st = stkde_bin(p, d_xyt, n, d_ws, ws_bytes, stream);
    if (st != STKDE_OK) return st;
    st = stkde_accumulate(p, n, d_out, d_ws, ws_bytes, d_stats, stream);
    if (st != STKDE_OK) return st;
    if (d_stats && (p->desc.flags & STKDE_FLAG_POINT_STATS)) {
        if (stkde::launch_point_stats(p->g, d_xyt, (int32_t)n, d_stats, c.ws, c.w, c.s) != hipSuccess)
            return STKDE_ERR_HIP;
    }
    return STKDE_OK;
}

}  // extern "C"
