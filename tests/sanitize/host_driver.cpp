// host_driver.cpp -- exercises the host side of the library's C ABI (plan,
// set and batch planning, workspace sizing, argument checks of every entry
// point) without a GPU, for a build of the host code under AddressSanitizer
// and UndefinedBehaviorSanitizer.  No call here reaches the HIP runtime:
// every compute call is rejected by the host-side validation first.  Exit
// status 0 when every expectation holds.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <vector>

#include "stkde.h"

static int failures = 0;
#define EXPECT(cond)                                                   \
    do {                                                               \
        if (!(cond)) {                                                 \
            fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                \
        }                                                              \
    } while (0)

static uint64_t rng = 0x243f6a8885a308d3ull;
static double uni() {
    uint64_t z = (rng += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static stkde_desc desc(int64_t gx, int64_t gy, int64_t gt, double hs, double ht, uint32_t flags = 0) {
    stkde_desc d;
    memset(&d, 0, sizeof d);
    d.gx = gx;
    d.gy = gy;
    d.gt = gt;
    d.sres = 1.0;
    d.tres = 1.0;
    d.hs = hs;
    d.ht = ht;
    d.flags = flags;
    return d;
}

int main() {
    void* fake = (void*)0x10000;
    // plans over random shapes, bandwidths, flags and tunings
    for (int k = 0; k < 400; ++k) {
        stkde_desc d = desc(1 + (int64_t)(uni() * 3000), 1 + (int64_t)(uni() * 3000), 1 + (int64_t)(uni() * 600),
                            0.2 + 80.0 * uni(), 0.2 + 60.0 * uni(),
                            (uni() < 0.5 ? STKDE_FLAG_KAHAN : 0u) | (uni() < 0.5 ? STKDE_FLAG_MASS : 0u) |
                                (uni() < 0.2 ? STKDE_FLAG_CORNER : 0u) | STKDE_FLAG_KERNEL(k % 4));
        d.sres = 0.25 + 2.0 * uni();
        d.tres = 0.25 + 2.0 * uni();
        d.x0 = 1e3 * (uni() - 0.5);
        stkde_tuning t;
        memset(&t, 0, sizeof t);
        const int tt[] = {0, 16, 32, 64};
        t.tile_t = tt[k % 4];
        t.cell_xy = uni() < 0.5 ? 0 : 4 + (int)(uni() * 250);
        t.cell_t = uni() < 0.5 ? 0 : 4 + (int)(uni() * 250);
        t.split_share = uni() < 0.5 ? 0 : 64 + (int)(uni() * 60000);
        t.kahan_mode = k % 3;
        t.operand_form = k % 2;
        stkde_plan_t p = nullptr;
        const stkde_status st = stkde_plan(&d, uni() < 0.5 ? &t : nullptr, &p);
        EXPECT(st == STKDE_OK);
        if (st != STKDE_OK) continue;
        size_t a = 0, b = 0;
        EXPECT(stkde_workspace_bytes(p, 1000, &a) == STKDE_OK);
        EXPECT(stkde_workspace_bytes(p, 2000000, &b) == STKDE_OK);
        EXPECT(a > 0 && b > a);
        // compute calls rejected on the host
        EXPECT(stkde_compute(p, nullptr, 10, (float*)fake, fake, a, nullptr, nullptr) == STKDE_ERR_INVALID_ARG);
        EXPECT(stkde_compute(p, (const double*)fake, 0, (float*)fake, fake, a, nullptr, nullptr) ==
               STKDE_ERR_INVALID_ARG);
        EXPECT(stkde_compute(p, (const double*)fake, 1000, (float*)fake, fake, a - 1, nullptr, nullptr) ==
               STKDE_ERR_WORKSPACE);
        EXPECT(stkde_compute_noalloc(p, (const double*)fake, 0, (float*)fake, nullptr, nullptr) ==
               STKDE_ERR_INVALID_ARG);
        EXPECT(stkde_plan_destroy(p) == STKDE_OK);
    }
    // invalid descriptions and tunings
    {
        stkde_plan_t p = nullptr;
        stkde_desc d = desc(0, 4, 4, 1.0, 1.0);
        EXPECT(stkde_plan(&d, nullptr, &p) == STKDE_ERR_INVALID_ARG);
        d = desc(70000, 4, 4, 1.0, 1.0);
        EXPECT(stkde_plan(&d, nullptr, &p) == STKDE_ERR_TOO_LARGE);
        d = desc(4, 4, 4, NAN, 1.0);
        EXPECT(stkde_plan(&d, nullptr, &p) == STKDE_ERR_INVALID_ARG);
        d = desc(4, 4, 4, 1.0, 1.0, 0x80000000u);
        EXPECT(stkde_plan(&d, nullptr, &p) == STKDE_ERR_INVALID_ARG);
        d = desc(4, 4, 4, 1.0, 1.0);
        stkde_tuning t;
        memset(&t, 0, sizeof t);
        t.tile_t = 24;
        EXPECT(stkde_plan(&d, &t, &p) == STKDE_ERR_INVALID_ARG);
        EXPECT(stkde_plan(nullptr, nullptr, &p) == STKDE_ERR_INVALID_ARG);
        EXPECT(stkde_plan_destroy(nullptr) == STKDE_OK);
    }
    // binned sets and batches over them (fake device pointers: planning only)
    for (int k = 0; k < 40; ++k) {
        stkde_desc base = desc(64 + (int64_t)(uni() * 1000), 64 + (int64_t)(uni() * 1000), 32 + (int64_t)(uni() * 200),
                               3.0 + 30.0 * uni(), 2.0 + 20.0 * uni());
        stkde_set_t s = nullptr;
        const int64_t n = 1 + (int64_t)(uni() * 500000);
        EXPECT(stkde_set_plan(&base, nullptr, n, &s) == STKDE_OK);
        size_t sb = 0, scb = 0;
        EXPECT(stkde_set_bytes(s, &sb, &scb) == STKDE_OK);
        EXPECT(sb > 0 && scb > 0);
        std::vector<stkde_plan_t> plans;
        std::vector<stkde_item> items;
        const int m = 1 + (int)(uni() * 12);
        for (int i = 0; i < m; ++i) {
            const int64_t gx = 1 + (int64_t)(uni() * (double)(base.gx - 1));
            const int64_t gy = 1 + (int64_t)(uni() * (double)(base.gy - 1));
            const int64_t gt = 1 + (int64_t)(uni() * (double)(base.gt - 1));
            const int64_t ox = (int64_t)(uni() * (double)(base.gx - gx));
            const int64_t oy = (int64_t)(uni() * (double)(base.gy - gy));
            const int64_t ot = (int64_t)(uni() * (double)(base.gt - gt));
            stkde_desc d = desc(gx, gy, gt, base.hs * (0.3 + 0.7 * uni()), base.ht * (0.3 + 0.7 * uni()),
                                (i % 2) ? STKDE_FLAG_KAHAN : 0u);
            d.x0 = base.x0 + (double)ox;
            d.y0 = base.y0 + (double)oy;
            d.t0 = base.t0 + (double)ot;
            stkde_tuning t;
            memset(&t, 0, sizeof t);
            t.tile_t = 16;
            stkde_plan_t p = nullptr;
            EXPECT(stkde_plan(&d, &t, &p) == STKDE_OK);
            plans.push_back(p);
            stkde_item it;
            memset(&it, 0, sizeof it);
            it.plan = p;
            it.set = s;
            it.d_set = fake;
            it.ox = ox;
            it.oy = oy;
            it.ot = ot;
            it.d_out = (float*)fake;
            items.push_back(it);
        }
        stkde_batch_t b = nullptr;
        const stkde_status st = stkde_batch_plan(items.data(), (int32_t)items.size(), &b);
        EXPECT(st == STKDE_OK || st == STKDE_ERR_UNSUPPORTED);
        if (st == STKDE_OK) {
            size_t wb = 0;
            EXPECT(stkde_batch_workspace_bytes(b, &wb) == STKDE_OK && wb > 0);
            EXPECT(stkde_batch_run(b, nullptr, wb, nullptr) == STKDE_ERR_WORKSPACE);
            EXPECT(stkde_batch_replay(b, nullptr) == STKDE_ERR_UNSUPPORTED);
            EXPECT(stkde_batch_destroy(b) == STKDE_OK);
        }
        // an item whose window leaves the base grid is refused
        items[0].ox = base.gx;
        EXPECT(stkde_batch_plan(items.data(), (int32_t)items.size(), &b) == STKDE_ERR_INVALID_ARG);
        for (stkde_plan_t p : plans) stkde_plan_destroy(p);
        EXPECT(stkde_set_build(s, nullptr, fake, sb, fake, scb, nullptr) == STKDE_ERR_INVALID_ARG);
        EXPECT(stkde_set_destroy(s) == STKDE_OK);
    }
    for (int c = -6; c <= 1; ++c) EXPECT(stkde_status_string((stkde_status)c) != nullptr);
    EXPECT(stkde_version() > 0);
    if (failures) {
        fprintf(stderr, "%d failures\n", failures);
        return 1;
    }
    printf("host sanitizer driver: ok\n");
    return 0;
}
