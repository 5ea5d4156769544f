"""GPU parity of binned sets and batches, through the C ABI.

A batch computes many grids in one work list (one gather launch when its
grids are all plain or all compensated with 16- or 32-row tiles, else one per
(tile_t, Kahan, operand form) group):
bandwidth sweeps over one binned set, voxel-aligned windows of a base grid,
mixed tile shapes, split hot tiles.  Every grid is compared with the FP64
oracle on the same points (bar: max |gpu - oracle| <= 1e-5 max(oracle));
a grid in a batch is bitwise the grid of the same item alone when none of
its tiles is split; graph replays are bitwise the eager run.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads
from oracle import Grid

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_09366_amd as m
    m.lib()
    return torch


def _check_close(gpu, ref, tol=TOL):
    scale = float(np.max(np.abs(ref)))
    err = float(np.max(np.abs(gpu.astype(np.float64) - ref))) if ref.size else 0.0
    assert err <= tol * max(scale, 1e-300), f"max err {err:.3e} vs scale {scale:.3e}"
    z = ref == 0.0
    if np.any(z):
        assert float(np.max(np.abs(gpu[z]))) <= 1e-6 * max(scale, 1e-300)
    return err / max(scale, 1e-300)


def _points(rng, n, gx, gy, gt, margin=4.0):
    lo = np.array([-margin, -margin, -margin])
    hi = np.array([gx + margin, gy + margin, gt + margin])
    return lo + rng.uniform(0, 1, (n, 3)) * (hi - lo)


def _set(torch, m, pts, base, tuning=None):
    s = m.BinnedSet(m.Desc(**base), len(pts), tuning)
    s.build(torch.from_numpy(np.ascontiguousarray(pts)).cuda())
    return s


def _out(torch, d):
    return torch.full((d["gx"], d["gy"], d["gt"]), float("nan"), dtype=torch.float32, device="cuda")


def _grid_of(d):
    return Grid(gx=d["gx"], gy=d["gy"], gt=d["gt"], hs=d["hs"], ht=d["ht"], sres=d.get("sres", 1.0),
                tres=d.get("tres", 1.0), x0=d.get("x0", 0.0), y0=d.get("y0", 0.0), t0=d.get("t0", 0.0))


def test_bandwidth_sweep_one_set(torch_cuda):
    import paper_1705_09366_amd as m
    torch = torch_cuda
    rng = np.random.default_rng(11)
    base = dict(gx=83, gy=57, gt=45, hs=7.0, ht=5.0)
    pts = _points(rng, 700, 83, 57, 45)
    s = _set(torch, m, pts, base)
    bws = [(7.0, 5.0), (2.5, 1.5), (4.2, 3.7), (6.1, 0.8), (1.1, 4.9)]
    items, plans, descs = [], [], []
    for k, (hs, ht) in enumerate(bws):
        d = dict(gx=83, gy=57, gt=45, hs=hs, ht=ht, flags=4 if k % 2 else 5)
        p = m.Plan(m.Desc(**d))
        plans.append(p)
        descs.append(d)
        items.append(m.Item(plan=p, set=s, out=_out(torch, d),
                            stats=torch.zeros(8, dtype=torch.float64, device="cuda")))
    _say(f"sweep of {len(items)} bandwidths on one set")
    b = m.Batch(items)
    b.run()
    torch.cuda.synchronize()
    for d, it in zip(descs, items):
        ref, _ = oracle.pbsym(pts, _grid_of(d))
        got = it.out.cpu().numpy()
        rel = _check_close(got, ref)
        st = it.stats.cpu().numpy()
        assert st[0] == pytest.approx(float(np.sum(got, dtype=np.float64)), rel=1e-9)
        assert st[3] == 0 and st[1] == 0 and st[2] == 0
        _say(f"hs={d['hs']} ht={d['ht']}: rel err {rel:.2e}")
    # each item alone (a batch of one over the same set) is bitwise the same
    for d, it, p in zip(descs, items, plans):
        alone = m.Item(plan=p, set=s, out=_out(torch, d))
        b1 = m.Batch([alone])
        b1.run()
        torch.cuda.synchronize()
        assert torch.equal(alone.out, it.out)
        b1.close()
    b.close()
    for p in plans:
        p.close()
    s.close()


def test_windows_of_a_base_grid(torch_cuda):
    import paper_1705_09366_amd as m
    torch = torch_cuda
    rng = np.random.default_rng(12)
    base = dict(gx=96, gy=80, gt=48, hs=6.0, ht=4.0, x0=-3.0, y0=2.0, t0=10.0, sres=0.5, tres=2.0)
    n = 900
    pts = np.array([base["x0"], base["y0"], base["t0"]]) + \
        _points(rng, n, 96, 80, 48) * np.array([0.5, 0.5, 2.0])
    s = _set(torch, m, pts, base)
    wins = [(0, 0, 0, 96, 80, 48), (5, 7, 3, 33, 21, 17), (60, 50, 30, 36, 30, 18),
            (95, 79, 47, 1, 1, 1), (17, 0, 16, 40, 80, 16)]
    items, descs = [], []
    for k, (ox, oy, ot, gx, gy, gt) in enumerate(wins):
        d = dict(gx=gx, gy=gy, gt=gt, hs=6.0 - 0.5 * k, ht=4.0 - 0.3 * k, sres=0.5, tres=2.0,
                 x0=base["x0"] + ox * 0.5, y0=base["y0"] + oy * 0.5, t0=base["t0"] + ot * 2.0, flags=4)
        descs.append(d)
        items.append(m.Item(plan=m.Plan(m.Desc(**d)), set=s, out=_out(torch, d), ox=ox, oy=oy, ot=ot,
                            stats=torch.zeros(8, dtype=torch.float64, device="cuda")))
    _say(f"{len(items)} windows")
    b = m.Batch(items)
    b.run()
    torch.cuda.synchronize()
    for d, it in zip(descs, items):
        # the window's estimate divides by the whole set's n
        ref, _ = oracle.pbsym(pts, _grid_of(d))
        got = it.out.cpu().numpy()
        rel = _check_close(got, ref)
        _say(f"window {d['gx']}x{d['gy']}x{d['gt']} at ({d['x0']}, {d['y0']}, {d['t0']}): rel err {rel:.2e}")
    b.close()
    s.close()


def test_mixed_tile_shapes_and_accumulation(torch_cuda):
    import paper_1705_09366_amd as m
    torch = torch_cuda
    rng = np.random.default_rng(13)
    base = dict(gx=70, gy=66, gt=90, hs=5.0, ht=9.0)
    pts = _points(rng, 800, 70, 66, 90)
    s = _set(torch, m, pts, base, m.Tuning(tile_t=64))
    items, descs = [], []
    for k, (tt, flags) in enumerate([(16, 0), (32, 1), (64, 0), (16, 1), (32, 4), (64, 4)]):
        d = dict(gx=70, gy=66, gt=90, hs=5.0 - 0.4 * k, ht=9.0 - k, flags=flags)
        descs.append(d)
        items.append(m.Item(plan=m.Plan(m.Desc(**d), m.Tuning(tile_t=tt)), set=s, out=_out(torch, d)))
    _say("mixed tile_t / Kahan groups")
    b = m.Batch(items)
    b.run()
    torch.cuda.synchronize()
    for d, it in zip(descs, items):
        ref, _ = oracle.pbsym(pts, _grid_of(d))
        _check_close(it.out.cpu().numpy(), ref)
    b.close()
    s.close()


def test_graph_replays_match_eager(torch_cuda):
    import paper_1705_09366_amd as m
    torch = torch_cuda
    rng = np.random.default_rng(14)
    base = dict(gx=64, gy=48, gt=40, hs=5.0, ht=4.0)
    pts = _points(rng, 600, 64, 48, 40)
    s = _set(torch, m, pts, base)
    items = []
    for k in range(3):
        d = dict(gx=64, gy=48, gt=40, hs=5.0 - k, ht=4.0 - k, flags=4)
        items.append(m.Item(plan=m.Plan(m.Desc(**d)), set=s, out=_out(torch, d),
                            stats=torch.zeros(8, dtype=torch.float64, device="cuda")))
    b = m.Batch(items)
    b.run()
    torch.cuda.synchronize()
    ref = [it.out.clone() for it in items]
    ref_st = [it.stats.clone() for it in items]
    b.capture()
    for r in range(3):
        for it in items:
            it.out.fill_(float("nan"))
            it.stats.fill_(-1.0)
        x = torch.randn(1 << 20, device="cuda")
        _ = (x * 2).sum()  # unrelated eager work between replays
        torch.cuda.synchronize()
        _say(f"replay {r}")
        b.replay()
        torch.cuda.synchronize()
        for it, o, st in zip(items, ref, ref_st):
            assert torch.equal(it.out, o)
            assert torch.equal(it.stats, st)
    b.close()
    s.close()


def test_split_hot_tiles_in_a_batch(torch_cuda):
    """A dense pile makes tiles far costlier than their instance's share, so
    they are cut into parts whose partial grids are reduced in order."""
    import paper_1705_09366_amd as m
    torch = torch_cuda
    rng = np.random.default_rng(15)
    base = dict(gx=48, gy=48, gt=40, hs=6.0, ht=5.0)
    pile = np.array([24.0, 24.0, 20.0]) + rng.uniform(0, 1, (40_000, 3))
    spread = _points(rng, 2000, 48, 48, 40)
    pts = np.concatenate([pile, spread])
    s = _set(torch, m, pts, base)
    items, descs = [], []
    for k, flags in enumerate([1 | 4, 4, 1 | 4]):
        d = dict(gx=48, gy=48, gt=40, hs=6.0 - k, ht=5.0 - k, flags=flags)
        descs.append(d)
        items.append(m.Item(plan=m.Plan(m.Desc(**d)), set=s, out=_out(torch, d),
                            stats=torch.zeros(8, dtype=torch.float64, device="cuda")))
    _say("split hot tiles")
    b = m.Batch(items)
    b.run()
    torch.cuda.synchronize()
    cut = []
    for d, it in zip(descs, items):
        ref, _ = oracle.pbsym(pts, _grid_of(d))
        got = it.out.cpu().numpy()
        rel = _check_close(got, ref)
        st = it.stats.cpu().numpy()
        assert st[0] == pytest.approx(float(np.sum(got, dtype=np.float64)), rel=1e-9)
        _say(f"hs={d['hs']} flags={d['flags']}: rel err {rel:.2e}, {int(st[6])} tiles in parts")
        cut.append(int(st[6]))
    # the pile's tiles are cut (their count is reported per grid)
    assert max(cut) > 0
    b.close()
    s.close()


def test_one_gather_launch_for_mixed_variants(torch_cuda):
    """Grids with 16- and 32-row tiles, two-term FP16 and full-cover FP32
    kernels (and an FP32 grid below the full-cover bandwidth), all
    compensated, then all plain, run as one pass: one gather launch.  Every
    grid matches the FP64 oracle; a grid is bitwise the same item run alone
    when neither run cuts one of its tiles; a dense pile makes hot tiles that
    are cut and reduced with their grid's tile height; a graph replay is
    bitwise the eager run."""
    import paper_1705_09366_amd as m
    torch = torch_cuda
    rng = np.random.default_rng(21)
    base = dict(gx=80, gy=72, gt=72, hs=18.0, ht=6.0)
    pile = np.array([40.0, 36.0, 36.0]) + rng.uniform(0, 1, (30_000, 3))
    pts = np.concatenate([pile, _points(rng, 3000, 80, 72, 72)])
    s = _set(torch, m, pts, base, m.Tuning(tile_t=32))
    mixed = [(4.0, 16, 0), (4.0, 32, 0), (16.0, 16, 0), (16.0, 32, 0), (6.0, 32, 1)]  # hs, rows, operand form
    rows16 = [(4.0, 16, 0), (16.0, 16, 0)]  # 16-row grids only: slots still spaced for 32 rows
    for flags, specs in ((1 | 4, mixed), (4, mixed), (1 | 4, rows16)):
        items, descs = [], []
        for hs, tt, form in specs:
            d = dict(gx=80, gy=72, gt=72, hs=hs, ht=5.0, flags=flags)
            descs.append(d)
            items.append(m.Item(plan=m.Plan(m.Desc(**d), m.Tuning(tile_t=tt, operand_form=form)), set=s,
                                out=_out(torch, d), stats=torch.zeros(8, dtype=torch.float64, device="cuda")))
        _say(f"one-launch batch flags={flags}")
        b = m.Batch(items)
        assert b.passes() == 1
        b.run()
        torch.cuda.synchronize()
        cut = []
        for d, it in zip(descs, items):
            ref, _ = oracle.pbsym(pts, _grid_of(d))
            got = it.out.cpu().numpy()
            rel = _check_close(got, ref)
            st = it.stats.cpu().numpy()
            assert st[0] == pytest.approx(float(np.sum(got, dtype=np.float64)), rel=1e-9)
            cut.append(int(st[6]))
            _say(f"hs={d['hs']}: rel err {rel:.2e}, {int(st[6])} tiles in parts")
        assert max(cut) > 0
        for it, d, c in zip(items, descs, cut):
            alone = m.Item(plan=it.plan, set=s, out=_out(torch, d),
                           stats=torch.zeros(8, dtype=torch.float64, device="cuda"))
            ba = m.Batch([alone])
            ba.run()
            torch.cuda.synchronize()
            if c == 0 and int(alone.stats[6].item()) == 0:
                assert torch.equal(alone.out, it.out)
            ba.close()
        ref = [it.out.clone() for it in items]
        b.capture()
        for it in items:
            it.out.fill_(float("nan"))
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        for it, o in zip(items, ref):
            assert torch.equal(it.out, o)
        b.close()
    s.close()


def test_set_counts_culled_and_non_finite(torch_cuda):
    import paper_1705_09366_amd as m
    torch = torch_cuda
    rng = np.random.default_rng(16)
    base = dict(gx=40, gy=30, gt=20, hs=3.0, ht=2.0)
    pts = np.concatenate([_points(rng, 100, 40, 30, 20, margin=0.0),
                          [[-10.0, 5.0, 5.0], [5.0, 45.0, 5.0], [np.nan, 1.0, 1.0]]])
    s = _set(torch, m, pts, base)
    d = dict(base)
    it = m.Item(plan=m.Plan(m.Desc(**d)), set=s, out=_out(torch, d),
                stats=torch.zeros(8, dtype=torch.float64, device="cuda"))
    b = m.Batch([it])
    b.run()
    torch.cuda.synchronize()
    st = it.stats.cpu().numpy()
    assert st[3] == 1 and st[4] == 2
    ref, _ = oracle.pbsym(pts, _grid_of(d))
    _check_close(it.out.cpu().numpy(), ref)
    b.close()
    s.close()
