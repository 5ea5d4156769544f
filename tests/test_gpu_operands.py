"""GPU parity of the gather's two matrix-core operand forms against the FP64
oracle, through the C ABI: two FP16 terms per operand (hi + lo, the default
where the gather has that form: one bandwidth pair, no full-cover path, 16-
or 32-row tiles, every kernel pair) and FP32 (tuning operand_form = 1).

Both forms meet the bar of every other path, max |gpu - oracle| <= 1e-5
max(oracle).  Because every product in the sum is non-negative, the
two-term form also meets a per-voxel bound: each operand keeps 22
significant bits (truncation error below 2^-21 of its value, or below 2^-24
absolute where lo falls in FP16's subnormal range) and lo*lo is dropped
(below 2^-20 of the product), so each product is low by less than 2^-19 of
itself, each voxel likewise, plus the FP32 accumulation error and the
subnormal terms (at most 2^-24 per operand, far below 2e-7 of the largest
voxel); with compensated accumulation the test asserts |gpu - oracle| <=
4e-6 |oracle| + 2e-7 max(oracle) voxel by voxel.
Lists of every length modulo the 32-point group (the padded tail) and dense
piles that take many matrix-core phases are covered; a batch mixing both
forms and the full-cover path gives each grid the bits it has alone.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads
from oracle import Grid

pytestmark = pytest.mark.gpu

TOL = 1e-5
REL_VOXEL = 4e-6
ABS_VOXEL = 2e-7


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


def _grid(g):
    return Grid(gx=g["gx"], gy=g["gy"], gt=g["gt"], hs=g["hs"], ht=g["ht"], sres=g.get("sres", 1.0),
                tres=g.get("tres", 1.0), x0=g.get("x0", 0.0), y0=g.get("y0", 0.0), t0=g.get("t0", 0.0))


def _desc(g, flags):
    import paper_1705_09366_amd as m
    return m.Desc(gx=g["gx"], gy=g["gy"], gt=g["gt"], hs=g["hs"], ht=g["ht"], sres=g.get("sres", 1.0),
                  tres=g.get("tres", 1.0), x0=g.get("x0", 0.0), y0=g.get("y0", 0.0), t0=g.get("t0", 0.0),
                  flags=flags)


def _run(torch, pts, g, flags, tuning):
    import paper_1705_09366_amd as m
    plan = m.Plan(_desc(g, flags), tuning)
    st = torch.zeros(8, dtype=torch.float64, device="cuda")
    out = plan(torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float64)).cuda(), stats=st)
    torch.cuda.synchronize()
    res, s = out.cpu().numpy(), st.cpu().numpy()
    plan.close()
    return res, s


def _check(gpu, ref, per_voxel):
    scale = float(np.max(np.abs(ref))) if ref.size else 0.0
    d = np.abs(gpu.astype(np.float64) - ref)
    err = float(np.max(d)) if ref.size else 0.0
    assert err <= TOL * max(scale, 1e-300), f"max err {err:.3e} vs scale {scale:.3e}"
    if per_voxel and ref.size:
        bound = REL_VOXEL * np.abs(ref) + ABS_VOXEL * scale
        worst = float(np.max(d - bound))
        assert worst <= 0.0, f"per-voxel bound exceeded by {worst:.3e} (scale {scale:.3e})"
    return err / max(scale, 1e-300)


@pytest.mark.parametrize("form", [0, 1], ids=["fp16x2", "fp32"])
@pytest.mark.parametrize("seed", range(8))
def test_random_cases(torch_cuda, seed, form):
    import paper_1705_09366_amd as m
    pts, g = workloads.small_random_case(2100 + seed, max_g=80, max_n=900)
    tt = (16, 32)[seed % 2]
    _say(f"operand_form={form} seed={seed} tile_t={tt} grid={g['gx']}x{g['gy']}x{g['gt']} n={len(pts)} "
         f"hv={g['hs'] / g['sres']:.2f}")
    ref, evals = oracle.pbsym(pts, _grid(g))
    gpu, st = _run(torch_cuda, pts, g, 1 | 4 | 8, m.Tuning(tile_t=tt, operand_form=form))
    _check(gpu, ref, per_voxel=True)
    assert int(st[2]) == evals
    assert st[0] == pytest.approx(st[1], rel=1e-5, abs=1e-300)


@pytest.mark.parametrize("form", [0, 1], ids=["fp16x2", "fp32"])
@pytest.mark.parametrize("kernel", [1, 2, 3], ids=["quartic", "gaussian", "printed"])
def test_other_pairs_both_forms(torch_cuda, kernel, form):
    """The other kernel pairs (operands up to 16 for the printed pair, exact
    support tests near the boundary for the Gaussian and printed pairs) in
    both forms, with the per-voxel bound."""
    import paper_1705_09366_amd as m
    for seed in range(3):
        pts, g = workloads.small_random_case(2300 + 10 * kernel + seed, max_g=70, max_n=700)
        tt = (16, 32)[seed % 2]
        grid = Grid(gx=g["gx"], gy=g["gy"], gt=g["gt"], hs=g["hs"], ht=g["ht"], sres=g["sres"], tres=g["tres"],
                    x0=g["x0"], y0=g["y0"], t0=g["t0"], kernel=kernel)
        ref, evals = oracle.pbsym(pts, grid)
        _say(f"pair {kernel} operand_form={form} seed={seed} tile_t={tt} n={len(pts)}")
        gpu, st = _run(torch_cuda, pts, g, 1 | 4 | 8 | m.kernel_flag(kernel), m.Tuning(tile_t=tt, operand_form=form))
        _check(gpu, ref, per_voxel=True)
        assert int(st[2]) == evals


@pytest.mark.parametrize("hv,tv", [(0.3, 0.4), (0.75, 9.0), (3.3, 0.6), (13.9, 2.2), (9.5, 15.0)])
def test_disc_and_window_extremes(torch_cuda, hv, tv):
    """Discs from a fraction of a voxel to just below the full-cover path,
    windows from under one row to longer than a tile."""
    import paper_1705_09366_amd as m
    rng = np.random.default_rng(int(hv * 100 + tv))
    g = dict(gx=53, gy=47, gt=70, hs=hv * 0.5, ht=tv * 2.0, sres=0.5, tres=2.0, x0=3.0, y0=-1.0, t0=5.0)
    lo = np.array([g["x0"], g["y0"], g["t0"]])
    ext = np.array([53 * 0.5, 47 * 0.5, 70 * 2.0])
    pts = lo - 2.0 + rng.uniform(0, 1, (2500, 3)) * (ext + 4.0)
    ref, evals = oracle.pbsym(pts, _grid(g))
    for tt in (16, 32):
        gpu, st = _run(torch_cuda, pts, g, 1 | 8, m.Tuning(tile_t=tt))
        rel = _check(gpu, ref, per_voxel=True)
        _say(f"hv={hv} tv={tv} tile_t={tt}: max rel err {rel:.2e}")
        assert int(st[2]) == evals


def test_every_tail_length(torch_cuda):
    """One 16 x 16 column block holding k points for k = 1..70: every wave's
    list ends at each position of its last 32-point group."""
    import paper_1705_09366_amd as m
    rng = np.random.default_rng(7)
    g = dict(gx=16, gy=16, gt=32, hs=3.5, ht=2.5)
    for k in range(1, 71):
        pts = rng.uniform([0.0, 0.0, 0.0], [16.0, 16.0, 32.0], (k, 3))
        ref, _ = oracle.pbsym(pts, _grid(g))
        for tt in (16, 32):
            gpu, _ = _run(torch_cuda, pts, g, 1, m.Tuning(tile_t=tt))
            _check(gpu, ref, per_voxel=True)
    _say("tails 1..70 checked")


@pytest.mark.parametrize("tt", [16, 32])
def test_dense_pile_many_phases(torch_cuda, tt):
    """40,000 points within one voxel plus a background: the pile's tiles take
    dozens of matrix-core phases; plain and compensated sums against the
    oracle, the compensated one also voxel by voxel."""
    import paper_1705_09366_amd as m
    rng = np.random.default_rng(19)
    g = dict(gx=40, gy=36, gt=48, hs=4.5, ht=3.5)
    pile = np.array([20.0, 18.0, 24.0]) + rng.uniform(0, 1, (40_000, 3))
    pts = np.concatenate([pile, rng.uniform(0, 1, (4000, 3)) * [40, 36, 48]])
    ref, _ = oracle.pbsym(pts, _grid(g))
    for flags in (1 | 8, 8):
        gpu, st = _run(torch_cuda, pts, g, flags, m.Tuning(tile_t=tt, split_share=65536))
        rel = _check(gpu, ref, per_voxel=bool(flags & 1))
        _say(f"pile tile_t={tt} flags={flags}: max rel err {rel:.2e}")


def test_forms_agree_on_uniform_10k(torch_cuda):
    """The two forms on the uniform-10k workload: both within the bar of the
    oracle on sampled voxels, and within the per-voxel bound of each other."""
    import paper_1705_09366_amd as m
    inst = workloads.config0()
    g = dict(gx=inst.gx, gy=inst.gy, gt=inst.gt, hs=inst.hs, ht=inst.ht)
    a, sa = _run(torch_cuda, inst.points, g, 1 | 8, m.Tuning(operand_form=0))
    b, sb = _run(torch_cuda, inst.points, g, 1 | 8, m.Tuning(operand_form=1))
    assert sa[2] == sb[2]
    d = np.abs(a.astype(np.float64) - b.astype(np.float64))
    assert float(np.max(d - (REL_VOXEL * np.abs(b) + ABS_VOXEL * float(np.max(b))))) <= 0.0
    rng = np.random.default_rng(3)
    vox = np.stack([rng.integers(0, g["gx"], 400), rng.integers(0, g["gy"], 400),
                    rng.integers(0, g["gt"], 400)], 1)
    ref = oracle.vb_voxels(inst.points, _grid(g), vox)
    for x in (a, b):
        got = x[vox[:, 0], vox[:, 1], vox[:, 2]].astype(np.float64)
        assert float(np.max(np.abs(got - ref))) <= TOL * float(np.max(ref))


def test_batch_mixing_forms_keeps_each_grids_bits(torch_cuda):
    """A batch whose grids take two-term FP16 operands, FP32 operands and the
    full-cover path: each grid is bitwise the grid of the same item alone and
    within the bar of the oracle."""
    import paper_1705_09366_amd as m
    torch = torch_cuda
    rng = np.random.default_rng(29)
    base = dict(gx=72, gy=60, gt=44, hs=18.0, ht=6.0)
    pts = rng.uniform(0, 1, (1200, 3)) * [72, 60, 44]
    s = m.BinnedSet(m.Desc(**base), len(pts), None)
    s.build(torch.from_numpy(np.ascontiguousarray(pts)).cuda())
    specs = [(4.0, 3.0, 0, 5), (4.0, 3.0, 1, 5), (18.0, 6.0, 0, 5), (7.5, 2.0, 0, 4), (7.5, 2.0, 1, 4),
             (2.0, 5.5, 0, 1)]
    items, descs, plans = [], [], []
    for hs, ht, form, flags in specs:
        d = dict(gx=72, gy=60, gt=44, hs=hs, ht=ht, flags=flags)
        p = m.Plan(m.Desc(**d), m.Tuning(tile_t=32, operand_form=form))
        plans.append(p)
        descs.append(d)
        items.append(m.Item(plan=p, set=s, out=torch.full((72, 60, 44), float("nan"), dtype=torch.float32,
                                                          device="cuda")))
    _say(f"batch of {len(items)} mixing operand forms and the full-cover path")
    b = m.Batch(items)
    b.run()
    torch.cuda.synchronize()
    for (hs, ht, form, flags), d, it, p in zip(specs, descs, items, plans):
        ref, _ = oracle.pbsym(pts, Grid(gx=72, gy=60, gt=44, hs=hs, ht=ht))
        _check(it.out.cpu().numpy(), ref, per_voxel=bool(flags & 1))
        alone = m.Item(plan=p, set=s, out=torch.full((72, 60, 44), float("nan"), dtype=torch.float32,
                                                     device="cuda"))
        b1 = m.Batch([alone])
        b1.run()
        torch.cuda.synchronize()
        assert torch.equal(alone.out, it.out), (hs, ht, form)
        b1.close()
    b.close()
    for p in plans:
        p.close()
    s.close()
