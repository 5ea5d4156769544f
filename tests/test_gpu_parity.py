"""GPU parity: the HIP path against the FP64 oracle, through the C ABI.

Bar (per run): max |gpu - oracle| <= 1e-5 * max(oracle), FP32 grid compared in
FP64; integer results (evaluation counts, non-finite and culled counters)
exact; repeated runs bit-identical.  Small cases are compared element by
element over several tiles with ragged tails; the full-size workloads are
compared on sampled voxels that the oracle evaluates one by one (Alg. VB) and
through the exact mass identity.
"""
import os
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


def _desc(g, flags=0):
    import paper_1705_09366_amd as m
    return m.Desc(gx=g["gx"], gy=g["gy"], gt=g["gt"], hs=g["hs"], ht=g["ht"],
                  sres=g.get("sres", 1.0), tres=g.get("tres", 1.0), x0=g.get("x0", 0.0),
                  y0=g.get("y0", 0.0), t0=g.get("t0", 0.0), flags=flags)


def _run(torch, pts, g, flags=0, tuning=None, with_stats=True):
    import paper_1705_09366_amd as m
    plan = m.Plan(_desc(g, flags), tuning)
    d = torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float64)).cuda()
    stats = torch.zeros(8, dtype=torch.float64, device="cuda") if with_stats else None
    out = plan(d, stats=stats)
    torch.cuda.synchronize()
    res = out.cpu().numpy()
    st = stats.cpu().numpy() if with_stats else None
    plan.close()
    return res, st


def _check_close(gpu, ref, tol=TOL):
    scale = float(np.max(np.abs(ref)))
    err = float(np.max(np.abs(gpu.astype(np.float64) - ref))) if ref.size else 0.0
    assert err <= tol * max(scale, 1e-300), f"max err {err:.3e} vs scale {scale:.3e}"
    # support: where the oracle is exactly zero the GPU may only hold values
    # that are negligible (rounding at the support boundary)
    z = ref == 0.0
    if np.any(z):
        assert float(np.max(np.abs(gpu[z]))) <= 1e-6 * max(scale, 1e-300)
    return err / max(scale, 1e-300)


def _grid(g):
    return Grid(gx=g["gx"], gy=g["gy"], gt=g["gt"], hs=g["hs"], ht=g["ht"], sres=g.get("sres", 1.0),
                tres=g.get("tres", 1.0), x0=g.get("x0", 0.0), y0=g.get("y0", 0.0), t0=g.get("t0", 0.0))


# --------------------------------------------------------------- small cases
@pytest.mark.parametrize("seed", range(16))
def test_random_small_cases(torch_cuda, seed):
    pts, g = workloads.small_random_case(seed, max_g=70, max_n=400)
    _say(f"random seed={seed} grid={g['gx']}x{g['gy']}x{g['gt']} n={len(pts)}")
    ref, evals = oracle.pbsym(pts, _grid(g))
    gpu, st = _run(torch_cuda, pts, g, flags=4 | 8)
    _check_close(gpu, ref)
    assert int(st[2]) == evals
    assert st[1] == pytest.approx(oracle.exact_mass(pts, _grid(g)), rel=1e-12, abs=1e-300)
    assert st[0] == pytest.approx(ref.sum() * g.get("sres", 1) ** 2 * g.get("tres", 1), rel=1e-6, abs=1e-300)


def test_config0_uniform_full(torch_cuda):
    inst = workloads.config0()
    g = dict(gx=inst.gx, gy=inst.gy, gt=inst.gt, hs=inst.hs, ht=inst.ht)
    _say(f"config0 {inst.name}")
    ref, evals = oracle.pbsym(inst.points, _grid(g))
    gpu, st = _run(torch_cuda, inst.points, g, flags=4 | 8)
    rel = _check_close(gpu, ref)
    _say(f"config0 max rel err {rel:.3e}")
    assert int(st[2]) == evals
    assert st[3] == 0 and st[4] == 0


def test_golden_tiny_case(torch_cuda):
    from tests.test_oracle_pins import _read_golden
    grid, pts, vals, evals = _read_golden()
    g = dict(gx=grid.gx, gy=grid.gy, gt=grid.gt, hs=grid.hs, ht=grid.ht)
    ref = np.zeros((grid.gx, grid.gy, grid.gt))
    for k, v in vals.items():
        ref[k] = v
    gpu, st = _run(torch_cuda, pts, g, flags=8)
    _check_close(gpu, ref)
    assert int(st[2]) == evals


@pytest.mark.parametrize("tuning", [None, (16, 8, 4), (32, 32, 32), (16, 64, 8), (32, 8, 64), (64, 16, 16), (64, 4, 32)])
def test_tunings_agree(torch_cuda, tuning):
    import paper_1705_09366_amd as m
    pts, g = workloads.small_random_case(77, max_g=90, max_n=600)
    g.update(gx=83, gy=57, gt=45)
    tun = m.Tuning(*tuning) if tuning else None
    _say(f"tuning {tuning}")
    ref, _ = oracle.pbsym(pts, _grid(g))
    a, _ = _run(torch_cuda, pts, g, tuning=tun)
    b, _ = _run(torch_cuda, pts, g, tuning=tun)
    assert np.array_equal(a, b)
    _check_close(a, ref)


def test_repeatable_bitwise(torch_cuda):
    inst = workloads.config0()
    g = dict(gx=inst.gx, gy=inst.gy, gt=inst.gt, hs=inst.hs, ht=inst.ht)
    a, _ = _run(torch_cuda, inst.points, g)
    b, _ = _run(torch_cuda, inst.points, g)
    c, _ = _run(torch_cuda, inst.points, g, flags=1)
    d, _ = _run(torch_cuda, inst.points, g, flags=1)
    assert np.array_equal(a, b) and np.array_equal(c, d)


@pytest.mark.parametrize("case", ["corner", "dense", "wide"])
def test_queues_handed_out_without_counters(torch_cuda, case):
    """The gather hands out a queue that fits the grid of workgroups without
    counters (heavy item b to workgroup b; spatial item j after the heavy
    items).  corner: a 96x96x64 grid whose points sit in one corner, so most
    tiles hold no candidate and go through the spatial queue (zeros written);
    dense: every tile of a 128x128x32 grid is heavy (empty spatial queue);
    wide: 2048 tiles, more than the grid of workgroups, so the heavy queue is
    handed out directly and the spatial queue from the counters.  Each is
    compared voxel by voxel with the oracle and repeated bitwise."""
    rng = np.random.default_rng(53)
    if case == "corner":
        g = dict(gx=96, gy=96, gt=64, hs=3.0, ht=2.0)
        pts = rng.uniform(0, 1, (3000, 3)) * [20, 20, 12]
    elif case == "dense":
        g = dict(gx=128, gy=128, gt=32, hs=4.0, ht=3.0)
        pts = rng.uniform(0, 1, (20000, 3)) * [128, 128, 32]
    else:
        g = dict(gx=512, gy=512, gt=64, hs=2.0, ht=2.0)
        pts = np.concatenate([rng.uniform(0, 1, (15000, 3)) * [512, 512, 64],
                              rng.normal([256, 256, 32], [20, 20, 6], (15000, 3)).clip(0, [511, 511, 63])])
    _say(f"queue hand-out case {case}")
    a, st = _run(torch_cuda, pts, g, flags=1 | 4)
    b, _ = _run(torch_cuda, pts, g, flags=1 | 4)
    ref, _ = oracle.pbsym(pts, _grid(g))
    _check_close(a, ref)
    assert np.array_equal(a, b)


# ------------------------------------------------------------- edge cases
def test_single_point_closed_form(torch_cuda):
    g = dict(gx=21, gy=21, gt=15, hs=5.0, ht=4.0)
    pts = np.array([[10.5, 10.5, 7.5]])
    ref, _ = oracle.pbsym(pts, _grid(g))
    gpu, _ = _run(torch_cuda, pts, g)
    _check_close(gpu, ref, tol=2e-7)
    # voxel-centred point: the GPU grid is mirror symmetric bit for bit
    assert np.array_equal(gpu, gpu[::-1, :, :]) and np.array_equal(gpu, gpu[:, :, ::-1])
    assert np.array_equal(gpu, gpu[:, ::-1, :])


def test_all_points_outside(torch_cuda):
    g = dict(gx=40, gy=30, gt=20, hs=3.0, ht=2.0)
    pts = np.array([[-10.0, 5.0, 5.0], [5.0, 45.0, 5.0], [5.0, 5.0, 30.0], [100.0, 100.0, 100.0]])
    gpu, st = _run(torch_cuda, pts, g)
    assert np.all(gpu == 0.0) and not np.any(np.signbit(gpu))
    assert st[4] == 4 and st[3] == 0


def test_non_finite_points(torch_cuda):
    pts, g = workloads.small_random_case(5, max_g=40, max_n=100)
    bad = np.array([[np.nan, 1.0, 1.0], [1.0, np.inf, 1.0], [1.0, 1.0, -np.inf]])
    allp = np.concatenate([pts, bad])
    ref, _ = oracle.pbsym(allp, _grid(g))
    gpu, st = _run(torch_cuda, allp, g)
    _check_close(gpu, ref)
    assert st[3] == 3


def test_tiny_bandwidth_and_tiny_grids(torch_cuda):
    rng = np.random.default_rng(4)
    for g in (dict(gx=1, gy=1, gt=1, hs=0.7, ht=0.6), dict(gx=9, gy=7, gt=3, hs=0.3, ht=0.4),
              dict(gx=5, gy=40, gt=130, hs=2.5, ht=1.1), dict(gx=33, gy=17, gt=5, hs=40.0, ht=9.0)):
        pts = rng.uniform(-2, 1, (50, 3)) * 0 + rng.uniform(0, 1, (50, 3)) * [g["gx"], g["gy"], g["gt"]]
        _say(f"edge grid {g}")
        ref, evals = oracle.pbsym(pts, _grid(g))
        gpu, st = _run(torch_cuda, pts, g, flags=8)
        _check_close(gpu, ref)
        assert int(st[2]) == evals


def test_many_points_in_one_voxel(torch_cuda):
    """A dense pile: 50k points in one voxel; Kahan keeps the error small."""
    rng = np.random.default_rng(9)
    g = dict(gx=48, gy=48, gt=40, hs=6.0, ht=5.0)
    pts = np.array([24.0, 24.0, 20.0]) + rng.uniform(0, 1, (50_000, 3))
    ref, _ = oracle.pbsym(pts, _grid(g))
    plain, _ = _run(torch_cuda, pts, g)
    kahan, _ = _run(torch_cuda, pts, g, flags=1)
    ek = _check_close(kahan, ref)
    _say(f"pile: kahan rel err {ek:.3e}, plain rel err "
         f"{float(np.max(np.abs(plain - ref)) / np.max(ref)):.3e}")


# ------------------------------------------------- full-size workloads, sampled
def _sample_voxels(pts, g, rng, m_near=192, m_rand=64):
    idx = rng.integers(0, len(pts), m_near)
    near = np.floor(pts[idx]).astype(np.int64) + rng.integers(-2, 3, (m_near, 3))
    rand = np.stack([rng.integers(0, g["gx"], m_rand), rng.integers(0, g["gy"], m_rand),
                     rng.integers(0, g["gt"], m_rand)], axis=1)
    v = np.concatenate([near, rand])
    v[:, 0] = np.clip(v[:, 0], 0, g["gx"] - 1)
    v[:, 1] = np.clip(v[:, 1], 0, g["gy"] - 1)
    v[:, 2] = np.clip(v[:, 2], 0, g["gt"] - 1)
    return v


@pytest.mark.parametrize("which,flags", [(1, 4 | 8), (2, 1 | 4 | 8), (2, 4)])
def test_full_size_sampled(torch_cuda, which, flags):
    inst = workloads.config1() if which == 1 else workloads.config2()
    g = dict(gx=inst.gx, gy=inst.gy, gt=inst.gt, hs=inst.hs, ht=inst.ht)
    _say(f"full {inst.name} flags={flags}")
    gpu, st = _run(torch_cuda, inst.points, g, flags=flags)
    rng = np.random.default_rng(100 + which)
    vox = _sample_voxels(inst.points, g, rng)
    ref = oracle.vb_voxels(inst.points, _grid(g), vox)
    got = gpu[vox[:, 0], vox[:, 1], vox[:, 2]].astype(np.float64)
    scale = float(np.max(ref))
    err = float(np.max(np.abs(got - ref))) / scale
    _say(f"full {inst.name} flags={flags}: sampled max rel err {err:.3e}")
    assert err <= TOL
    # mass: FP64 sum of the stored grid vs the per-point separable sums
    if flags & 8:
        m_pts = oracle.exact_mass(inst.points, _grid(g))
        assert st[1] == pytest.approx(m_pts, rel=1e-10)
        assert int(st[2]) == oracle.exact_evals(inst.points, _grid(g))
        assert st[0] == pytest.approx(m_pts, rel=1e-5)
    assert st[3] == 0


@pytest.mark.parametrize("grid,cells", [
    ((64, 80, 40), (16, 8)),       # 8 x 5 x 5 bins (x bins 8 voxels): one 8-bit pass
    ((512, 512, 64), (4, 4)),      # 2^18 bins: 19-bit keys, two 10-bit passes
    ((512, 512, 256), (4, 4)),     # 2^20 bins: 21-bit keys, two 11-bit passes
    ((1024, 1024, 256), (4, 4)),   # 2^22 bins: 23-bit keys, three 8-bit passes
    ((2048, 2048, 68), (4, 4)),    # 4.5M bins with 4-voxel x bins: x bins widen to 8,
                                   # 2.2M bins, 22-bit keys, two 11-bit passes
])
def test_radix_digit_widths(torch_cuda, grid, cells):
    """Small bins force keys of 7 to 23 bits through every digit width of the
    binning sort; the grid is checked on sampled voxels (Alg. VB) and by the
    exact evaluation count."""
    import paper_1705_09366_amd as m
    gx, gy, gt = grid
    rng = np.random.default_rng(31)
    pts = rng.uniform(-2, 1, (20_000, 3)) * 0 + rng.uniform(0, 1, (20_000, 3)) * [gx, gy, gt]
    # bandwidths below a voxel keep the bins at the requested 4 voxels
    g = dict(gx=gx, gy=gy, gt=gt, hs=0.9, ht=0.9)
    _say(f"radix grid {grid} cells {cells}")
    gpu, st = _run(torch_cuda, pts, g, flags=4 | 8, tuning=m.Tuning(32, cells[0], cells[1]))
    vox = _sample_voxels(pts, g, rng, m_near=256, m_rand=64)
    ref = oracle.vb_voxels(pts, _grid(g), vox)
    got = gpu[vox[:, 0], vox[:, 1], vox[:, 2]].astype(np.float64)
    assert float(np.max(np.abs(got - ref))) <= TOL * float(np.max(ref))
    assert int(st[2]) == oracle.exact_evals(pts, _grid(g))
    assert st[0] == pytest.approx(st[1], rel=1e-6)


@pytest.mark.parametrize("n", [3000, 70_000])
def test_one_pass_binning_matches_two_pass(torch_cuda, n):
    """Keys of at most 11 bits take one sort pass, in which the scatter moves
    the records the transform wrote and the bin offsets come from the digit
    totals; finer bins on the same grid take two passes and the offsets and
    records kernel.  The records do not depend on the bins, so the two sets
    hold the same records (as multisets: the bins order them differently),
    and the same number of them (the valid points); the grids from the two
    sets agree with the oracle."""
    import paper_1705_09366_amd as m
    torch = torch_cuda
    g = dict(gx=64, gy=64, gt=32, hs=0.9, ht=0.9)
    rng = np.random.default_rng(47)
    pts = rng.uniform(-0.1, 1.1, (n, 3)) * [g["gx"], g["gy"], g["gt"]]  # some points outside (culled)
    pts[::97] = np.nan
    base = m.Desc(**g)
    rows = []
    for cells in ((16, 16), (4, 4)):  # 8 x 4 x 2 bins (one pass); 16 x 16 x 8 bins (two)
        _say(f"binning n={n} cells {cells}")
        s = m.BinnedSet(base, n, m.Tuning(32, cells[0], cells[1]))
        s.mem = torch.zeros(s.set_bytes + 256, dtype=torch.uint8, device="cuda")
        s.build(torch.from_numpy(np.ascontiguousarray(pts)).cuda())
        torch.cuda.synchronize()
        off = s.device_ptr().value - s.mem.data_ptr()
        r0 = s.set_bytes - (n * 32 + 255) // 256 * 256  # the records follow the bin offsets
        rec = s.mem[off + r0:off + r0 + n * 32].cpu().numpy().reshape(n, 32)
        s.close()
        rec = rec[np.any(rec != 0, axis=1)]  # positions of culled and non-finite points stay zero
        rows.append(rec[np.lexsort(rec.T[::-1])])
    assert rows[0].shape == rows[1].shape and 0 < rows[0].shape[0] < n
    assert np.array_equal(rows[0], rows[1])
    for cells in ((16, 16), (4, 4)):
        gpu, st = _run(torch, pts, g, flags=4 | 8, tuning=m.Tuning(32, cells[0], cells[1]))
        ref, _ = oracle.pbsym(pts, _grid(g))
        _check_close(gpu, ref)
        assert int(st[3]) == len(pts[::97])


@pytest.mark.parametrize("operand_form", [0, 1])
@pytest.mark.parametrize("split_share", [0, 65536])
def test_kahan_modes_identical(torch_cuda, split_share, operand_form):
    """Compensated accumulation with its running pair in registers or in the
    per-workgroup scratch slot performs the same operations: identical bits,
    also for tiles that take many passes (a dense pile) and for split parts
    (FP32 operands; two-term FP16 operands have the scratch form only, which
    a register-form request selects)."""
    import paper_1705_09366_amd as m
    rng = np.random.default_rng(41)
    g = dict(gx=48, gy=48, gt=40, hs=6.0, ht=5.0)
    pile = np.array([24.0, 24.0, 20.0]) + rng.uniform(0, 1, (30_000, 3))
    pts = np.concatenate([pile, rng.uniform(0, 1, (3000, 3)) * [48, 48, 40]])
    res = []
    for mode in (1, 2):
        for tt in (16, 32):
            _say(f"kahan mode {mode} tile_t {tt} split_share {split_share} operand_form {operand_form}")
            out, st = _run(torch_cuda, pts, g, flags=1 | 4,
                           tuning=m.Tuning(tile_t=tt, split_share=split_share, kahan_mode=mode,
                                           operand_form=operand_form))
            res.append((mode, tt, out, st))
    ref, _ = oracle.pbsym(pts, _grid(g))
    for mode, tt, out, st in res:
        _check_close(out, ref)
    for tt in (16, 32):
        a = [r for r in res if r[1] == tt]
        assert np.array_equal(a[0][2], a[1][2]) and np.array_equal(a[0][3], a[1][3])


@pytest.mark.parametrize("tuning", [(16, 0), (32, 0), (16, 1), (32, 1), (16, 2), (32, 2), (64, 0)])
def test_large_bandwidth_full_cover(torch_cuda, tuning):
    """Discs much larger than a tile take the full-cover path (Ks separable in
    x and y over the whole tile); checked against the oracle with clustered
    points, ragged grid edges, a non-unit voxel and an origin."""
    import paper_1705_09366_amd as m
    tt, kmode = tuning
    rng = np.random.default_rng(51)
    g = dict(gx=75, gy=61, gt=37, hs=40.0, ht=7.0, sres=2.0, tres=1.5, x0=-10.0, y0=4.0, t0=100.0)
    centre = np.array([g["x0"] + 70.0, g["y0"] + 60.0, g["t0"] + 25.0])
    pts = np.concatenate([centre + rng.normal(0, 6.0, (1500, 3)),
                          np.array([g["x0"], g["y0"], g["t0"]]) + rng.uniform(0, 1, (1500, 3))
                          * [75 * 2.0, 61 * 2.0, 37 * 1.5]])
    flags = (1 if kmode else 0) | 4 | 8
    _say(f"full cover tile_t={tt} kahan_mode={kmode}")
    ref, evals = oracle.pbsym(pts, _grid(g))
    gpu, st = _run(torch_cuda, pts, g, flags=flags, tuning=m.Tuning(tile_t=tt, kahan_mode=kmode))
    _check_close(gpu, ref)
    assert int(st[2]) == evals
    assert st[0] == pytest.approx(st[1], rel=1e-6)
