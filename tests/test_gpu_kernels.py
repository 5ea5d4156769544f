"""GPU parity of the kernel pairs (Epanechnikov, quartic, truncated Gaussian,
the pair as printed) and of corner sampling against the FP64 oracle,
through the C ABI.

Bar: max |gpu - oracle| <= 1e-5 * max(oracle) element by element on small
cases with ragged grids, and on sampled voxels (Alg. VB) at the clustered
1M-point size; exact evaluation counts and per-point FP64 mass; corner
sampling equal, bit for bit, to centre sampling of the grid shifted by half
a voxel.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads
from oracle import Grid

pytestmark = pytest.mark.gpu

TOL = 1e-5
PAIRS = (0, 1, 2, 3)
NAMES = {0: "epanechnikov", 1: "quartic", 2: "gaussian", 3: "printed"}


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


def _grid(g, kernel, corner):
    return Grid(gx=g["gx"], gy=g["gy"], gt=g["gt"], hs=g["hs"], ht=g["ht"], sres=g.get("sres", 1.0),
                tres=g.get("tres", 1.0), x0=g.get("x0", 0.0), y0=g.get("y0", 0.0), t0=g.get("t0", 0.0),
                kernel=kernel, corner=corner)


def _run(torch, pts, g, kernel, corner, flags=0, tuning=None):
    import paper_1705_09366_amd as m
    fl = flags | m.kernel_flag(kernel) | (m.FLAG_CORNER if corner else 0)
    d = m.Desc(gx=g["gx"], gy=g["gy"], gt=g["gt"], hs=g["hs"], ht=g["ht"], sres=g.get("sres", 1.0),
               tres=g.get("tres", 1.0), x0=g.get("x0", 0.0), y0=g.get("y0", 0.0), t0=g.get("t0", 0.0), flags=fl)
    plan = m.Plan(d, tuning)
    st = torch.zeros(8, dtype=torch.float64, device="cuda")
    out = plan(torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float64)).cuda(), stats=st)
    torch.cuda.synchronize()
    res, s = out.cpu().numpy(), st.cpu().numpy()
    plan.close()
    return res, s


def _check_close(gpu, ref, tol=TOL):
    scale = float(np.max(np.abs(ref))) if ref.size else 0.0
    err = float(np.max(np.abs(gpu.astype(np.float64) - ref))) if ref.size else 0.0
    assert err <= tol * max(scale, 1e-300), f"max err {err:.3e} vs scale {scale:.3e}"
    z = ref == 0.0
    if np.any(z):
        assert float(np.max(np.abs(gpu[z]))) <= 1e-6 * max(scale, 1e-300)
    return err / max(scale, 1e-300)


@pytest.mark.parametrize("kernel", PAIRS, ids=[NAMES[k] for k in PAIRS])
@pytest.mark.parametrize("seed", range(5))
def test_random_small_cases(torch_cuda, kernel, seed):
    import paper_1705_09366_amd as m
    pts, g = workloads.small_random_case(1700 + 10 * kernel + seed, max_g=70, max_n=400)
    corner = bool(seed & 1)
    flags = [4 | 8, 1 | 4 | 8][seed % 2]
    tt = [16, 32, 64][seed % 3]
    _say(f"pair {NAMES[kernel]} seed={seed} corner={corner} flags={flags} tile_t={tt} "
         f"grid={g['gx']}x{g['gy']}x{g['gt']} n={len(pts)}")
    grid = _grid(g, kernel, corner)
    ref, evals = oracle.pbsym(pts, grid)
    gpu, st = _run(torch_cuda, pts, g, kernel, corner, flags, m.Tuning(tile_t=tt))
    _check_close(gpu, ref)
    assert int(st[2]) == evals
    assert st[1] == pytest.approx(oracle.exact_mass(pts, grid), rel=1e-12, abs=1e-300)
    assert st[0] == pytest.approx(st[1], rel=1e-5, abs=1e-300)


@pytest.mark.parametrize("kernel", PAIRS, ids=[NAMES[k] for k in PAIRS])
def test_corner_is_half_voxel_shift_bitwise(torch_cuda, kernel):
    rng = np.random.default_rng(23)
    pts = np.round(rng.uniform(-3, 70, (3000, 3)) * 64) / 64
    g = dict(gx=67, gy=61, gt=45, hs=5.25, ht=4.5, sres=1.0, tres=1.0, x0=1.5, y0=-2.0, t0=6.0)
    a, _ = _run(torch_cuda, pts, g, kernel, True)
    shifted = {**g, "x0": g["x0"] - 0.5, "y0": g["y0"] - 0.5, "t0": g["t0"] - 0.5}
    b, _ = _run(torch_cuda, pts, shifted, kernel, False)
    assert np.array_equal(a, b)
    ref, _ = oracle.pbsym(pts, _grid(g, kernel, True))
    _check_close(a, ref)


@pytest.mark.parametrize("kernel", (1, 2, 3), ids=["quartic", "gaussian", "printed"])
def test_large_bandwidth_and_dense_pile(torch_cuda, kernel):
    """Discs larger than a tile (no full-cover path for these pairs) and a
    pile of points in one voxel with compensation."""
    rng = np.random.default_rng(31 + kernel)
    g = dict(gx=75, gy=61, gt=37, hs=40.0, ht=7.0, sres=2.0, tres=1.5, x0=-10.0, y0=4.0, t0=100.0)
    centre = np.array([g["x0"] + 70.0, g["y0"] + 60.0, g["t0"] + 25.0])
    pts = np.concatenate([centre + rng.normal(0, 6.0, (1500, 3)), centre + rng.uniform(0, 1, (8000, 3))])
    ref, evals = oracle.pbsym(pts, _grid(g, kernel, False))
    gpu, st = _run(torch_cuda, pts, g, kernel, False, 1 | 8)
    rel = _check_close(gpu, ref)
    _say(f"pair {NAMES[kernel]} large bandwidth + pile: max rel err {rel:.3e}")
    assert int(st[2]) == evals


def _sample_voxels(pts, g, rng, m_near=160, m_rand=48):
    idx = rng.integers(0, len(pts), m_near)
    near = np.floor(pts[idx]).astype(np.int64) + rng.integers(-2, 3, (m_near, 3))
    rand = np.stack([rng.integers(0, g["gx"], m_rand), rng.integers(0, g["gy"], m_rand),
                     rng.integers(0, g["gt"], m_rand)], axis=1)
    v = np.concatenate([near, rand])
    for a, k in enumerate(("gx", "gy", "gt")):
        v[:, a] = np.clip(v[:, a], 0, g[k] - 1)
    return v


@pytest.mark.parametrize("kernel", (1, 2, 3), ids=["quartic", "gaussian", "printed"])
def test_clustered_1m_sampled(torch_cuda, kernel):
    inst = workloads.config1()
    g = dict(gx=inst.gx, gy=inst.gy, gt=inst.gt, hs=inst.hs, ht=inst.ht)
    _say(f"pair {NAMES[kernel]} full {inst.name}")
    gpu, st = _run(torch_cuda, inst.points, g, kernel, False, 1 | 4 | 8)
    grid = _grid(g, kernel, False)
    vox = _sample_voxels(inst.points, g, np.random.default_rng(500 + kernel))
    ref = oracle.vb_voxels(inst.points, grid, vox)
    got = gpu[vox[:, 0], vox[:, 1], vox[:, 2]].astype(np.float64)
    err = float(np.max(np.abs(got - ref))) / float(np.max(ref))
    _say(f"pair {NAMES[kernel]} full: sampled max rel err {err:.3e}")
    assert err <= TOL
    m_pts = oracle.exact_mass(inst.points, grid)
    assert st[1] == pytest.approx(m_pts, rel=1e-10)
    assert st[0] == pytest.approx(m_pts, rel=1e-5)
    assert int(st[2]) == oracle.exact_evals(inst.points, grid)


@pytest.mark.parametrize("kernel", PAIRS, ids=[NAMES[k] for k in PAIRS])
def test_boundary_pairs(torch_cuda, kernel):
    """Events on voxel centres and quarter offsets with integer bandwidths put
    many (voxel, event) pairs exactly on the support boundaries (3-4-5
    distances, time offsets equal to ht): membership must match the oracle
    there, which matters for the pairs that are not zero on the boundary."""
    rng = np.random.default_rng(71)
    g = dict(gx=48, gy=44, gt=30, hs=5.0, ht=4.0)
    centres = rng.integers(0, [48, 44, 30], (2500, 3)) + 0.5
    quarters = rng.integers(0, [48, 44, 30], (1500, 3)) + rng.integers(0, 4, (1500, 3)) * 0.25
    pts = np.concatenate([centres, quarters])
    grid = _grid(g, kernel, False)
    ref, evals = oracle.pbsym(pts, grid)
    gpu, st = _run(torch_cuda, pts, g, kernel, False, 1 | 8)
    rel = _check_close(gpu, ref)
    _say(f"pair {NAMES[kernel]} boundary pairs: max rel err {rel:.3e}")
    assert int(st[2]) == evals
