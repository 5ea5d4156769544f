"""Pins for the FP64 oracle: checks against facts other than the oracle itself.

Every pin below is chosen so that a plausible mistake in the oracle (a dropped
normalisation constant, a wrong sign or index, a transposed axis, an
off-by-one loop bound, a wrong support test) fails at least one of them:

* library routine: with all events at one time (or one place), the estimator
  factorises into a 2-D (or 1-D) Epanechnikov KDE times a single kernel; both
  factors are checked against scikit-learn's KernelDensity;
* brute force: Alg. VB written separately in numpy agrees with Alg. PB-SYM;
* closed form: one event at a voxel centre, exact rationals times 1/pi;
* exact lattice sums and the continuum limit of the total mass (the kernels
  integrate to one);
* invariants: mirror symmetry, superposition, translation, zero outside the
  cylinders, thread-count independence, non-finite events.
"""
import math
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import Grid
from workloads import small_random_case


def _rel_err(a, b):
    scale = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / scale)


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("seed", range(12))
def test_pbsym_matches_numpy_vb(seed):
    pts, g = small_random_case(seed, max_g=24, max_n=120)
    grid = Grid(**g)
    f, evals = oracle.pbsym(pts, grid, nthreads=3)
    ref = oracle.vb_grid_numpy(pts, grid)
    assert _rel_err(f, ref) <= 1e-13
    # pairs counted by PB-SYM == pairs passing both tests in the brute force
    assert evals == oracle.exact_evals(pts, grid)


def test_vb_voxels_matches_grid():
    pts, g = small_random_case(99, max_g=20, max_n=80)
    grid = Grid(**g)
    f, _ = oracle.pbsym(pts, grid)
    rng = np.random.default_rng(5)
    vox = np.stack([rng.integers(0, grid.gx, 50), rng.integers(0, grid.gy, 50),
                    rng.integers(0, grid.gt, 50)], axis=1)
    v = oracle.vb_voxels(pts, grid, vox)
    ref = f[vox[:, 0], vox[:, 1], vox[:, 2]]
    assert np.max(np.abs(v - ref)) <= 1e-13 * max(np.max(np.abs(f)), 1e-300)


# ------------------------------------------------------------ library routine
def test_spatial_factor_is_sklearn_2d_epanechnikov():
    """All events at the same time t*: f(x,y,t) = KDE2(x,y) * kt((t-t*)/ht)/ht
    where KDE2 is the 2-D Epanechnikov KDE with bandwidth hs."""
    KernelDensity = pytest.importorskip("sklearn.neighbors").KernelDensity
    rng = np.random.default_rng(11)
    hs, ht = 4.37, 2.9
    grid = Grid(gx=30, gy=26, gt=9, hs=hs, ht=ht, x0=-1.25, y0=2.5, t0=0.0)
    n = 200
    tstar = 4.5  # centre of row T = 4
    pts = np.stack([rng.uniform(-4, 32, n), rng.uniform(0, 32, n), np.full(n, tstar)], axis=1)
    f, _ = oracle.pbsym(pts, grid)
    xs = grid.x0 + np.arange(grid.gx) + 0.5
    ys = grid.y0 + np.arange(grid.gy) + 0.5
    q = np.stack(np.meshgrid(xs, ys, indexing="ij"), axis=-1).reshape(-1, 2)
    kde = KernelDensity(kernel="epanechnikov", bandwidth=hs, rtol=0.0, atol=0.0).fit(pts[:, :2])
    kde2 = np.exp(kde.score_samples(q)).reshape(grid.gx, grid.gy)
    kde1 = KernelDensity(kernel="epanechnikov", bandwidth=ht, rtol=0.0, atol=0.0).fit([[tstar]])
    ts = (np.arange(grid.gt) + 0.5).reshape(-1, 1)
    ktt = np.exp(kde1.score_samples(ts))  # = kt((t - t*)/ht)/ht
    ref = kde2[:, :, None] * ktt[None, None, :]
    assert _rel_err(f, ref) <= 1e-12


def test_temporal_factor_is_sklearn_1d_epanechnikov():
    """All events at one place: f(x,y,t) = ks((x-x*)/hs,(y-y*)/hs)/hs^2 * KDE1(t)."""
    KernelDensity = pytest.importorskip("sklearn.neighbors").KernelDensity
    rng = np.random.default_rng(12)
    hs, ht = 3.3, 5.61
    grid = Grid(gx=11, gy=9, gt=70, hs=hs, ht=ht, t0=-3.0)
    n = 150
    xs, ys = 5.5, 4.5
    pts = np.stack([np.full(n, xs), np.full(n, ys), rng.uniform(-10, 75, n)], axis=1)
    f, _ = oracle.pbsym(pts, grid)
    ts = (grid.t0 + np.arange(grid.gt) + 0.5).reshape(-1, 1)
    kde = KernelDensity(kernel="epanechnikov", bandwidth=ht, rtol=0.0, atol=0.0).fit(pts[:, 2:3])
    kde1 = np.exp(kde.score_samples(ts))
    cx = (np.arange(grid.gx) + 0.5)[:, None]
    cy = (np.arange(grid.gy) + 0.5)[None, :]
    k2 = KernelDensity(kernel="epanechnikov", bandwidth=hs, rtol=0.0, atol=0.0).fit([[xs, ys]])
    q = np.stack(np.broadcast_arrays(cx, cy), axis=-1).reshape(-1, 2)
    ksx = np.exp(k2.score_samples(q)).reshape(grid.gx, grid.gy)  # = ks(.)/hs^2
    ref = ksx[:, :, None] * kde1[None, None, :]
    assert _rel_err(f, ref) <= 1e-12


# ----------------------------------------------------------------- closed form
def _single_point_exact(hs, ht, a, b, k):
    """f * pi for one event at a voxel centre, offset (a, b, k) voxels, unit
    voxels: (2 * 3/4) (1 - (a^2+b^2)/hs^2) (1 - k^2/ht^2) / (hs^2 ht), zero off
    the support (strict in space, and zero on |k| = ht in time anyway)."""
    hs, ht = Fraction(hs), Fraction(ht)
    r2 = Fraction(a * a + b * b)
    if r2 >= hs * hs or abs(Fraction(k)) > ht:
        return Fraction(0)
    return Fraction(3, 2) * (1 - r2 / (hs * hs)) * (1 - Fraction(k * k) / (ht * ht)) / (hs * hs * ht)


@pytest.mark.parametrize("hs,ht", [(5, 4), (10, 7), (3, 2), (Fraction(7, 2), Fraction(5, 2))])
def test_single_point_closed_form(hs, ht):
    H = int(math.ceil(hs)) + 2
    Tt = int(math.ceil(ht)) + 2
    grid = Grid(gx=2 * H + 1, gy=2 * H + 1, gt=2 * Tt + 1, hs=float(hs), ht=float(ht))
    pts = np.array([[H + 0.5, H + 0.5, Tt + 0.5]])
    f, evals = oracle.pbsym(pts, grid)
    cnt = 0
    for a in range(-H, H + 1):
        for b in range(-H, H + 1):
            for k in range(-Tt, Tt + 1):
                ex = _single_point_exact(hs, ht, a, b, k)
                assert abs(f[H + a, H + b, Tt + k] * math.pi - float(ex)) <= 1e-15 * (1 + float(ex))
                if a * a + b * b < hs * hs and abs(k) <= ht:
                    cnt += 1
    assert evals == cnt


def test_single_point_peak_values():
    """Peak 3/(2 pi hs^2 ht) and a few off-centre values at hs=5, ht=4."""
    grid = Grid(gx=13, gy=13, gt=11, hs=5.0, ht=4.0)
    f, _ = oracle.pbsym(np.array([[6.5, 6.5, 5.5]]), grid)
    assert f[6, 6, 5] == pytest.approx(3.0 / (2.0 * math.pi * 25.0 * 4.0), rel=1e-15)
    assert f[7, 6, 5] == pytest.approx(4.583662361046585e-3, rel=1e-14)
    assert f[9, 8, 6] == pytest.approx(2.148591731740587e-3, rel=1e-14)
    assert f[6, 10, 8] == pytest.approx(7.520071061092056e-4, rel=1e-14)
    assert f[9, 10, 5] == 0.0 and f[6, 6, 9] == 0.0  # on the support boundary


# ------------------------------------------------------- mass: lattice sums
@pytest.mark.parametrize("H,expect", [(5, Fraction(973, 25)), (10, Fraction(3922, 25)),
                                      (50, Fraction(490868, 125))])
def test_lattice_sum_disc(H, expect):
    """One event at a voxel centre with integer hs = H: the in-disc sum of
    (1 - r^2/H^2) over the integer lattice is a known rational, so
    Ss = (2/pi) * that sum."""
    grid = Grid(gx=2 * H + 3, gy=2 * H + 3, gt=3, hs=float(H), ht=1.0)
    Ss, St, cs, ct = oracle.point_sums(np.array([[H + 1.5, H + 1.5, 1.5]]), grid)
    assert Ss[0] == pytest.approx(2.0 / math.pi * float(expect), rel=1e-13)
    # lattice points strictly inside the disc of radius H
    cnt = sum(1 for a in range(-H, H + 1) for b in range(-H, H + 1) if a * a + b * b < H * H)
    assert cs[0] == cnt


@pytest.mark.parametrize("Ht", [4, 7, 30])
def test_lattice_sum_window(Ht):
    """Integer ht = Ht, event at a row centre: sum_k (3/4)(1 - k^2/Ht^2) over
    |k| <= Ht equals Ht (1 - 1/(4 Ht^2)) * ... exactly (3/4)(2Ht+1) -
    (3/4)(Ht+1)(2Ht+1)/(3Ht); the ratio St/ht is 1 - 1/(4 Ht^2)."""
    grid = Grid(gx=3, gy=3, gt=2 * Ht + 5, hs=1.0, ht=float(Ht))
    _, St, _, ct = oracle.point_sums(np.array([[1.5, 1.5, Ht + 2.5]]), grid)
    assert St[0] / Ht == pytest.approx(1.0 - 1.0 / (4.0 * Ht * Ht), rel=1e-14)
    assert ct[0] == 2 * Ht + 1


def test_mass_identity_pbsym_vs_point_sums():
    """Sum of the grid times voxel volume equals sum_i Ss St / (n hs^2 ht) for
    any placement, clipped or not."""
    for seed in range(6):
        pts, g = small_random_case(200 + seed, max_g=30, max_n=200)
        grid = Grid(**g)
        f, _ = oracle.pbsym(pts, grid)
        m_grid = f.sum() * grid.sres ** 2 * grid.tres
        m_pts = oracle.exact_mass(pts, grid)
        assert m_grid == pytest.approx(m_pts, rel=1e-12, abs=1e-300)


def test_mass_continuum_limit():
    """Events uniform within interior voxels: the expected mass of a Riemann
    sum over a random offset is the kernel integral, i.e. exactly 1.  The
    sample mean over many events must be 1 within a few standard errors; a
    dropped or wrong normalisation constant misses by far more."""
    rng = np.random.default_rng(3)
    hs, ht = 4.3, 3.2
    grid = Grid(gx=64, gy=64, gt=40, hs=hs, ht=ht)
    n = 4000
    pts = np.stack([rng.uniform(10, 54, n), rng.uniform(10, 54, n), rng.uniform(8, 32, n)], axis=1)
    Ss, St, _, _ = oracle.point_sums(pts, grid)
    m = Ss * St / (hs * hs * ht)
    se = m.std(ddof=1) / math.sqrt(n)
    assert abs(m.mean() - 1.0) < max(5 * se, 1e-6)
    assert m.std() < 0.05  # a single Riemann sum is already close to 1


# ----------------------------------------------------------------- invariants
def test_mirror_symmetry_voxel_centred():
    grid = Grid(gx=21, gy=21, gt=15, hs=6.3, ht=4.6)
    f, _ = oracle.pbsym(np.array([[10.5, 10.5, 7.5]]), grid)
    assert np.array_equal(f, f[::-1, :, :])
    assert np.array_equal(f, f[:, ::-1, :])
    assert np.array_equal(f, f[:, :, ::-1])
    # (1 - u^2) - v^2 and (1 - v^2) - u^2 round differently: swap holds to rounding
    assert _rel_err(f, np.transpose(f, (1, 0, 2))) <= 1e-15


def test_superposition():
    pa, g = small_random_case(31, max_g=24, max_n=100)
    grid = Grid(**g)
    rng = np.random.default_rng(1)
    pb = pa[rng.permutation(pa.shape[0])][: max(1, pa.shape[0] // 2)] + 0.37
    fa, _ = oracle.pbsym(pa, grid)
    fb, _ = oracle.pbsym(pb, grid)
    fab, _ = oracle.pbsym(np.concatenate([pa, pb]), grid)
    na, nb = pa.shape[0], pb.shape[0]
    assert _rel_err(na * fa + nb * fb, (na + nb) * fab) <= 1e-13


def test_zero_outside_cylinders():
    pts, g = small_random_case(41, max_g=30, max_n=5)
    grid = Grid(**g)
    f, _ = oracle.pbsym(pts, grid)
    X, Y, T = np.meshgrid(np.arange(grid.gx), np.arange(grid.gy), np.arange(grid.gt), indexing="ij")
    x = grid.x0 + (X + 0.5) * grid.sres
    y = grid.y0 + (Y + 0.5) * grid.sres
    t = grid.t0 + (T + 0.5) * grid.tres
    near = np.zeros(f.shape, bool)
    for p in pts:
        near |= (np.hypot(x - p[0], y - p[1]) < grid.hs) & (np.abs(t - p[2]) <= grid.ht)
    assert np.all(f[~near] == 0.0)
    assert np.all(f >= 0.0)


def test_translation_whole_voxels():
    """Dyadic coordinates: moving the events and the origin together by whole
    voxels leaves every x - x0 unchanged, so the grid is identical."""
    rng = np.random.default_rng(8)
    pts = np.round(rng.uniform(0, 32, (60, 3)) * 64) / 64
    g1 = Grid(gx=32, gy=32, gt=32, hs=4.25, ht=3.5, sres=0.5, tres=2.0)
    g2 = Grid(gx=32, gy=32, gt=32, hs=4.25, ht=3.5, sres=0.5, tres=2.0, x0=3.5, y0=-2.0, t0=8.0)
    f1, _ = oracle.pbsym(pts, g1)
    f2, _ = oracle.pbsym(pts + np.array([3.5, -2.0, 8.0]), g2)
    assert np.array_equal(f1, f2)


def test_thread_count_independence():
    pts, g = small_random_case(55, max_g=40, max_n=300)
    grid = Grid(**g)
    f1, e1 = oracle.pbsym(pts, grid, nthreads=1)
    f5, e5 = oracle.pbsym(pts, grid, nthreads=5)
    assert np.array_equal(f1, f5) and e1 == e5


def test_non_finite_events_count_in_n_only():
    pts, g = small_random_case(61, max_g=20, max_n=50)
    grid = Grid(**g)
    f, _ = oracle.pbsym(pts, grid)
    bad = np.array([[np.nan, 1.0, 1.0], [1.0, np.inf, 2.0], [0.0, 0.0, -np.inf]])
    f2, _ = oracle.pbsym(np.concatenate([pts, bad]), grid)
    n = pts.shape[0]
    assert _rel_err(f2 * (n + 3), f * n) <= 1e-14


def test_invalid_arguments():
    with pytest.raises(ValueError):
        oracle.pbsym(np.zeros((0, 3)), Grid(gx=4, gy=4, gt=4, hs=1.0, ht=1.0))
    with pytest.raises(ValueError):
        oracle.pbsym(np.zeros((1, 3)), Grid(gx=4, gy=4, gt=4, hs=0.0, ht=1.0))
    with pytest.raises(ValueError):
        oracle.pbsym(np.zeros((1, 3)), Grid(gx=0, gy=4, gt=4, hs=1.0, ht=1.0))


# --------------------------------------------------- the pins have teeth
_MUTANTS = [
    ("dropped 2/pi", "return (2.0 / ORACLE_PI) * (1.0 - u * u - v * v);",
     "return (1.0 - u * u - v * v);"),
    ("sign in kt", "return 0.75 * (1.0 - w * w);", "return 0.75 * (1.0 + w * w);"),
    ("transposed Y", "grid + (X * Gy + Y) * Gt + Ta", "grid + (Y * Gx + X) * Gt + Ta"),
    ("corner sampling", "return g->corner ? 0.0 : 0.5;", "return 0.0;"),
    ("short loop bound", "const int64_t Hs = (int64_t)ceil(g->hs / g->sres);\n"
     "    const int64_t Ht = (int64_t)ceil(g->ht / g->tres);\n    const double norm",
     "const int64_t Hs = (int64_t)floor(g->hs / g->sres);\n"
     "    const int64_t Ht = (int64_t)ceil(g->ht / g->tres);\n    const double norm"),
]


@pytest.mark.parametrize("name,old,new", _MUTANTS, ids=[m[0] for m in _MUTANTS])
def test_pins_detect_planted_mistake(name, old, new, tmp_path):
    """Plant a mistake in a private copy of the oracle (on the CPU) and check
    that the brute-force or library pins reject it."""
    import ctypes
    src = open(os.path.join(os.path.dirname(oracle.__file__), "stkde_oracle.c")).read()
    assert old in src, name
    d = tmp_path
    shutil.copy(os.path.join(os.path.dirname(oracle.__file__), "stkde_oracle.h"), d / "stkde_oracle.h")
    (d / "m.c").write_text(src.replace(old, new))
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", str(d / "m.c"), "-o",
                    str(d / "m.so"), "-lm"], check=True)
    lib = ctypes.CDLL(str(d / "m.so"))
    from oracle import _Grid
    lib.oracle_pbsym.argtypes = [ctypes.POINTER(_Grid), ctypes.c_void_p, ctypes.c_int64,
                                 ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    detected = False
    for seed in range(4):
        pts, g = small_random_case(300 + seed, max_g=18, max_n=40)
        grid = Grid(**g)
        out = np.empty((grid.gx, grid.gy, grid.gt))
        ev = ctypes.c_int64(0)
        lib.oracle_pbsym(ctypes.byref(grid._c()), np.ascontiguousarray(pts).ctypes.data,
                         pts.shape[0], out.ctypes.data, ctypes.byref(ev), 1)
        ref = oracle.vb_grid_numpy(pts, grid)
        if _rel_err(out, ref) > 1e-13:
            detected = True
            break
    # the numpy brute force shares no code with the C loops, so it must see every mutant
    assert detected, name


# ------------------------------------------------------ regression fixture
def _read_golden():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tiny_case.txt")
    grid, pts, vals, evals = None, [], {}, None
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        tok = line.split()
        if tok[0] == "grid":
            kv = dict(t.split("=") for t in tok[1:])
            grid = Grid(**{k: (int(v) if k in ("gx", "gy", "gt") else float(v)) for k, v in kv.items()})
        elif tok[0] == "point":
            pts.append([float(v) for v in tok[1:]])
        elif tok[0] == "evals":
            evals = int(tok[1])
        elif tok[0] == "v":
            vals[(int(tok[1]), int(tok[2]), int(tok[3]))] = float(tok[4])
    return grid, np.array(pts), vals, evals


def test_golden_tiny_case():
    """Regression: the oracle reproduces its committed output bit for bit,
    and the brute force agrees with that output."""
    grid, pts, vals, evals = _read_golden()
    f, ev = oracle.pbsym(pts, grid, nthreads=2)
    assert ev == evals
    ref = np.zeros_like(f)
    for k, v in vals.items():
        ref[k] = v
    assert np.array_equal(f, ref)
    assert _rel_err(oracle.vb_grid_numpy(pts, grid), ref) <= 1e-13
