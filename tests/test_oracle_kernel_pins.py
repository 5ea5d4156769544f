"""Pins for the oracle's other kernel pairs and for corner sampling.

PB-SYM needs only that the kernel is a product of a spatial and a temporal
factor (Sec. 3.2); besides the default Epanechnikov reading the oracle
offers the quartic (biweight) pair, a Gaussian truncated at the bandwidth
(sigma = half of it, normalised on its support) and the pair exactly as
Sec. 2.1 prints it.  Pins, each independent of the C loops:

* brute force: Alg. VB in numpy (its own kernel code) on random grids;
* closed forms at a voxel-centred event (exact rationals times pi or 1/pi);
* continuum limit of each event's mass: 1 for the normalised pairs,
  37 pi^2 / 24 for the printed pair (its integral over the cylinder);
* corner sampling equals centre sampling of the grid shifted by half a voxel;
* planted mistakes in each pair are detected.
"""
import ctypes
import math
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import Grid, KERNEL_GAUSSIAN, KERNEL_PRINTED, KERNEL_QUARTIC
from workloads import small_random_case

FAMILIES = (KERNEL_QUARTIC, KERNEL_GAUSSIAN, KERNEL_PRINTED)
NAMES = {KERNEL_QUARTIC: "quartic", KERNEL_GAUSSIAN: "gaussian", KERNEL_PRINTED: "printed"}


def _rel_err(a, b):
    scale = max(float(np.max(np.abs(b))), 1e-300)
    return float(np.max(np.abs(a - b)) / scale)


@pytest.mark.parametrize("kernel", FAMILIES, ids=[NAMES[k] for k in FAMILIES])
@pytest.mark.parametrize("seed", range(6))
def test_matches_numpy_brute_force(kernel, seed):
    pts, g = small_random_case(1300 + seed, max_g=24, max_n=120)
    for corner in (False, True):
        grid = Grid(**g, kernel=kernel, corner=corner)
        f, _ = oracle.pbsym(pts, grid)
        assert _rel_err(f, oracle.vb_grid_numpy(pts, grid)) <= 1e-13


def test_default_pair_unchanged_by_the_selector():
    pts, g = small_random_case(1400, max_g=24, max_n=120)
    a, ea = oracle.pbsym(pts, Grid(**g))
    b, eb = oracle.pbsym(pts, Grid(**g, kernel=0, corner=False))
    assert np.array_equal(a, b) and ea == eb


@pytest.mark.parametrize("hs,ht", [(4, 3), (Fraction(11, 2), Fraction(7, 2))])
def test_single_event_closed_forms(hs, ht):
    H, Tt = int(math.ceil(hs)) + 1, int(math.ceil(ht)) + 1
    grid = dict(gx=2 * H + 1, gy=2 * H + 1, gt=2 * Tt + 1, hs=float(hs), ht=float(ht))
    pts = np.array([[H + 0.5, H + 0.5, Tt + 0.5]])
    hs_f, ht_f = Fraction(hs), Fraction(ht)
    fq, eq = oracle.pbsym(pts, Grid(**grid, kernel=KERNEL_QUARTIC))
    fp, ep = oracle.pbsym(pts, Grid(**grid, kernel=KERNEL_PRINTED))
    fg, _ = oracle.pbsym(pts, Grid(**grid, kernel=KERNEL_GAUSSIAN))
    cnt = 0
    for a in range(-H, H + 1):
        for b in range(-H, H + 1):
            for k in range(-Tt, Tt + 1):
                inside = Fraction(a * a + b * b) < hs_f * hs_f and abs(Fraction(k)) <= ht_f
                cnt += inside
                if not inside:
                    assert fq[H + a, H + b, Tt + k] == 0.0 and fp[H + a, H + b, Tt + k] == 0.0
                    continue
                r2 = Fraction(a * a + b * b) / (hs_f * hs_f)
                w = Fraction(k) / ht_f
                # quartic: (3/pi)(1 - r^2)^2 (15/16)(1 - w^2)^2 / (hs^2 ht)
                q = Fraction(45, 16) * (1 - r2) ** 2 * (1 - w * w) ** 2 / (hs_f * hs_f * ht_f)
                assert abs(fq[H + a, H + b, Tt + k] * math.pi - float(q)) <= 1e-14 * float(q) + 1e-300
                # printed: (pi/2)(1 - u)^2 (1 - v)^2 (3/4)(1 - w)^2 / (hs^2 ht), u = a/hs
                u, v = Fraction(a) / hs_f, Fraction(b) / hs_f
                pr = Fraction(3, 8) * (1 - u) ** 2 * (1 - v) ** 2 * (1 - w) ** 2 / (hs_f * hs_f * ht_f)
                assert abs(fp[H + a, H + b, Tt + k] / math.pi - float(pr)) <= 1e-14 * float(pr) + 1e-300
                # Gaussian: the ratio to the peak is exp(-2 r^2 - 2 w^2)
                ratio = fg[H + a, H + b, Tt + k] / fg[H, H, Tt]
                assert ratio == pytest.approx(math.exp(-2.0 * float(r2) - 2.0 * float(w * w)), rel=1e-13)
    assert eq == cnt and ep == cnt


@pytest.mark.parametrize("kernel,expect", [(KERNEL_QUARTIC, 1.0), (KERNEL_GAUSSIAN, 1.0),
                                           (KERNEL_PRINTED, 37.0 * math.pi ** 2 / 24.0)],
                         ids=["quartic", "gaussian", "printed"])
def test_mass_continuum_limit(kernel, expect):
    """Events uniform within interior voxels: the expected Riemann sum of each
    event's kernel over the grid is the kernel's integral over its cylinder."""
    rng = np.random.default_rng(11)
    hs, ht = 6.3, 4.7
    grid = Grid(gx=48, gy=48, gt=32, hs=hs, ht=ht, kernel=kernel)
    n = 3000
    pts = np.stack([rng.uniform(12, 36, n), rng.uniform(12, 36, n), rng.uniform(8, 24, n)], axis=1)
    Ss, St, _, _ = oracle.point_sums(pts, grid)
    m = Ss * St / (hs * hs * ht)
    se = m.std(ddof=1) / math.sqrt(n)
    assert abs(m.mean() - expect) < max(5 * se, 1e-6 * expect)


@pytest.mark.parametrize("kernel", (0,) + FAMILIES, ids=["epanechnikov"] + [NAMES[k] for k in FAMILIES])
def test_corner_sampling_is_a_half_voxel_shift(kernel):
    """Dyadic coordinates: sampling at lower corners with origin (x0, y0, t0)
    is sampling at centres with the origin moved back by half a voxel."""
    rng = np.random.default_rng(21)
    pts = np.round(rng.uniform(-3, 35, (80, 3)) * 64) / 64
    g = dict(gx=32, gy=30, gt=28, hs=4.25, ht=3.5, sres=0.5, tres=2.0, x0=1.5, y0=-2.0, t0=6.0)
    fc, ec = oracle.pbsym(pts, Grid(**g, kernel=kernel, corner=True))
    shifted = {**g, "x0": g["x0"] - 0.25, "y0": g["y0"] - 0.25, "t0": g["t0"] - 1.0}
    fs, es = oracle.pbsym(pts, Grid(**shifted, kernel=kernel))
    assert np.array_equal(fc, fs) and ec == es


def test_mass_identity_all_pairs():
    for kernel in FAMILIES:
        pts, g = small_random_case(1500 + kernel, max_g=30, max_n=200)
        grid = Grid(**g, kernel=kernel, corner=bool(kernel & 1))
        f, evals = oracle.pbsym(pts, grid)
        assert f.sum() * grid.sres ** 2 * grid.tres == pytest.approx(oracle.exact_mass(pts, grid), rel=1e-12,
                                                                     abs=1e-300)
        assert evals == oracle.exact_evals(pts, grid)


_MUTANTS = [
    ("quartic without its square", "return (3.0 / ORACLE_PI) * e * e;", "return (3.0 / ORACLE_PI) * e;",
     KERNEL_QUARTIC),
    ("quartic temporal constant", "return (15.0 / 16.0) * e * e;", "return 0.75 * e * e;", KERNEL_QUARTIC),
    ("gaussian sigma", "return exp(-2.0 * (u * u + v * v))", "return exp(-0.5 * (u * u + v * v))",
     KERNEL_GAUSSIAN),
    ("gaussian temporal normalisation", "(sqrt(0.5 * ORACLE_PI) * erf(sqrt(2.0)))",
     "(sqrt(0.5 * ORACLE_PI) * erf(sqrt(0.5)))", KERNEL_GAUSSIAN),
    ("printed sign", "(ORACLE_PI / 2.0) * (1.0 - u) * (1.0 - u) * (1.0 - v) * (1.0 - v)",
     "(ORACLE_PI / 2.0) * (1.0 + u) * (1.0 + u) * (1.0 - v) * (1.0 - v)", KERNEL_PRINTED),
    ("printed temporal sign", "return 0.75 * (1.0 - w) * (1.0 - w);", "return 0.75 * (1.0 + w) * (1.0 + w);",
     KERNEL_PRINTED),
]


@pytest.mark.parametrize("name,old,new,kernel", _MUTANTS, ids=[m[0] for m in _MUTANTS])
def test_pins_detect_planted_mistake(name, old, new, kernel, tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "stkde_oracle.c")).read()
    assert src.count(old) == 1, name
    shutil.copy(os.path.join(os.path.dirname(oracle.__file__), "stkde_oracle.h"), tmp_path / "stkde_oracle.h")
    (tmp_path / "m.c").write_text(src.replace(old, new))
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", str(tmp_path / "m.c"), "-o",
                    str(tmp_path / "m.so"), "-lm"], check=True)
    lib = ctypes.CDLL(str(tmp_path / "m.so"))
    from oracle import _Grid
    lib.oracle_pbsym.argtypes = [ctypes.POINTER(_Grid), ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                 ctypes.POINTER(ctypes.c_int64), ctypes.c_int]
    detected = False
    for seed in range(4):
        pts, g = small_random_case(1600 + seed, max_g=18, max_n=40)
        grid = Grid(**g, kernel=kernel)
        out = np.empty((grid.gx, grid.gy, grid.gt))
        ev = ctypes.c_int64(0)
        lib.oracle_pbsym(ctypes.byref(grid._c()), np.ascontiguousarray(pts).ctypes.data, len(pts),
                         out.ctypes.data, ctypes.byref(ev), 1)
        if _rel_err(out, oracle.vb_grid_numpy(pts, grid)) > 1e-13:
            detected = True
            break
    assert detected, name
