"""Pins for the oracle's per-event (sample-point adaptive) bandwidths.

Sec. 8 names a bandwidth that adapts to the local density as future work
without a rule for choosing it; the reading here is the sample-point
estimator, f = 1/n sum_i ks(./hs_i) kt(./ht_i) / (hs_i^2 ht_i), with the
pairs (hs_i, ht_i) given as input.  The pins tie it to facts other than
itself:

* special case: equal pairs reduce it bit for bit to the fixed-bandwidth
  PB-SYM, which test_oracle_pins.py pins to library routines, closed forms
  and brute force;
* superposition across bandwidths: the union of two sets, each with its own
  fixed pair, is the n-weighted mean of their fixed-bandwidth densities (a
  normalisation by any shared bandwidth breaks it);
* brute force: Alg. VB with per-event bandwidths written separately in numpy;
* closed form: one event at a voxel centre with a pair unlike the grid's;
* mass: the grid sum equals the per-event separable sums, and each event's
  mass tends to one;
* invalid pairs contribute nothing but count in n;
* planted mistakes in a private copy of the C source are all detected.
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
from oracle import Grid
from workloads import small_random_case


def _rel_err(a, b):
    scale = max(float(np.max(np.abs(b))), 1e-300)
    return float(np.max(np.abs(a - b)) / scale)


def _pairs(rng, n, grid, lo=0.3, hi=1.6):
    return np.stack([grid.hs * rng.uniform(lo, hi, n), grid.ht * rng.uniform(lo, hi, n)], axis=1)


def test_equal_pairs_are_the_fixed_estimator():
    for seed in range(6):
        pts, g = small_random_case(400 + seed, max_g=30, max_n=200)
        grid = Grid(**g)
        h = np.tile([grid.hs, grid.ht], (len(pts), 1))
        fa, ea = oracle.pbsym_adaptive(pts, h, grid)
        f, e = oracle.pbsym(pts, grid)
        assert np.array_equal(fa, f) and ea == e


@pytest.mark.parametrize("seed", range(12))
def test_matches_numpy_brute_force(seed):
    pts, g = small_random_case(500 + seed, max_g=26, max_n=120)
    grid = Grid(**g)
    h = _pairs(np.random.default_rng(seed), len(pts), grid)
    f, _ = oracle.pbsym_adaptive(pts, h, grid)
    ref = oracle.vb_grid_numpy_adaptive(pts, h, grid)
    assert _rel_err(f, ref) <= 1e-13


def test_union_of_two_fixed_bandwidth_sets():
    pa, g = small_random_case(611, max_g=24, max_n=90)
    grid_a = Grid(**g)
    rng = np.random.default_rng(2)
    pb = pa[rng.permutation(len(pa))][: max(1, len(pa) // 2)] + 0.41
    grid_b = Grid(**{**g, "hs": g["hs"] * 0.55, "ht": g["ht"] * 1.7})
    fa, _ = oracle.pbsym(pa, grid_a)
    fb, _ = oracle.pbsym(pb, grid_b)
    h = np.concatenate([np.tile([grid_a.hs, grid_a.ht], (len(pa), 1)),
                        np.tile([grid_b.hs, grid_b.ht], (len(pb), 1))])
    fab, _ = oracle.pbsym_adaptive(np.concatenate([pa, pb]), h, grid_a)
    na, nb = len(pa), len(pb)
    assert _rel_err((na * fa + nb * fb) / (na + nb), fab) <= 1e-13


def _single_point_exact(hs, ht, a, b, k):
    hs, ht = Fraction(hs), Fraction(ht)
    r2 = Fraction(a * a + b * b)
    if r2 >= hs * hs or abs(Fraction(k)) > ht:
        return Fraction(0)
    return Fraction(3, 2) * (1 - r2 / (hs * hs)) * (1 - Fraction(k * k) / (ht * ht)) / (hs * hs * ht)


@pytest.mark.parametrize("hs,ht", [(4, 3), (Fraction(13, 2), Fraction(5, 2))])
def test_single_event_closed_form(hs, ht):
    """One event at a voxel centre, its pair unlike the grid's: values are
    exact rationals over pi; a second event with an invalid pair halves them
    (n = 2)."""
    H, Tt = int(math.ceil(hs)) + 2, int(math.ceil(ht)) + 2
    grid = Grid(gx=2 * H + 1, gy=2 * H + 1, gt=2 * Tt + 1, hs=1.0, ht=1.0)
    pts = np.array([[H + 0.5, H + 0.5, Tt + 0.5], [H + 0.5, H + 0.5, Tt + 0.5]])
    h = np.array([[float(hs), float(ht)], [np.nan, 1.0]])
    f, evals = oracle.pbsym_adaptive(pts, h, grid)
    cnt = 0
    for a in range(-H, H + 1):
        for b in range(-H, H + 1):
            for k in range(-Tt, Tt + 1):
                ex = float(_single_point_exact(hs, ht, a, b, k)) / 2.0
                assert abs(f[H + a, H + b, Tt + k] * math.pi - ex) <= 1e-15 * (1 + ex)
                cnt += a * a + b * b < hs * hs and abs(k) <= ht
    assert evals == cnt


def test_mass_identity_and_eval_count():
    for seed in range(6):
        pts, g = small_random_case(700 + seed, max_g=30, max_n=200)
        grid = Grid(**g)
        h = _pairs(np.random.default_rng(seed), len(pts), grid)
        f, evals = oracle.pbsym_adaptive(pts, h, grid)
        m_grid = f.sum() * grid.sres ** 2 * grid.tres
        assert m_grid == pytest.approx(oracle.exact_mass_adaptive(pts, h, grid), rel=1e-12, abs=1e-300)
        assert evals == oracle.exact_evals_adaptive(pts, h, grid)


def test_mass_continuum_limit():
    """Interior events with pairs spread over a decade: each deposits mass
    close to one, and the mean is one within a few standard errors."""
    rng = np.random.default_rng(5)
    grid = Grid(gx=80, gy=80, gt=48, hs=9.0, ht=7.0)
    n = 3000
    pts = np.stack([rng.uniform(25, 55, n), rng.uniform(25, 55, n), rng.uniform(16, 32, n)], axis=1)
    h = np.stack([rng.uniform(1.5, 9.0, n), rng.uniform(1.2, 7.0, n)], axis=1)
    Ss, St, _, _ = oracle.point_sums_adaptive(pts, h, grid)
    m = Ss * St / (h[:, 0] ** 2 * h[:, 1])
    se = m.std(ddof=1) / math.sqrt(n)
    assert abs(m.mean() - 1.0) < max(5 * se, 1e-6)
    assert np.all(np.abs(m - 1.0) < 0.35)


def test_invalid_pairs_contribute_nothing():
    pts, g = small_random_case(811, max_g=20, max_n=60)
    grid = Grid(**g)
    h = _pairs(np.random.default_rng(1), len(pts), grid)
    f, _ = oracle.pbsym_adaptive(pts, h, grid)
    extra = np.array([[3.0, 3.0, 3.0]] * 5)
    bad = np.array([[np.nan, 1.0], [1.0, np.inf], [0.0, 1.0], [1.0, -2.0], [-1.0, 1.0]])
    f2, _ = oracle.pbsym_adaptive(np.concatenate([pts, extra]), np.concatenate([h, bad]), grid)
    n = len(pts)
    assert _rel_err(f2 * (n + 5), f * n) <= 1e-14


def test_vb_voxels_and_far_event_with_huge_bandwidth():
    """Alg. VB at sampled voxels equals the grid, also for an event far
    outside the grid whose bandwidth still reaches it."""
    pts, g = small_random_case(901, max_g=24, max_n=80)
    grid = Grid(**g)
    h = _pairs(np.random.default_rng(3), len(pts), grid)
    far = np.array([[grid.x0 - 200.0 * grid.sres, grid.y0 + 3.0 * grid.sres, grid.t0 + 2.0 * grid.tres]])
    hf = np.array([[205.0 * grid.sres, 3.0 * grid.tres]])
    P, Hh = np.concatenate([pts, far]), np.concatenate([h, hf])
    f, _ = oracle.pbsym_adaptive(P, Hh, grid)
    assert _rel_err(f, oracle.vb_grid_numpy_adaptive(P, Hh, grid)) <= 1e-13
    f_near, _ = oracle.pbsym_adaptive(pts, h, grid)
    assert not np.allclose(f * len(P), f_near * len(pts))  # the far event reaches the grid
    rng = np.random.default_rng(4)
    vox = np.stack([rng.integers(0, grid.gx, 40), rng.integers(0, grid.gy, 40), rng.integers(0, grid.gt, 40)], 1)
    v = oracle.vb_voxels_adaptive(P, Hh, grid, vox)
    assert _rel_err(v, f[vox[:, 0], vox[:, 1], vox[:, 2]]) <= 1e-13


def test_thread_count_independence():
    pts, g = small_random_case(955, max_g=40, max_n=300)
    grid = Grid(**g)
    h = _pairs(np.random.default_rng(9), len(pts), grid)
    f1, e1 = oracle.pbsym_adaptive(pts, h, grid, nthreads=1)
    f6, e6 = oracle.pbsym_adaptive(pts, h, grid, nthreads=6)
    assert np.array_equal(f1, f6) and e1 == e6


_MUTANTS = [
    ("normalisation by the grid's pair", "const double norm = 1.0 / ((double)n * hs * hs * ht);",
     "const double norm = 1.0 / ((double)n * g->hs * g->hs * g->ht);"),
    ("support by the grid's hs", "if (d < hs) {", "if (d < g->hs) {"),
    ("kt scaled by the grid's ht", "Kt[T - Ta] = kt_of(g->kernel, (t - ti) / ht);",
     "Kt[T - Ta] = kt_of(g->kernel, (t - ti) / g->ht);"),
    ("short loop bound", "const double Hs = ceil(hs / g->sres), Ht = ceil(ht / g->tres);\n"
     "                const double norm",
     "const double Hs = floor(hs / g->sres), Ht = ceil(ht / g->tres);\n"
     "                const double norm"),
]


@pytest.mark.parametrize("name,old,new", _MUTANTS, ids=[m[0] for m in _MUTANTS])
def test_pins_detect_planted_mistake(name, old, new, tmp_path):
    src = open(os.path.join(os.path.dirname(oracle.__file__), "stkde_oracle.c")).read()
    assert src.count(old) == 1, name
    shutil.copy(os.path.join(os.path.dirname(oracle.__file__), "stkde_oracle.h"), tmp_path / "stkde_oracle.h")
    (tmp_path / "m.c").write_text(src.replace(old, new))
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", str(tmp_path / "m.c"), "-o",
                    str(tmp_path / "m.so"), "-lm"], check=True)
    lib = ctypes.CDLL(str(tmp_path / "m.so"))
    from oracle import _Grid
    lib.oracle_pbsym_adaptive.argtypes = [ctypes.POINTER(_Grid), ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                          ctypes.c_int]
    detected = False
    for seed in range(4):
        pts, g = small_random_case(1000 + seed, max_g=18, max_n=40)
        grid = Grid(**g)
        h = np.ascontiguousarray(_pairs(np.random.default_rng(seed), len(pts), grid))
        out = np.empty((grid.gx, grid.gy, grid.gt))
        ev = ctypes.c_int64(0)
        lib.oracle_pbsym_adaptive(ctypes.byref(grid._c()), np.ascontiguousarray(pts).ctypes.data,
                                  h.ctypes.data, len(pts), out.ctypes.data, ctypes.byref(ev), 1)
        if _rel_err(out, oracle.vb_grid_numpy_adaptive(pts, h, grid)) > 1e-13:
            detected = True
            break
    assert detected, name
