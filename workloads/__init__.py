"""Seeded synthetic point clouds shaped like the paper's workloads.

The paper measures on four real datasets (Sec. 6.1: an epidemiology set of a
city, a social-media set of a continent, two ornithology sets of the world;
shapes in Table "tab:instance").  None of them is available here, so every
run uses the seeded stand-ins below.  This module holds input generation
only -- no part of the density estimate -- and is the one module that both
the oracle-side tests and the GPU-side tests and benchmark import.

All generators use numpy's PCG64 with seed ``SEED_BASE + config index`` and
return an (n, 3) float64 array of (x, y, t) in domain units with unit voxels
and the origin at 0 (sres = tres = 1, x0 = y0 = t0 = 0).
"""
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

SEED_BASE = 170509366


def rng_for(index: int, salt: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + index + 1000003 * salt))


def uniform(rng: np.random.Generator, n: int, gx: float, gy: float, gt: float) -> np.ndarray:
    """i.i.d. uniform points over [0,gx) x [0,gy) x [0,gt)."""
    out = np.empty((n, 3), dtype=np.float64)
    out[:, 0] = rng.uniform(0.0, gx, n)
    out[:, 1] = rng.uniform(0.0, gy, n)
    out[:, 2] = rng.uniform(0.0, gt, n)
    return out


def clustered(rng: np.random.Generator, k: int, n: int, gx: int, gy: int, gt: int,
              sigma_range: Tuple[float, float] = (5.0, 80.0), seasons: int = 8,
              background: float = 0.2) -> np.ndarray:
    """Gaussian-mixture events in (x, y) with seasonal bumps in t.

    * k components, means uniform in the central 80 % of each spatial axis,
      isotropic sigma log-uniform in ``sigma_range`` voxels, weights
      log-uniform over two decades;
    * t: with probability 1 - background from one of ``seasons`` bumps centred
      at (j + 1/2) gt / seasons with sigma gt / 48, else uniform over [0, gt);
    * t is drawn independently of the spatial component;
    * any coordinate that falls outside the grid is drawn again, so every
      point is inside the grid (footprints near the border are still clipped).
    """
    mix = _mixture(rng, k, gx, gy, sigma_range)
    return _mixture_events(rng, mix, n, gx, gy, gt, seasons, background)


def _mixture(rng, k, gx, gy, sigma_range):
    mu = np.stack([rng.uniform(0.1 * gx, 0.9 * gx, k), rng.uniform(0.1 * gy, 0.9 * gy, k)], axis=1)
    sig = np.exp(rng.uniform(np.log(sigma_range[0]), np.log(sigma_range[1]), k))
    w = np.exp(rng.uniform(0.0, np.log(100.0), k))
    w /= w.sum()
    return mu, sig, w


def _mixture_events(rng, mix, n, gx, gy, gt, seasons, background, season_sigma=None):
    mu, sig, w = mix
    ssig = gt / 48.0 if season_sigma is None else season_sigma
    comp = rng.choice(len(w), size=n, p=w)
    xy = np.empty((n, 2))
    todo = np.arange(n)
    while todo.size:
        c = comp[todo]
        cand = mu[c] + rng.standard_normal((todo.size, 2)) * sig[c][:, None]
        ok = (cand[:, 0] >= 0) & (cand[:, 0] < gx) & (cand[:, 1] >= 0) & (cand[:, 1] < gy)
        xy[todo[ok]] = cand[ok]
        todo = todo[~ok]
    t = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        m = todo.size
        bg = rng.uniform(0.0, 1.0, m) < background
        j = rng.integers(0, seasons, m)
        bump = (j + 0.5) * gt / seasons + rng.standard_normal(m) * ssig
        cand = np.where(bg, rng.uniform(0.0, gt, m), bump)
        ok = (cand >= 0) & (cand < gt)
        t[todo[ok]] = cand[ok]
        todo = todo[~ok]
    out = np.empty((n, 3), dtype=np.float64)
    out[:, :2] = xy
    out[:, 2] = t
    return out


@dataclass
class Instance:
    """One density-estimation problem: points plus grid and bandwidths
    (voxel units, unit voxels, origin 0 unless stated)."""
    name: str
    points: np.ndarray
    gx: int
    gy: int
    gt: int
    hs: float
    ht: float
    x0: float = 0.0
    y0: float = 0.0
    t0: float = 0.0
    sres: float = 1.0
    tres: float = 1.0
    meta: dict = field(default_factory=dict)


def config0() -> Instance:
    """Small uniform case: n = 10,000 over 128 x 128 x 64, hs = 5, ht = 4."""
    rng = rng_for(0)
    return Instance("uniform-10k-128x128x64-hs5-ht4", uniform(rng, 10_000, 128, 128, 64),
                    128, 128, 64, 5.0, 4.0)


def config1(n: int = 1_000_000) -> Instance:
    """Large clustered case: 64-component mixture, n = 1M,
    1024 x 1024 x 256 grid (1 GiB of FP32), hs = 10, ht = 7."""
    rng = rng_for(1)
    return Instance(f"clustered-{n}-1024x1024x256-hs10-ht7",
                    clustered(rng, 64, n, 1024, 1024, 256), 1024, 1024, 256, 10.0, 7.0)


def config2(n: int = 200_000) -> Instance:
    """Large-bandwidth case: 16-component mixture, n = 200k,
    512 x 512 x 365 grid, hs = 50, ht = 30."""
    rng = rng_for(2)
    return Instance(f"clustered-{n}-512x512x365-hs50-ht30",
                    clustered(rng, 16, n, 512, 512, 365), 512, 512, 365, 50.0, 30.0)


def config3_sets(count: int = 8) -> List[Instance]:
    """Bandwidth sweep over shared point sets: ``count`` sets, each with 8
    bandwidth pairs (hs ~ U[3,30], ht ~ U[2,20]).  Set sizes n log-uniform in
    [1e3, 5e5]; gx = gy log-uniform in [64, 512] rounded to a multiple of 16;
    gt uniform over the multiples of 16 in [64, 128]."""
    rng = rng_for(3)
    out = []
    for s in range(count):
        n = int(np.exp(rng.uniform(np.log(1e3), np.log(5e5))))
        g = int(round(np.exp(rng.uniform(np.log(64), np.log(512))) / 16.0)) * 16
        g = max(64, min(512, g))
        gt = int(rng.choice(np.arange(64, 129, 16)))
        pts = clustered(rng, 16, n, g, g, gt)
        for b in range(8):
            hs = float(rng.uniform(3.0, 30.0))
            ht = float(rng.uniform(2.0, 20.0))
            out.append(Instance(f"sweep-set{s}-bw{b}", pts, g, g, gt, hs, ht,
                                meta={"set": s}))
    return out


def config4_sets() -> List[Instance]:
    """Resident point sets of the serving case: n in {100k, 300k, 800k, 2M},
    each clustered over a 2048 x 2048 x 512 base domain (64 components)."""
    rng = rng_for(4)
    return [Instance(f"resident-{n}", clustered(rng, 64, n, 2048, 2048, 512), 2048, 2048, 512,
                     10.0, 10.0) for n in (100_000, 300_000, 800_000, 2_000_000)]


def config4_requests(count: int, seed_salt: int = 0):
    """Requests of the serving case: a set index, a sub-region grid
    (gx, gy log-uniform in [64, 1024], gt log-uniform in [64, 128]) placed
    inside the 2048 x 2048 x 512 base domain, and hs, ht ~ U[3, 40]."""
    rng = rng_for(4, salt=1 + seed_salt)
    reqs = []
    for _ in range(count):
        s = int(rng.integers(0, 4))
        gx = int(np.exp(rng.uniform(np.log(64), np.log(1024))))
        gy = int(np.exp(rng.uniform(np.log(64), np.log(1024))))
        gt = int(np.exp(rng.uniform(np.log(64), np.log(128))))
        x0 = float(rng.integers(0, 2048 - gx + 1))
        y0 = float(rng.integers(0, 2048 - gy + 1))
        t0 = float(rng.integers(0, 512 - gt + 1))
        reqs.append(dict(set=s, gx=gx, gy=gy, gt=gt, x0=x0, y0=y0, t0=t0,
                         hs=float(rng.uniform(3, 40)), ht=float(rng.uniform(3, 40))))
    return reqs


WORLD_EVENTS = 291_990_435


def _world_chunk(args):
    index, mix, m, gx, gy, gt = args
    return _mixture_events(rng_for(5, salt=1 + index), mix, m, gx, gy, gt, 40, 0.2, season_sigma=10.0)


def world_scale(resolution: str = "Hr", bandwidth: str = "Hb", n: int = WORLD_EVENTS,
                chunk: int = 1 << 23, workers: int = 0) -> Instance:
    """Stand-in for the paper's largest instances, the worldwide bird-spotting
    set of Sec. 6.1 (291,990,435 events over 20 years at 3-day resolution;
    Table tab:instance): grid 1781 x 3601 x 2435 at high resolution (60 GB of
    FP32) or 357 x 721 x 2435 at low; bandwidths (Hs, Ht) = (10, 3) / (30, 5)
    voxels at high resolution and (2, 3) / (6, 5) at low, as in that table.

    Events: a 256-component Gaussian mixture in space (sigma log-uniform 3-150
    voxels at high resolution, a fifth of that at low), 40 seasonal bumps in
    time (two migrations a year, sigma 10 voxels = 30 days) with 20 % uniform
    background.  Chunk c of ``chunk`` events comes from its own seeded stream,
    so the events do not depend on how many worker processes draw them
    (``workers`` > 1: a pool of freshly started processes that only run numpy)."""
    hi = resolution == "Hr"
    gx, gy, gt = (1781, 3601, 2435) if hi else (357, 721, 2435)
    hs, ht = {("Hr", "Lb"): (10.0, 3.0), ("Hr", "Hb"): (30.0, 5.0),
              ("Lr", "Lb"): (2.0, 3.0), ("Lr", "Hb"): (6.0, 5.0)}[(resolution, bandwidth)]
    scale = 1.0 if hi else 0.2
    mix = _mixture(rng_for(5), 256, gx, gy, (3.0 * scale, 150.0 * scale))
    out = np.empty((n, 3), dtype=np.float64)
    jobs = [(c, mix, min(chunk, n - b), gx, gy, gt) for c, b in enumerate(range(0, n, chunk))]
    if workers > 1 and len(jobs) > 1:
        import multiprocessing as mp
        from concurrent.futures import ProcessPoolExecutor
        with ProcessPoolExecutor(max_workers=min(workers, len(jobs)),
                                 mp_context=mp.get_context("spawn")) as ex:
            for (c, _, m, *_r), part in zip(jobs, ex.map(_world_chunk, jobs)):
                out[c * chunk:c * chunk + m] = part
    else:
        for (c, _, m, *_r) in jobs:
            out[c * chunk:c * chunk + m] = _world_chunk(jobs[c])
    return Instance(f"world-{n}-{gx}x{gy}x{gt}-hs{hs:g}-ht{ht:g}", out, gx, gy, gt, hs, ht)


def small_random_case(seed: int, max_g: int = 40, max_n: int = 300):
    """A randomised small problem for parity checks: odd grid sizes,
    non-integer bandwidths and origin, points inside, near and outside the
    grid edges.  Returns (points, dict of grid parameters)."""
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 7919 * (seed + 1)))
    gx, gy, gt = (int(v) for v in rng.integers(3, max_g + 1, 3))
    sres = float(rng.choice([1.0, 0.5, 2.0, 0.75]))
    tres = float(rng.choice([1.0, 0.5, 3.0, 1.25]))
    hs = float(rng.uniform(0.6, 9.0)) * sres
    ht = float(rng.uniform(0.6, 7.0)) * tres
    x0, y0, t0 = (float(v) for v in rng.uniform(-50, 50, 3))
    n = int(rng.integers(1, max_n + 1))
    lo = np.array([x0 - 1.5 * hs, y0 - 1.5 * hs, t0 - 1.5 * ht])
    hi = np.array([x0 + gx * sres + 1.5 * hs, y0 + gy * sres + 1.5 * hs, t0 + gt * tres + 1.5 * ht])
    pts = lo + rng.uniform(0, 1, (n, 3)) * (hi - lo)
    return pts, dict(gx=gx, gy=gy, gt=gt, hs=hs, ht=ht, sres=sres, tres=tres, x0=x0, y0=y0, t0=t0)


def adaptive_pairs(points: np.ndarray, gx: int, gy: int, hs: float, ht: float, sres: float = 1.0,
                   x0: float = 0.0, y0: float = 0.0, block: int = 16, floor: float = 0.25) -> np.ndarray:
    """Per-event bandwidth pairs that shrink where the events are dense (the
    adaptive bandwidth of Sec. 8, read as one pair per event): a pilot count
    c_i of the events in the event's block x block spatial cell (all times),
    lambda_i = sqrt(g / c_i) with g the geometric mean of the pilot counts,
    hs_i = hs * clip(lambda_i, floor, 1) and ht_i = ht * clip(sqrt(lambda_i),
    sqrt(floor), 1).  The largest pairs are (hs, ht).  Returns (n, 2) float64."""
    p = np.asarray(points, dtype=np.float64)
    nbx = max(1, -(-gx // block))
    nby = max(1, -(-gy // block))
    cx = np.clip(np.floor((p[:, 0] - x0) / (sres * block)), 0, nbx - 1).astype(np.int64)
    cy = np.clip(np.floor((p[:, 1] - y0) / (sres * block)), 0, nby - 1).astype(np.int64)
    counts = np.bincount(cx * nby + cy, minlength=nbx * nby).astype(np.float64)
    c = counts[cx * nby + cy]
    g = float(np.exp(np.mean(np.log(c))))
    lam = np.sqrt(g / c)
    out = np.empty((len(p), 2))
    out[:, 0] = hs * np.clip(lam, floor, 1.0)
    out[:, 1] = ht * np.clip(np.sqrt(lam), np.sqrt(floor), 1.0)
    return out
