"""Autotuner of the gather's tunables on gfx950.

What it searches, per plan (stkde_tuning):
  tile_t       time rows of an output tile (16, 32; 64 without Kahan),
  cell_xy, ct  bin edges in y and t (library default = bandwidth-sized; x bins are narrower),
  split_share  the work list's split threshold (a tile costlier than
               1/split_share of its grid's candidates is cut into parts).

The paper's discussion (Sec. 6.5) asks for a model that picks the best
strategy for an instance from its shape; this is the measured form of that
choice for the one strategy implemented here.  Entries are keyed by the
device architecture, the bandwidths in voxels (power-of-two buckets of
hs/sres and ht/tres), a density class (mean number of points whose cylinder
covers a voxel, in powers of 4), a grid-size class (voxels in powers of 4),
the accumulation mode and the gather's matrix-core operand form (keys of
gathers with FP32 operands -- per-point bandwidths, or operand_form = 1 --
end in "/fp32"; their costs differ enough to want other bins); each entry
stores the fastest measured tuning.  A lookup is deterministic: a given
description always resolves to the same pinned tuning, so results stay
bitwise repeatable.

Caches: ``tuned_gfx950.json`` beside this file is measured on an MI355X by
``python -m paper_1705_09366_amd.autotune --build-cache PATH`` over synthetic
workloads spanning the bandwidths and densities of the benchmark
configurations; a user cache (``STKDE_TUNE_CACHE`` or an explicit path) is
consulted first.
"""
import json
import math
import os
import sys
import time
from typing import Dict, List, Optional, Tuple

from . import Desc, Plan, Tuning, FLAG_ADAPTIVE, FLAG_KAHAN

ARCH = "gfx950"
HERE = os.path.dirname(os.path.abspath(__file__))
SHIPPED_CACHE = os.path.join(HERE, "tuned_gfx950.json")
CACHE_VERSION = 1


def _bucket(v: float) -> int:
    """Power-of-two bucket: 1 -> 0, 2 -> 1, (2,4] -> 2, (4,8] -> 3, ..."""
    return max(0, int(math.ceil(math.log2(max(float(v), 1.0)))))


def density(desc: Desc, n: int) -> float:
    """Mean number of points whose support cylinder covers a voxel, assuming
    the points lie in the grid: n * pi hv^2 * 2 tv / voxels."""
    hv, tv = desc.hs / desc.sres, desc.ht / desc.tres
    return n * math.pi * hv * hv * 2.0 * tv / float(desc.gx * desc.gy * desc.gt)


def density_class(desc: Desc, n: int) -> int:
    m = density(desc, n)
    return int(min(8, max(-4, round(math.log(max(m, 1e-6), 4.0)))))


def grid_class(desc: Desc) -> int:
    """Grid size in factors of 4 of voxels (2^22 -> 11, 2^28 -> 14)."""
    return int(round(math.log2(float(desc.gx * desc.gy * desc.gt)) / 2.0))


def fp32_operands(desc: Desc, fp32: bool = False) -> bool:
    """Whether the plan's gather takes FP32 matrix-core operands whatever its
    shape: asked for (operand_form = 1) or per-point bandwidths."""
    return bool(fp32 or (desc.flags & FLAG_ADAPTIVE))


def key(desc: Desc, n: int, fp32: bool = False) -> str:
    mode = "kahan" if desc.flags & FLAG_KAHAN else "plain"
    return (f"{ARCH}/hs{_bucket(desc.hs / desc.sres)}/ht{_bucket(desc.ht / desc.tres)}"
            f"/d{density_class(desc, n)}/g{grid_class(desc)}/{mode}"
            + ("/fp32" if fp32_operands(desc, fp32) else ""))


_LOADED: Dict[Tuple[str, int, int], Dict] = {}


def _load(path: str) -> Dict:
    """The entries of a cache file (parsed once per file version: a server
    looks up every request)."""
    if not path or not os.path.exists(path):
        return {}
    st = os.stat(path)
    k = (os.path.abspath(path), st.st_mtime_ns, st.st_size)
    entries = _LOADED.get(k)
    if entries is None:
        with open(path) as f:
            data = json.load(f)
        ok = data.get("version") == CACHE_VERSION and data.get("arch") == ARCH
        entries = data.get("entries", {}) if ok else {}
        _LOADED[k] = entries
    return entries


def _tuning(e, desc: Desc, fp32: bool) -> Tuning:
    tt, cxy, ct, ss = e["tuning"]
    if (desc.flags & FLAG_KAHAN) and tt > 32:
        tt = 32
    return Tuning(tt, cxy, ct, ss, 0, 1 if fp32 else 0)


def lookup(desc: Desc, n: int, cache: Optional[str] = None, fp32: bool = False) -> Optional[Tuning]:
    """The pinned tuning for (desc, n), or None when no cache covers it
    (fp32: for a plan with FP32 operands, which the tuning then asks for)."""
    k = key(desc, n, fp32)
    for path in (cache, os.environ.get("STKDE_TUNE_CACHE"), SHIPPED_CACHE):
        e = _load(path).get(k)
        if e is not None:
            return _tuning(e, desc, fp32)
    return None


def _parse_key(k: str):
    """(hs bucket, ht bucket, density class, grid class, mode, operand form) of
    a cache key."""
    parts = k.split("/")
    _, hs, ht, d, g, mode = parts[:6]
    form = parts[6] if len(parts) > 6 else "default"
    return int(hs[2:]), int(ht[2:]), int(d[1:]), int(g[1:]), mode, form


def resolve(desc: Desc, n: int, cache: Optional[str] = None, max_distance: float = 4.0,
            fp32: bool = False):
    """(tuning, source) for (desc, n): the entry of its own key; else the
    nearest entry of the same accumulation mode and operand form, by
    |d hs bucket| + |d ht bucket| + |d density class| + |d grid class| / 2
    (ties: the first key in sorted order), if within ``max_distance``; else
    (None, reason).  Deterministic, so results stay bitwise repeatable."""
    t = lookup(desc, n, cache, fp32)
    k = key(desc, n, fp32)
    if t is not None:
        return t, f"autotune {k}"
    hs, ht, d, g, mode, form = _parse_key(k)
    best, best_key = None, None
    for path in (cache, os.environ.get("STKDE_TUNE_CACHE"), SHIPPED_CACHE):
        entries = _load(path)
        for ek in sorted(entries):
            ehs, eht, ed, eg, emode, eform = _parse_key(ek)
            if emode != mode or eform != form:
                continue
            dist = abs(ehs - hs) + abs(eht - ht) + abs(ed - d) + 0.5 * abs(eg - g)
            if dist <= max_distance and (best is None or dist < best):
                best, best_key = dist, ek
        if best_key is not None:
            return _tuning(entries[best_key], desc, fp32), f"autotune nearest {best_key} (for {k})"
    return None, f"default (no cache entry near {k})"


def plan_for(desc: Desc, n: int, cache: Optional[str] = None) -> Plan:
    """A plan with the cached tuning for (desc, n), else the library's defaults."""
    return Plan(desc, lookup(desc, n, cache))


def measure(points, desc: Desc, tuning: Optional[Tuning], reps: int = 5) -> float:
    """Median milliseconds of one full stkde_compute (binning included) on
    the current stream, points already on the device."""
    import torch
    plan = Plan(desc, tuning)
    try:
        out = torch.empty((desc.gx, desc.gy, desc.gt), dtype=torch.float32, device=points.device)
        ws = plan.workspace(points.shape[0], points.device)
        plan.compute_into(points, out, workspace=ws)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(reps)]
        for a, b in ev:
            a.record()
            plan.compute_into(points, out, workspace=ws)
            b.record()
        torch.cuda.synchronize()
        ms = sorted(a.elapsed_time(b) for a, b in ev)
        return ms[len(ms) // 2]
    finally:
        plan.close()


def candidates_tile(desc: Desc) -> List[int]:
    return [16, 32] if desc.flags & FLAG_KAHAN else [16, 32, 64]


def tune(points, desc: Desc, reps: int = 5, log=None, operand_form: int = 0) -> Tuple[Tuning, float, List]:
    """Search: every (tile rows, bin edges) pair, then the split share of
    the best; returns (best tuning, its ms, every measurement)."""
    of = operand_form
    table = []

    def run(t: Tuning) -> float:
        try:
            ms = measure(points, desc, t, reps)
        except Exception as e:  # a tuning the plan refuses
            if log:
                log(f"  {t}: refused ({e})")
            return math.inf
        table.append(([t.tile_t, t.cell_xy, t.cell_t, t.split_share], ms))
        if log:
            log(f"  {t}: {ms:.3f} ms")
        return ms

    default_ms = measure(points, desc, Tuning(operand_form=of), reps)
    table.append(([0, 0, 0, 0], default_ms))
    if log:
        log(f"  library default: {default_ms:.3f} ms")
    hv, tv = desc.hs / desc.sres, desc.ht / desc.tres
    # y edges around the bandwidth (x bins are narrow whatever the y edge);
    # t edges of 8 voxels and about a half and a quarter of the window
    cell_opts = sorted({(c, d) for c in (12, 16, 20, 24, max(16, 8 * math.ceil(hv / 4)))
                        for d in (8, max(8, 4 * math.ceil(tv / 2)), max(8, 4 * math.ceil(tv / 4)))
                        if c <= 256 and d <= 256})
    # tile rows and bin edges together (the best edges depend on the rows)
    best, best_ms = None, math.inf
    for tt in candidates_tile(desc):
        for cxy, ct in [(0, 0)] + cell_opts:
            t = Tuning(tt, cxy, ct, 0, 0, of)
            ms = run(t)
            if ms < best_ms:
                best, best_ms = t, ms
    for ss in (512, 8192):
        t = Tuning(best.tile_t, best.cell_xy, best.cell_t, ss, 0, of)
        ms = run(t)
        if ms < best_ms:
            best, best_ms = t, ms
    return best, best_ms, table


def tuning_workloads():
    """Synthetic workloads spanning the benchmark bandwidths and densities
    (yielded one at a time): clustered sets (the benchmark generator with
    other seeds) on 256^2 x 64, 512^2 x 365 and 1024^2 x 256 grids,
    hs 3..50, ht 2..30 voxels (ht about 0.6 hs, and the short windows of
    the world-scale pairs, hs 10 / ht 3 and hs 30 / ht 5), n 20k..1M."""
    import workloads
    rng = workloads.rng_for(90)
    shapes = [(256, 256, 64), (512, 512, 365), (1024, 1024, 256)]
    for gx, gy, gt in shapes:
        for hs, ht in ((3.0, 2.0), (5.0, 4.0), (10.0, 7.0), (20.0, 14.0), (30.0, 20.0), (50.0, 30.0),
                       (10.0, 3.0), (30.0, 5.0)):
            for n in (20_000, 200_000, 1_000_000):
                pts = workloads.clustered(rng, 64 if n >= 200_000 else 16, n, gx, gy, gt)
                yield (f"tune-{n}-{gx}x{gy}x{gt}-hs{hs:g}-ht{ht:g}", pts,
                       Desc(gx=gx, gy=gy, gt=gt, hs=hs, ht=ht))


def build_cache(path: str, kahan_modes=(True, False), reps: int = 5, log=print, forms=(0, 1),
                merge: Optional[str] = None):
    """Tune every synthetic workload and write the cache (fastest per key),
    for each operand form in ``forms`` (0 the default, 1 FP32).  With
    ``merge``, the entries of that cache whose keys this run does not tune
    are kept."""
    import torch
    entries: Dict[str, Dict] = {}
    tuned = set()
    for name, pts, d0 in tuning_workloads():
        dev_pts = torch.from_numpy(pts).cuda()
        for kahan, form in ((k_, f_) for k_ in kahan_modes for f_ in forms):
            desc = Desc(**{**d0.__dict__, "flags": FLAG_KAHAN if kahan else 0})
            k = key(desc, len(pts), fp32=form == 1)
            tuned.add(k)
            log(f"[tune] {name} kahan={kahan} operand_form={form} -> {k}")
            best, ms, table = tune(dev_pts, desc, reps, log, form)
            base = table[0][1]  # the library's default tuning
            prev = entries.get(k)
            # a key seen twice keeps the tuning with the larger gain
            gain = base / ms if ms > 0 else 1.0
            if prev is None or gain > prev["gain"]:
                entries[k] = {"tuning": [best.tile_t, best.cell_xy, best.cell_t, best.split_share],
                              "ms": ms, "gain": gain, "workload": name, "default_ms": base}
        del dev_pts
        torch.cuda.empty_cache()
    if merge:
        for k, e in _load(merge).items():
            if k not in tuned:
                entries[k] = e
    data = {"version": CACHE_VERSION, "arch": ARCH,
            "made": time.strftime("%Y-%m-%d"), "entries": entries}
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    return data


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="tune the gather on this GPU")
    ap.add_argument("--build-cache", metavar="PATH", required=True)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--kahan-only", action="store_true", help="tune the compensated keys only")
    ap.add_argument("--forms", default="0,1", help="operand forms to tune (0 two-term, 1 FP32)")
    ap.add_argument("--merge", metavar="PATH", help="keep this cache's entries for keys not tuned")
    a = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    build_cache(a.build_cache, kahan_modes=(True,) if a.kahan_only else (True, False), reps=a.reps,
                log=lambda m: print(m, flush=True), forms=tuple(int(f) for f in a.forms.split(",")),
                merge=a.merge)
