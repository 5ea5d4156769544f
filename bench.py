#!/usr/bin/env python3
"""Benchmark of the space-time kernel density hot path on one MI355X.

One step = one full density estimate of the workload through the C ABI
(stkde_compute: FP64 transform and binning, stable radix sort, per-point
tables, gather/accumulate, single FP32 store of every voxel, fused FP64 grid
mass), with the points already resident in HBM.

Default workload: 1,000,000 clustered events (64-component Gaussian mixture
in space, 8 seasonal bumps plus 20 % uniform background in time) on a
1024 x 1024 x 256 grid (1 GiB FP32), hs = 10, ht = 7 voxels -- a synthetic
stand-in shaped like the paper's social-media workload (Sec. 6.1; no dataset
is available here).

Prints ONE JSON line:
  value            kernel evaluations per second = exact in-grid
                   (voxel, point) pairs inside both supports / step time
  roofline         the gather kernel (dominant) against the roofline that
                   binds the workload: HBM (algorithmic bytes = grid written
                   once + points read once) when 2 flops per evaluation per
                   byte is below the ridge point, else FP32 matrix cores
                   (2 flops per evaluation); over its average duration in the
                   timed steps, from HIP events that the library records
                   around that launch on its stream
  cpu_baseline     the FP64 CPU oracle on a bounded sample of the same
                   workload, on this host's cores
"""
import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_F32_PEAK_TFLOPS = 157.3  # dense FP32 matrix-core peak of MI355X
KERNELS = ("epanechnikov", "quartic", "gaussian", "printed")
WORKLOADS = ("clustered-1M", "clustered-200k-hs50", "uniform-10k", "world-Hr-Hb", "world-Hr-Lb",
             "world-Lr-Hb", "world-Lr-Lb")


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _operand_form(inst, tuning, kahan, adaptive, kern):
    """Matrix-core operands of the gather, by the library's rule: two FP16
    terms with one bandwidth pair and 16- or 32-row tiles, unless the tuning
    asks for FP32; with the full-cover path (Epanechnikov pair with
    hs / sres >= 14) only at 16 rows and only for the points that reach a
    tile in part (the covering points keep FP32 separable sums)."""
    import math
    tt = tuning.tile_t if tuning and tuning.tile_t else (32 if math.ceil(inst.ht / inst.tres) <= 12 else 16)
    if kahan or kern != 0:
        tt = min(tt, 32)
    full = kern == 0 and inst.hs / inst.sres >= 14.0
    fp32 = (tuning is not None and tuning.operand_form == 1) or adaptive or tt > 32 or (full and tt != 16)
    if fp32:
        return "fp32"
    if full:
        return "fp16 hi+lo (points reaching a tile in part), fp32 (tile- and quadrant-cover sums), fp32 accumulate"
    return "fp16 hi+lo, fp32 accumulate"


def _instance(name):
    import workloads
    if name == "clustered-1M":
        return workloads.config1()
    if name == "clustered-200k-hs50":
        return workloads.config2()
    if name == "uniform-10k":
        return workloads.config0()
    if name.startswith("world-"):
        res, bw = name.split("-")[1:]
        t0 = time.perf_counter()
        inst = workloads.world_scale(res, bw, workers=min(16, _cpu_threads()))
        _log(f"generated {inst.name} in {time.perf_counter() - t0:.1f} s")
        return inst
    raise SystemExit(f"unknown workload {name}; choose from {WORKLOADS}")


def _cpu_threads():
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return n


def profiled_sources_hash():
    """SHA-256 of what shapes the gather's launches and memory traffic: every
    source file of the library (sorted by name) and the tuning cache."""
    csrc = os.path.join(ROOT, "paper_1705_09366_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h", ".inc")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    h.update(open(os.path.join(ROOT, "paper_1705_09366_amd", "tuned_gfx950.json"), "rb").read())
    return h.hexdigest()


def _traffic_from_profile(sources_hash):
    """HBM bytes per launch of the gather kernel from a committed rocprofv3
    counter summary, if it was taken on the current sources and tunings."""
    path = os.path.join(ROOT, "profiles", "gather_clustered1M_pmc.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except Exception:
        return None
    if rec.get("src_sha256") != sources_hash:
        return None
    return rec.get("hbm_bytes_per_launch")


def cpu_baseline(inst, budget_s=20.0, pairs=None, kernel=0, corner=False):
    """Time the FP64 oracle on a bounded sample (the first k events of the
    workload on the full grid, with their bandwidth pairs when the workload
    has per-event bandwidths), growing k until the run takes a few seconds
    or covers the whole workload.  Returns the record, the oracle's grid and
    k (the caller compares the GPU on the same sample)."""
    import oracle
    g = oracle.Grid(gx=inst.gx, gy=inst.gy, gt=inst.gt, hs=inst.hs, ht=inst.ht,
                    sres=inst.sres, tres=inst.tres, x0=inst.x0, y0=inst.y0, t0=inst.t0,
                    kernel=kernel, corner=corner)
    n = inst.points.shape[0]
    th = _cpu_threads()
    k = max(1, n // 64)
    while True:
        t0 = time.perf_counter()
        if pairs is None:
            ref, evals = oracle.pbsym(inst.points[:k], g, nthreads=th)
        else:
            ref, evals = oracle.pbsym_adaptive(inst.points[:k], pairs[:k], g, nthreads=th)
        dt = time.perf_counter() - t0
        _log(f"cpu oracle: {k} points, {evals} evals, {dt:.2f} s on {th} threads")
        if k >= n or dt * min(4, n / k) > budget_s:
            break
        k = min(n, k * 4)
    sample = (f"first {k} of {n} events of the workload on the full {inst.gx}x{inst.gy}x{inst.gt} "
              f"grid (FP64 grid zeroing + PB-SYM accumulation"
              f"{' with per-event bandwidths' if pairs is not None else ''}, IO excluded)")
    model, ncpu = cpu_info()
    return ({"value": evals / dt, "unit": "evals/s", "cores": th, "kind": "oracle",
             "sample": sample, "seconds": round(dt, 3), "evals": int(evals), "cpu_model": model,
             "host_cpus": ncpu}, ref, k)


def cpu_baseline_window(inst, out, budget_s=20.0, kernel=0, corner=False):
    """The FP64 oracle on a bounded sample of a grid too large for host memory
    in FP64: a window of the grid (all times, a square in space around the
    densest spatial cell) with the events that can reach it, the window
    doubling in area until the run takes a few seconds.  Dividing by the
    whole n makes the window's density the cut-out of the full grid, which is
    compared with the same cut-out of the GPU's grid ``out``."""
    import numpy as np
    import oracle
    p = inst.points
    th = _cpu_threads()
    cell = 64
    h, xe, ye = np.histogram2d(p[:, 0], p[:, 1], bins=[max(1, inst.gx // cell), max(1, inst.gy // cell)],
                               range=[[0, inst.gx], [0, inst.gy]])
    ci, cj = np.unravel_index(int(np.argmax(h)), h.shape)
    cx, cy = int(xe[ci] + cell / 2), int(ye[cj] + cell / 2)
    w = 32
    while True:
        x0 = max(0, min(inst.gx - w, cx - w // 2))
        y0 = max(0, min(inst.gy - w, cy - w // 2))
        wx, wy = min(w, inst.gx), min(w, inst.gy)
        reach = inst.hs + 2.0
        sel = ((p[:, 0] > x0 - reach) & (p[:, 0] < x0 + wx + reach) &
               (p[:, 1] > y0 - reach) & (p[:, 1] < y0 + wy + reach))
        sub = np.ascontiguousarray(p[sel])
        g = oracle.Grid(gx=wx, gy=wy, gt=inst.gt, hs=inst.hs, ht=inst.ht, x0=float(x0), y0=float(y0),
                        kernel=kernel, corner=corner)
        t0 = time.perf_counter()
        ref, evals = oracle.pbsym(sub, g, nthreads=th)
        dt = time.perf_counter() - t0
        _log(f"cpu oracle: window {wx}x{wy}x{inst.gt} at ({x0}, {y0}), {len(sub)} events, {evals} evals, "
             f"{dt:.2f} s on {th} threads")
        if dt * 2 > budget_s or (wx == inst.gx and wy == inst.gy) or w >= 1024:
            break
        w *= 2
    ref *= len(sub) / float(len(p))
    gpu = out[x0:x0 + wx, y0:y0 + wy, :].cpu().numpy().astype(np.float64)
    err = float(np.max(np.abs(gpu - ref)) / max(np.max(np.abs(ref)), 1e-300))
    sample = (f"window {wx}x{wy}x{inst.gt} voxels at ({x0}, {y0}) around the densest region, "
              f"{len(sub)} of {len(p)} events (those within reach); FP64 PB-SYM with the whole n, "
              f"IO excluded")
    model, ncpu = cpu_info()
    return {"value": evals / dt, "unit": "evals/s", "cores": th, "kind": "oracle", "sample": sample,
            "seconds": round(dt, 3), "evals": int(evals), "cpu_model": model, "host_cpus": ncpu}, err


def _median(v):
    v = sorted(v)
    return v[len(v) // 2]


def bench_batch(args, dev):
    """Bandwidth sweep (8 point sets x 8 bandwidth pairs = 64 grids).
    Baseline: 64 stkde_compute calls in sequence on one stream, each binning
    its own points.  Candidate: the 8 sets binned once each, then one batch
    (one work list, one gather launch per tile group) replayed from a HIP
    graph.  Both steps are timed with events around the whole sequence."""
    import numpy as np
    import torch
    import workloads
    import paper_1705_09366_amd as m
    from paper_1705_09366_amd import autotune
    insts = workloads.config3_sets()
    kahan = not args.plain
    flags = m.FLAG_KAHAN if kahan else 0
    by_set = {}
    for it in insts:
        by_set.setdefault(it.meta["set"], []).append(it)
    pts = {k: torch.from_numpy(v[0].points).to(dev) for k, v in by_set.items()}
    outs_a = [torch.empty((i.gx, i.gy, i.gt), dtype=torch.float32, device=dev) for i in insts]
    outs_b = [torch.empty_like(o) for o in outs_a]
    descs = [m.Desc(gx=i.gx, gy=i.gy, gt=i.gt, hs=i.hs, ht=i.ht, flags=flags) for i in insts]
    n_of = [i.points.shape[0] for i in insts]
    plans = [m.Plan(d, autotune.lookup(d, n) if args.tuning == "auto" else None)
             for d, n in zip(descs, n_of)]
    ws_bytes = max(p.workspace_bytes(n) for p, n in zip(plans, n_of))
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=dev)
    # exact evaluation counts, once
    evals = 0
    st = torch.zeros(8, dtype=torch.float64, device=dev)
    for i, d, o in zip(insts, descs, outs_a):
        c = m.Plan(m.Desc(**{**d.__dict__, "flags": m.FLAG_POINT_STATS}))
        c.compute_into(pts[i.meta["set"]], o, stats=st, workspace=ws)
        torch.cuda.synchronize()
        evals += int(st[2].item())
        c.close()
    _log(f"batch workload: {len(insts)} grids over {len(by_set)} sets, {evals} evals")

    def baseline():
        for i, p, o in zip(insts, plans, outs_a):
            p.compute_into(pts[i.meta["set"]], o, workspace=ws)

    # candidate: sets binned for the largest bandwidths of their instances
    sets, items = {}, []
    rows = {}
    for i, p in zip(insts, plans):
        tt = p.tuning.tile_t if (p.tuning and p.tuning.tile_t) else 32
        rows[i.meta["set"]] = max(rows.get(i.meta["set"], 16), tt)
    for k, lst in by_set.items():
        i0 = lst[0]
        base = m.Desc(gx=i0.gx, gy=i0.gy, gt=i0.gt, hs=max(i.hs for i in lst), ht=max(i.ht for i in lst))
        sets[k] = m.BinnedSet(base, i0.points.shape[0], m.Tuning(tile_t=rows[k]))
    scratch = torch.empty(max(s.scratch_bytes for s in sets.values()) + 256, dtype=torch.uint8, device=dev)
    for k, s in sets.items():
        s.build(pts[k], scratch=scratch)
    for i, p, o in zip(insts, plans, outs_b):
        items.append(m.Item(plan=p, set=sets[i.meta["set"]], out=o))
    batch = m.Batch(items)
    batch.capture()

    def candidate():
        for k, s in sets.items():
            s.build(pts[k], scratch=scratch)
        batch.replay()

    res = {}
    for name, fn in (("sequential", baseline), ("batched", candidate)):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        res[name] = _median(ts)
        _log(f"{name}: median {res[name]:.3f} ms over {args.steps}")
    torch.cuda.synchronize()
    diff = 0.0
    for oa, ob in zip(outs_a, outs_b):
        sc = float(oa.abs().max())
        if sc > 0:
            diff = max(diff, float((oa - ob).abs().max()) / sc)
    # every grid of both forms against the FP64 oracle on its whole grid
    import oracle
    th = _cpu_threads()
    errs = {"sequential": [], "batched": []}
    t0 = time.perf_counter()
    for i, oa, ob in zip(insts, outs_a, outs_b):
        ref, _ = oracle.pbsym(i.points, oracle.Grid(gx=i.gx, gy=i.gy, gt=i.gt, hs=i.hs, ht=i.ht), nthreads=th)
        errs["sequential"].append(error_stats(oa.cpu().numpy(), ref))
        errs["batched"].append(error_stats(ob.cpu().numpy(), ref))
        del ref
    odt = time.perf_counter() - t0
    vs_oracle = {k: {"max_rel_err": max(e["max_rel"] for e in v), "max_rms_rel_err": max(e["rms_rel"] for e in v),
                     "support_mismatch": sum(e["mismatch"] for e in v), "grids": len(v)}
                 for k, v in errs.items()}
    _log(f"oracle on all {len(insts)} grids in {odt:.1f} s: sequential max {vs_oracle['sequential']['max_rel_err']:.3e}, "
         f"batched max {vs_oracle['batched']['max_rel_err']:.3e}")
    rec = {"metric": "bandwidth-sweep makespan", "value": res["batched"], "unit": "ms",
           "higher_is_better": False, "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": "sweep-8sets-x8bw", "grids": len(insts), "evals": evals,
                      "accumulation": "kahan" if kahan else "plain", "tuning": args.tuning},
           "sequential_ms": res["sequential"], "batched_ms": res["batched"],
           "speedup": res["sequential"] / res["batched"],
           "evals_per_s": {"sequential": evals / (res["sequential"] * 1e-3),
                           "batched": evals / (res["batched"] * 1e-3)},
           "max_rel_diff_batched_vs_sequential": diff,
           "vs_oracle": vs_oracle, "oracle_seconds": round(odt, 2)}
    print(json.dumps(rec), flush=True)


def bench_serve(args, dev):
    """Serving: 4 resident sets (100k..2M points over a 2048 x 2048 x 512
    domain), requests for windows of 64..1024 x 64..1024 x 64..128 voxels
    at hs, ht in [3, 40].  First the saturation rate of the batching server
    (all requests at once); then Poisson arrivals at 0.25..0.9 of it, for
    the batching server and for one-request-at-a-time launches."""
    import numpy as np
    import torch
    import workloads
    import paper_1705_09366_amd as m
    from paper_1705_09366_amd.serve import GpuExecutor, Request, Server
    sets = workloads.config4_sets()
    ex = GpuExecutor(device=dev)
    names = []
    for k, inst in enumerate(sets):
        base = m.Desc(gx=inst.gx, gy=inst.gy, gt=inst.gt, hs=40.0, ht=40.0)
        ex.add_set(f"s{k}", torch.from_numpy(inst.points).to(dev), base, m.Tuning(tile_t=16))
        names.append(f"s{k}")
    resident = sum(s.set_bytes for s in ex.sets.values())
    nreq = args.requests
    raw = workloads.config4_requests(nreq + 100)

    def mk(r):
        return Request(set=names[r["set"]], gx=r["gx"], gy=r["gy"], gt=r["gt"], ox=int(r["x0"]),
                       oy=int(r["y0"]), ot=int(r["t0"]), hs=r["hs"], ht=r["ht"])
    reqs = [mk(r) for r in raw]
    warm, reqs = reqs[:100], reqs[100:]

    def serve(requests, rate, batching, keep=()):
        """Serve `requests` (Poisson arrivals at `rate`, or all at once); the
        outputs of the requests whose positions are in `keep` are returned."""
        srv = Server(executor=ex, max_batch=256 if batching else 1, max_inflight=2 if batching else 1)
        srv.resident = resident
        rng = np.random.default_rng(170509366 + int(rate * 1000))
        t0 = time.perf_counter()
        arr = t0 + (np.cumsum(rng.exponential(1.0 / rate, len(requests))) if rate else np.zeros(len(requests)))
        i = 0
        vox = 0
        kept, tks = {}, []
        while i < len(requests) or not srv.idle():
            now = time.perf_counter()
            while i < len(requests) and arr[i] <= now:
                tks.append(srv.submit(requests[i], t_arrival=float(arr[i])))
                i += 1
            srv.poll()
            for tk in srv.finished:
                if tk.charged:
                    vox += tk.out.numel()
                    if tk.rid - tks[0].rid in keep:
                        kept[tk.rid - tks[0].rid] = tk.out
                    srv.release(tk)
        dt = time.perf_counter() - t0
        st = srv.latency_stats()
        st.update({"requests_per_s": len(requests) / dt, "voxels_per_s": vox / dt, "seconds": dt,
                   "failed": len(srv.failed)})
        return st, kept

    serve(warm, 0, True)
    # 32 sampled requests of the saturation run are kept for the oracle
    sample = sorted(int(v) for v in np.random.default_rng(170509366).choice(len(reqs), 32, replace=False))
    sat, kept = serve(reqs, 0, True, keep=set(sample))
    rate_sat = sat["requests_per_s"]
    _log(f"saturation: {rate_sat:.1f} req/s ({sat['ticks']} ticks)")
    levels = []
    for frac in (0.25, 0.5, 0.75, 0.9):
        lam = frac * rate_sat
        b, _ = serve(reqs, lam, True)
        f, _ = serve(reqs, lam, False)
        _log(f"load {frac:.2f} ({lam:.1f} req/s): batched p50 {b['p50_ms']:.2f} p99 {b['p99_ms']:.2f} ms; "
             f"one-at-a-time p50 {f['p50_ms']:.2f} p99 {f['p99_ms']:.2f} ms")
        levels.append({"load": frac, "rate": lam, "batched": b, "one_at_a_time": f})
    # the sampled requests against the FP64 oracle on their windows (whole set n)
    import oracle
    th = _cpu_threads()
    t0 = time.perf_counter()
    worst, worst_rms, mism = 0.0, 0.0, 0
    for j in sample:
        r = reqs[j]
        inst = sets[names.index(r.set)]
        ref, _ = oracle.pbsym(inst.points, oracle.Grid(gx=r.gx, gy=r.gy, gt=r.gt, hs=r.hs, ht=r.ht,
                                                       x0=float(r.ox), y0=float(r.oy), t0=float(r.ot)),
                              nthreads=th)
        got = kept[j].cpu().numpy()
        if float(np.max(ref)) > 0.0:
            e = error_stats(got, ref)
            worst, worst_rms, mism = max(worst, e["max_rel"]), max(worst_rms, e["rms_rel"]), mism + e["mismatch"]
        elif np.any(got):
            worst = float("inf")
        del ref
    odt = time.perf_counter() - t0
    _log(f"oracle on {len(sample)} sampled requests in {odt:.1f} s: max rel err {worst:.3e}")
    rec = {"metric": "serve saturation rate", "value": rate_sat, "unit": "requests/s",
           "higher_is_better": True, "n_gpus": 1, "data": "synthetic", "dtype": "f32",
           "config": {"workload": "serve-4sets-2048x2048x512", "requests": nreq,
                      "resident_bytes": resident},
           "saturation": sat, "levels": levels,
           "vs_oracle": {"requests": len(sample), "max_rel_err": worst, "max_rms_rel_err": worst_rms,
                         "support_mismatch": mism, "seconds": round(odt, 2)}}
    print(json.dumps(rec), flush=True)


def bench_ablation(args, dev):
    """The production gather against the two baselines of stkde_ablation.h
    (point-parallel atomic scatter, Alg. PB; voxel-parallel gather over
    bins, VB-DEC) on the workloads named in --ablation-workloads.  Each
    method's step is bin + accumulate through the C ABI, timed with events
    (median); the accumulation stage alone is timed after one binning.
    Accuracy is the max difference from the Kahan gather (which the parity
    tests hold to the oracle) relative to its max; repeatability counts the
    voxels that differ between two runs of the same method."""
    import torch
    import paper_1705_09366_amd as m
    from paper_1705_09366_amd import autotune
    names = [w for w in args.ablation_workloads.split(",") if w]
    results = []
    for wname in names:
        inst = _instance(wname)
        n = inst.points.shape[0]
        pts = torch.from_numpy(inst.points).to(dev)
        base = dict(gx=inst.gx, gy=inst.gy, gt=inst.gt, hs=inst.hs, ht=inst.ht, sres=inst.sres,
                    tres=inst.tres, x0=inst.x0, y0=inst.y0, t0=inst.t0)
        dk, dp = m.Desc(**base, flags=m.FLAG_KAHAN), m.Desc(**base)
        pk = m.Plan(dk, autotune.lookup(dk, n) if args.tuning == "auto" else None)
        pp = m.Plan(dp, autotune.lookup(dp, n) if args.tuning == "auto" else None)
        ws = torch.empty(max(pk.workspace_bytes(n), pp.workspace_bytes(n)) + 256, dtype=torch.uint8,
                         device=dev)
        ref = torch.empty((inst.gx, inst.gy, inst.gt), dtype=torch.float32, device=dev)
        out = torch.empty_like(ref)
        st = torch.zeros(8, dtype=torch.float64, device=dev)
        c = m.Plan(m.Desc(**base, flags=m.FLAG_POINT_STATS))
        c.compute_into(pts, out, stats=st, workspace=ws)
        torch.cuda.synchronize()
        evals = int(st[2].item())
        c.close()
        pk.compute_into(pts, ref, workspace=ws)
        torch.cuda.synchronize()
        scale = float(ref.abs().max())
        _log(f"ablation {inst.name}: n={n}, {evals} evals")

        methods = {
            "gather_kahan": (lambda o: pk.compute_into(pts, o, workspace=ws),
                             lambda o: pk.accumulate(n, o, ws)),
            "gather_plain": (lambda o: pp.compute_into(pts, o, workspace=ws),
                             lambda o: pp.accumulate(n, o, ws)),
            "scatter": (lambda o: pp.ablation_compute(m.ABLATION_SCATTER, pts, o),
                        lambda o: pp.ablation_accumulate(m.ABLATION_SCATTER, n, o, pp.workspace(n, dev))),
            "voxel": (lambda o: pp.ablation_compute(m.ABLATION_VOXEL, pts, o),
                      lambda o: pp.ablation_accumulate(m.ABLATION_VOXEL, n, o, pp.workspace(n, dev))),
        }

        def timed(fn, steps):
            ts = []
            for _ in range(steps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                fn(out)
                b.record()
                torch.cuda.synchronize()
                ts.append(a.elapsed_time(b))
            return _median(ts)

        rows = {}
        for meth, (step, acc) in methods.items():
            first = timed(step, 1)  # also the warm-up
            steps = args.steps if first < 50.0 else max(2, min(args.steps, int(2000.0 / first)))
            step_ms = timed(step, steps)
            if meth in ("scatter", "voxel"):
                pp.bin(pts, pp.workspace(n, dev))
            else:
                (pk if meth == "gather_kahan" else pp).bin(pts, ws)
            acc_ms = timed(acc, steps)
            step(out)
            torch.cuda.synchronize()
            err = float((out - ref).abs().max()) / scale if scale > 0 else 0.0
            again = out.clone()
            step(out)
            torch.cuda.synchronize()
            ndiff = int((out != again).sum())
            del again
            rows[meth] = {"step_ms": step_ms, "accumulate_ms": acc_ms, "steps": steps,
                          "evals_per_s": evals / (step_ms * 1e-3), "max_rel_diff_vs_gather_kahan": err,
                          "voxels_differing_between_runs": ndiff}
            _log(f"  {meth}: step {step_ms:.3f} ms, accumulate {acc_ms:.3f} ms, "
                 f"diff vs kahan gather {err:.2e}, {ndiff} voxels differ between runs")
        g = rows["gather_kahan"]["step_ms"]
        for meth in ("scatter", "voxel"):
            rows[meth]["gather_speedup"] = rows[meth]["step_ms"] / g
        results.append({"workload": inst.name, "n": n, "evals": evals, "methods": rows})
        pk.close()
        pp.close()
        del pts, ws, ref, out
        torch.cuda.empty_cache()
    rec = {"metric": "ablation step time", "unit": "ms", "higher_is_better": False, "n_gpus": 1,
           "dtype": "f32", "data": "synthetic", "config": {"workload": "ablation", "tuning": args.tuning},
           "results": results}
    print(json.dumps(rec), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="clustered-1M", choices=WORKLOADS)
    ap.add_argument("--plain", action="store_true", help="plain FP32 accumulation (no Kahan)")
    ap.add_argument("--kernel", default="epanechnikov", choices=KERNELS,
                    help="kernel pair (Epanechnikov is the default reading of Sec. 2.1)")
    ap.add_argument("--corner", action="store_true", help="sample voxels at their lower corners")
    ap.add_argument("--adaptive", action="store_true",
                    help="per-event bandwidth pairs shrinking with the local event density "
                         "(the workload's hs, ht are the largest)")
    ap.add_argument("--fp32-operands", action="store_true",
                    help="FP32 matrix-core operands in the gather (default: two FP16 terms where it has them)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload only: skip the FP32-operand run and the nested "
                         "uniform-10k and clustered-200k-hs50 records")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--tile-t", type=int, default=0, help="tuning: time rows per tile (16/32)")
    ap.add_argument("--cell-xy", type=int, default=0, help="tuning: bin edge in y (x bins are narrower)")
    ap.add_argument("--cell-t", type=int, default=0, help="tuning: bin edge in t")
    ap.add_argument("--tuning", default="auto", choices=("auto", "default"),
                    help="auto: the autotune cache's pinned tuning for the workload (when it has "
                         "one); default: the library defaults (explicit --tile-t etc. override both)")
    ap.add_argument("--mode", default="compute", choices=("compute", "batch", "serve", "ablation"),
                    help="compute: the headline step; batch: the bandwidth-sweep batch against "
                         "sequential computes; serve: request latency under Poisson load; "
                         "ablation: the gather against the atomic scatter and voxel baselines")
    ap.add_argument("--ablation-workloads", default="uniform-10k,clustered-1M,clustered-200k-hs50",
                    help="ablation mode: comma-separated workloads")
    ap.add_argument("--requests", type=int, default=400, help="serve mode: requests per load level")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the library runs on one GPU; sharding the output into per-GPU slabs is "
              "not implemented. Run with --gpus 1.", file=sys.stderr, flush=True)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1705_09366_amd as m

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    m.lib()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.mode == "batch":
        return bench_batch(args, dev)
    if args.mode == "serve":
        return bench_serve(args, dev)
    if args.mode == "ablation":
        return bench_ablation(args, dev)

    if args.calibrate_copy:
        # a plain copy kernel of known size: 1 GiB read + 1 GiB written per launch
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read_per_launch": src.numel() * 4,
                          "bytes_written_per_launch": dst.numel() * 4, "launches": 3}), flush=True)
        return

    inst = _instance(args.workload)
    n = inst.points.shape[0]
    kahan = not args.plain
    kern = KERNELS.index(args.kernel)
    flags = m.FLAG_MASS | (m.FLAG_KAHAN if kahan else 0) | (m.FLAG_ADAPTIVE if args.adaptive else 0) \
        | m.kernel_flag(kern) | (m.FLAG_CORNER if args.corner else 0)
    pairs_np = None
    if args.adaptive:
        import workloads
        pairs_np = workloads.adaptive_pairs(inst.points, inst.gx, inst.gy, inst.hs, inst.ht, inst.sres,
                                            inst.x0, inst.y0)
    desc = _desc_of(m, inst, flags)
    if args.tile_t or args.cell_xy or args.cell_t:
        tuning, tuning_src = m.Tuning(args.tile_t, args.cell_xy, args.cell_t), "manual"
    elif args.tuning == "auto":
        from paper_1705_09366_amd import autotune
        tuning, tuning_src = autotune.resolve(desc, n, fp32=args.fp32_operands)
    else:
        tuning, tuning_src = None, "default"
    if args.fp32_operands:
        tuning = dataclasses.replace(tuning or m.Tuning(), operand_form=1)
    operands = _operand_form(inst, tuning, kahan, args.adaptive, kern)
    pts = torch.from_numpy(inst.points).to(dev)
    pairs = torch.from_numpy(pairs_np).to(dev) if args.adaptive else None
    _log(f"workload {inst.name}: n={n}, grid {inst.gx}x{inst.gy}x{inst.gt}, kahan={kahan}")
    run = time_compute(m, desc, tuning, pts, pairs, args.steps, args.warmup, stages=True)
    evals, out = run["evals"], run["out"]
    grid_bytes = inst.gx * inst.gy * inst.gt * 4
    alg_bytes = grid_bytes + n * (40 if args.adaptive else 24)  # points (and pairs) read once
    roof = _roofline(alg_bytes, 2.0 * evals, run["gather_ms"])
    # the counters hold for the sources and tunings they were taken on, and
    # for the workload they were taken on (the default run)
    profiled = (args.workload == "clustered-1M" and kahan and not args.adaptive and kern == 0 and not args.corner
                and tuning_src.startswith("autotune") and not args.fp32_operands)
    traffic = _traffic_from_profile(profiled_sources_hash()) if profiled else None
    if roof["bound"] == "hbm":
        roof["traffic"] = traffic
    value = evals / (run["ms_per_step"] * 1e-3)
    rec = {
        "metric": "voxel-point kernel evals/s",
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": inst.name, "n": n, "grid": [inst.gx, inst.gy, inst.gt],
                   "hs": inst.hs, "ht": inst.ht, "accumulation": "kahan" if kahan else "plain",
                   "bandwidths": "per-event (density-adaptive)" if args.adaptive else "fixed",
                   "kernel": args.kernel, "sampling": "corner" if args.corner else "centre",
                   "operands": operands, "evals": evals,
                   "tuning": ([tuning.tile_t, tuning.cell_xy, tuning.cell_t, tuning.split_share]
                              if tuning else [0, 0, 0, 0]),
                   "tuning_source": tuning_src},
        "roofline": roof,
        "stage_ms": {"bin": run["bin_ms"], "pass": run["pass_ms"], "gather_kernel": run["gather_ms"],
                     "median_step_event": run["median_step_ms"]},
        "mass": {"grid": run["grid_mass"], "points": run["point_mass"]},
    }
    headline_default = (args.workload == "clustered-1M" and not args.adaptive and kern == 0 and not args.corner)

    if not args.no_cpu_baseline and args.workload.startswith("world-"):
        cb, err = cpu_baseline_window(inst, out, args.cpu_budget, kern, args.corner)
        rec["cpu_baseline"] = cb
        rec["max_rel_err_vs_oracle"] = err
        _log(f"gpu vs oracle on the window: max rel err {err:.3e}")
    elif not args.no_cpu_baseline:
        def gpu_sample(k, tun=tuning):
            sp = m.Plan(m.Desc(**{**desc.__dict__, "flags": flags & ~m.FLAG_MASS}), tun)
            xs = torch.from_numpy(np.ascontiguousarray(inst.points[:k])).to(dev)
            if args.adaptive:
                o = sp.compute_adaptive(xs, torch.from_numpy(np.ascontiguousarray(pairs_np[:k])).to(dev))
            else:
                o = sp(xs)
            torch.cuda.synchronize()
            r = o.cpu().numpy()
            sp.close()
            return r
        cb, ref, k = cpu_baseline(inst, args.cpu_budget, pairs_np, kern, args.corner)
        est = error_stats(gpu_sample(k), ref)
        rec["cpu_baseline"] = cb
        rec["max_rel_err_vs_oracle"] = est["max_rel"]
        rec["rms_rel_err_vs_oracle"] = est["rms_rel"]
        rec["support_mismatch"] = est["mismatch"]
        _log(f"gpu vs oracle on the cpu sample: max rel err {est['max_rel']:.3e}, rms {est['rms_rel']:.3e}, "
             f"support mismatch {est['mismatch']}")
        if headline_default and not args.no_extras:
            rec["precision"] = precision_record(m, inst, desc, tuning, pts, operands, est, ref, k, gpu_sample,
                                                args)
        del ref
        if headline_default:
            cb["single_thread"] = cpu_single_thread(inst, min(n, 62_500))
    if headline_default and not args.no_extras:
        del out
        run = None
        torch.cuda.empty_cache()
        rec["configs"] = other_configs(m, dev, args)
    print(json.dumps(rec), flush=True)


def _desc_of(m, inst, flags):
    return m.Desc(gx=inst.gx, gy=inst.gy, gt=inst.gt, hs=inst.hs, ht=inst.ht, sres=inst.sres,
                  tres=inst.tres, x0=inst.x0, y0=inst.y0, t0=inst.t0, flags=flags)


def _roofline(alg_bytes, alg_flops, gather_ms):
    """The binding roofline of a workload for the gather kernel: HBM below the
    ridge point, FP32 matrix cores above it."""
    if alg_flops / alg_bytes < MFMA_F32_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9):
        achieved = alg_bytes / (gather_ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "algorithmic": {"bytes": alg_bytes, "flops": alg_flops}}
    achieved = alg_flops / (gather_ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": achieved, "peak": MFMA_F32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / MFMA_F32_PEAK_TFLOPS, "traffic": None,
            "algorithmic": {"bytes": alg_bytes, "flops": alg_flops}}


def time_compute(m, desc, tuning, pts, pairs, steps, warmup, stages=False):
    """Time `steps` full computations (after `warmup`) with the points resident:
    wall time per step between two synchronisations, with nothing else on the
    stream; then, in a second run of `steps` computations, the median of
    per-step events and the gather kernel's duration from the events the
    library records around that launch on its stream (event records between
    launches cost a few microseconds per step, which the wall time leaves
    out).  Also the exact evaluation count and the per-point mass (a separate
    computation outside the timed region), and, with `stages`, the binning and
    accumulation stages timed apart."""
    import torch
    dev = pts.device
    stream = torch.cuda.current_stream(dev)
    n = int(pts.shape[0])
    adaptive = pairs is not None
    plan = m.Plan(desc, tuning)

    def compute(p, o, st=None, w=None):
        if adaptive:
            return p.compute_adaptive_into(pts, pairs, o, stats=st, workspace=w)
        return p.compute_into(pts, o, stats=st, workspace=w)
    out = torch.empty((desc.gx, desc.gy, desc.gt), dtype=torch.float32, device=dev)
    stats = torch.zeros(8, dtype=torch.float64, device=dev)
    ws = plan.workspace(n, dev)
    chk = m.Plan(m.Desc(**{**desc.__dict__, "flags": desc.flags | m.FLAG_POINT_STATS | m.FLAG_MASS}), tuning)
    cstats = torch.zeros(8, dtype=torch.float64, device=dev)
    compute(chk, out, cstats, ws)
    torch.cuda.synchronize()
    cs = cstats.cpu().numpy()
    chk.close()
    for _ in range(warmup):
        compute(plan, out, stats, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        compute(plan, out, stats, ws)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    plan.profile(steps)
    torch.cuda.synchronize()
    for k in range(steps):
        ev[k][0].record(stream)
        compute(plan, out, stats, ws)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    kern_ms = plan.profile_read()
    plan.profile(0)
    if len(kern_ms) != steps:
        raise SystemExit(f"expected {steps} gather timings, got {len(kern_ms)}")
    res = {"ms_per_step": (t1 - t0) * 1e3 / steps,
           "median_step_ms": _median([a.elapsed_time(b) for a, b in ev]),
           "gather_ms": sum(kern_ms) / len(kern_ms), "evals": int(cs[2]),
           "point_mass": float(cs[1]), "grid_mass": float(stats[0].item()), "out": out}
    _log(f"{desc.gx}x{desc.gy}x{desc.gt} hs={desc.hs:g} ht={desc.ht:g} flags={desc.flags}: "
         f"{res['ms_per_step']:.4f} ms/step wall, median event {res['median_step_ms']:.4f} ms, "
         f"gather {res['gather_ms']:.4f} ms, {res['evals']} evals")
    if stages:
        reps = max(5, steps)
        bev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        gev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for k in range(reps):
            bev[k][0].record(stream)
            if adaptive:
                plan.bin_adaptive(pts, pairs, ws)
            else:
                plan.bin(pts, ws)
            bev[k][1].record(stream)
            gev[k][0].record(stream)
            plan.accumulate(n, out, ws)
            gev[k][1].record(stream)
        torch.cuda.synchronize()
        res["bin_ms"] = sum(a.elapsed_time(b) for a, b in bev) / reps
        res["pass_ms"] = sum(a.elapsed_time(b) for a, b in gev) / reps
        _log(f"stage times: bin {res['bin_ms']:.3f} ms, accumulation pass {res['pass_ms']:.3f} ms")
    plan.close()
    return res


def time_graph(m, desc, tuning, pts, eager_out, steps, warmup):
    """Wall time per step of the same computation recorded once as a HIP graph
    (stkde_plan_capture) and replayed `steps` times after `warmup` replays,
    and whether a replay's grid is bitwise the eager one."""
    import torch
    n = int(pts.shape[0])
    plan = m.Plan(desc, tuning)
    out = torch.empty_like(eager_out)
    stats = torch.zeros(8, dtype=torch.float64, device=pts.device)
    ws = plan.workspace(n, pts.device)
    plan.capture(pts, out, stats=stats, workspace=ws)
    for _ in range(warmup):
        plan.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    same = bool(torch.equal(out, eager_out))
    plan.close()
    ms = (t1 - t0) * 1e3 / steps
    _log(f"{desc.gx}x{desc.gy}x{desc.gt} graph replay: {ms:.4f} ms/step, bitwise equal to eager: {same}")
    return {"ms_per_step": ms, "bitwise_equal_eager": same}


def error_stats(gpu, ref):
    """Max and RMS error of a GPU grid against the oracle's, relative to the
    oracle's peak (RMS over voxels where either side is nonzero), and the
    support mismatch: voxels where exactly one side is nonzero."""
    import numpy as np
    g = np.asarray(gpu, dtype=np.float64)
    peak = max(float(np.max(np.abs(ref))), 1e-300)
    d = np.abs(g - ref)
    supp = (g != 0.0) | (ref != 0.0)
    ns = int(np.count_nonzero(supp))
    return {"max_rel": float(np.max(d)) / peak,
            "rms_rel": (float(np.sqrt(np.mean(d[supp] ** 2))) / peak) if ns else 0.0,
            "mismatch": int(np.count_nonzero((g != 0.0) != (ref != 0.0)))}


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_single_thread(inst, k):
    """The oracle on one thread over the first k events (the paper's
    sequential times are single-threaded, Sec. 6.2)."""
    import oracle
    g = oracle.Grid(gx=inst.gx, gy=inst.gy, gt=inst.gt, hs=inst.hs, ht=inst.ht, sres=inst.sres,
                    tres=inst.tres, x0=inst.x0, y0=inst.y0, t0=inst.t0)
    t0 = time.perf_counter()
    _, evals = oracle.pbsym(inst.points[:k], g, nthreads=1)
    dt = time.perf_counter() - t0
    _log(f"cpu oracle, one thread: {k} events of {inst.name}, {evals} evals, {dt:.2f} s")
    return {"value": evals / dt, "unit": "evals/s", "cores": 1, "seconds": round(dt, 3),
            "sample": f"first {k} of {inst.points.shape[0]} events on the full grid"}


def precision_record(m, inst, desc, tuning, pts, operands, est, ref, k, gpu_sample, args):
    """What the headline's arithmetic is and what it costs in accuracy: the
    two-term operand form and its stated bias bound, and the FP32-operand
    gather timed and checked on the same oracle sample."""
    from paper_1705_09366_amd import autotune
    rec = {"operands": operands,
           "per_product_relative_bias_bound": 2.0 ** -19 if operands.startswith("fp16") else 0.0,
           "bias_note": "two-term FP16 operands keep 22 significant bits each and drop the lo*lo term, "
                        "so each product is low by less than 2^-19 of itself (all products are "
                        "non-negative); accumulation is FP32 on the matrix cores",
           "max_rel_err_vs_oracle": est["max_rel"], "rms_rel_err_vs_oracle": est["rms_rel"],
           "support_mismatch": est["mismatch"], "oracle_sample_events": k}
    t32, src32 = autotune.resolve(desc, inst.points.shape[0], fp32=True)
    t32 = dataclasses.replace(t32 or m.Tuning(), operand_form=1)
    r32 = time_compute(m, desc, t32, pts, None, max(5, args.steps // 2), 2)
    e32 = error_stats(gpu_sample(k, t32), ref)
    alg_bytes = inst.gx * inst.gy * inst.gt * 4 + inst.points.shape[0] * 24
    rec["fp32_operands"] = {"ms_per_step": r32["ms_per_step"], "gather_ms": r32["gather_ms"],
                            "roofline_frac": _roofline(alg_bytes, 2.0 * r32["evals"], r32["gather_ms"])["frac"],
                            "tuning_source": src32, "max_rel_err_vs_oracle": e32["max_rel"],
                            "rms_rel_err_vs_oracle": e32["rms_rel"], "support_mismatch": e32["mismatch"]}
    del r32
    return rec


def other_configs(m, dev, args):
    """The latency-bound small case and the large-bandwidth case, each timed
    and checked against the FP64 oracle on the whole grid (the large-bandwidth
    case twice: compensated and plain FP32 accumulation)."""
    import numpy as np
    import torch
    import oracle
    import workloads
    from paper_1705_09366_amd import autotune
    out = {}
    th = _cpu_threads()
    for name, inst, modes in (("uniform-10k", workloads.config0(), ("kahan",)),
                              ("clustered-200k-hs50", workloads.config2(), ("kahan", "plain"))):
        n = inst.points.shape[0]
        pts = torch.from_numpy(inst.points).to(dev)
        g = oracle.Grid(gx=inst.gx, gy=inst.gy, gt=inst.gt, hs=inst.hs, ht=inst.ht)
        t0 = time.perf_counter()
        ref, evals = oracle.pbsym(inst.points, g, nthreads=th)
        dt = time.perf_counter() - t0
        _log(f"cpu oracle: {name} whole grid, {evals} evals, {dt:.2f} s on {th} threads")
        rec = {"workload": inst.name, "n": n, "grid": [inst.gx, inst.gy, inst.gt], "hs": inst.hs,
               "ht": inst.ht, "evals": int(evals),
               "cpu_oracle": {"value": evals / dt, "unit": "evals/s", "cores": th, "seconds": round(dt, 3),
                              "sample": "whole workload"}}
        if name == "uniform-10k":
            rec["cpu_oracle"]["single_thread"] = cpu_single_thread(inst, n)
        for mode in modes:
            flags = m.FLAG_MASS | (m.FLAG_KAHAN if mode == "kahan" else 0)
            desc = _desc_of(m, inst, flags)
            tun, src = autotune.resolve(desc, n)
            r = time_compute(m, desc, tun, pts, None, 200 if name == "uniform-10k" else args.steps, 3)
            est = error_stats(r["out"].cpu().numpy(), ref)
            alg_bytes = inst.gx * inst.gy * inst.gt * 4 + n * 24
            roof = _roofline(alg_bytes, 2.0 * r["evals"], r["gather_ms"])
            rec[mode] = {"ms_per_step": r["ms_per_step"], "median_step_ms": r["median_step_ms"],
                         "evals_per_s": r["evals"] / (r["ms_per_step"] * 1e-3), "gather_ms": r["gather_ms"],
                         "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac")},
                         "operands": _operand_form(inst, tun, mode == "kahan", False, 0),
                         "tuning_source": src, "max_rel_err_vs_oracle": est["max_rel"],
                         "rms_rel_err_vs_oracle": est["rms_rel"], "support_mismatch": est["mismatch"]}
            if name == "uniform-10k":
                rec[mode]["graph_replay"] = time_graph(m, desc, tun, pts, r["out"], 200, 10)
            _log(f"{name} {mode}: {r['ms_per_step']:.4f} ms/step, max rel err {est['max_rel']:.3e}, "
                 f"rms {est['rms_rel']:.3e}, mismatch {est['mismatch']}")
            del r
        del ref, pts
        torch.cuda.empty_cache()
        out[name] = rec
    return out


if __name__ == "__main__":
    main()
