"""GPU: continuous batching over resident sets.  Requests arrive while
earlier ticks are on the device (two ticks in flight on two streams, a few
requests per tick); each result equals the same request run alone (bitwise
with the same tuning and set when neither run cut one of its tiles into
parts, else within tolerance) and matches the FP64 oracle on the window grid
with the whole set's points.  The second test does the same at the serving
workload's size: 4 resident sets of 100k..2M clustered points over
2048 x 2048 x 512, 32 requests for windows of 64..1024 x 64..1024 x 64..128
voxels at hs, ht in [3, 40], every window compared whole with the oracle."""
import sys

import numpy as np
import pytest

import oracle
import workloads
from oracle import Grid
from parity import assert_parity

pytestmark = pytest.mark.gpu

# cycles of the spin kernel that holds the first tick's stream, so that the
# second tick is admitted while the first is still on the device
HOLD_CYCLES = 20_000_000


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


def _serve(torch, srv, ex, reqs):
    """Submit the requests one by one with a poll after each (the first tick's
    stream held briefly by a spin kernel), then drain."""
    with torch.cuda.stream(ex.streams[0]):
        torch.cuda._sleep(HOLD_CYCLES)
    tks = []
    for r in reqs:
        tks.append(srv.submit(r))
        srv.poll()
    srv.drain()
    torch.cuda.synchronize()
    return tks


def _check_alone(torch, m, ex, tk):
    """The request run alone (a batch of one) gives the served grid bit for
    bit when neither run computed one of its tiles in parts (stats[6] = 0 in
    both; which tiles are cut depends on the batch), else the two agree
    within the parity tolerance of the peak."""
    item = ex.prepare(type(tk)(rid=-1, req=tk.req, t_arrival=0.0))
    b = m.Batch([item])
    b.run()
    torch.cuda.synchronize()
    cut = (int(item.stats[6].item()), int(tk.stats[6].item()))
    if cut == (0, 0):
        same = torch.equal(item.out, tk.out)
    else:
        a, c = item.out.double(), tk.out.double()
        peak = float(a.abs().max())
        same = float((a - c).abs().max()) <= 1e-5 * peak
        _say(f"request {tk.rid}: tiles in parts alone / served {cut}, compared within tolerance")
    b.close()
    item.plan.close()
    return same


def test_mix_equals_alone_and_oracle(torch_cuda):
    import paper_1705_09366_amd as m
    from paper_1705_09366_amd.serve import GpuExecutor, Request, Server
    torch = torch_cuda
    rng = np.random.default_rng(21)
    base = m.Desc(gx=128, gy=112, gt=64, hs=8.0, ht=8.0)
    sets = {}
    ex = GpuExecutor()
    srv = Server(executor=ex, max_batch=3, max_inflight=2)
    for name, n in (("a", 2500), ("b", 4000)):
        pts = rng.uniform(0, 1, (n, 3)) * [128, 112, 64]
        sets[name] = pts
        srv.add_set(name, torch.from_numpy(pts).cuda(), base)
    reqs = []
    for k in range(12):
        gx, gy, gt = int(rng.integers(1, 60)), int(rng.integers(1, 60)), int(rng.integers(1, 40))
        reqs.append(Request(set="ab"[k % 2], gx=gx, gy=gy, gt=gt, ox=int(rng.integers(0, 128 - gx + 1)),
                            oy=int(rng.integers(0, 112 - gy + 1)), ot=int(rng.integers(0, 64 - gt + 1)),
                            hs=float(rng.uniform(1.5, 8.0)), ht=float(rng.uniform(1.5, 8.0)),
                            flags=m.FLAG_MASS))
    tks = _serve(torch, srv, ex, reqs)
    st = srv.latency_stats()
    _say(f"served {st['count']} in {st['ticks']} ticks, {st['max_inflight_seen']} in flight at most, "
         f"p50 {st['p50_ms']:.3f} ms")
    assert st["count"] == 12 and all(t.done and t.error is None for t in tks)
    assert st["ticks"] >= 4 and st["max_inflight_seen"] == 2
    assert srv.high_water <= srv.budget
    for tk in tks:
        r = tk.req
        assert _check_alone(torch, m, ex, tk), f"request {tk.rid} differs alone"
        g = Grid(gx=r.gx, gy=r.gy, gt=r.gt, hs=r.hs, ht=r.ht, x0=float(r.ox), y0=float(r.oy),
                 t0=float(r.ot))
        ref, _ = oracle.pbsym(sets[r.set], g)
        got = tk.out.cpu().numpy()
        assert_parity(got, ref, what=f"request {tk.rid}")
        mass = tk.stats.cpu().numpy()[0]
        assert mass == pytest.approx(float(got.astype(np.float64).sum()), rel=1e-9, abs=1e-300)
        srv.release(tk)
    assert srv.active_bytes == 0


def test_serving_workload_requests_vs_oracle(torch_cuda):
    import paper_1705_09366_amd as m
    from paper_1705_09366_amd.serve import GpuExecutor, Request, Server
    torch = torch_cuda
    sets = workloads.config4_sets()
    ex = GpuExecutor()
    srv = Server(executor=ex, max_batch=4, max_inflight=2)
    names = []
    for k, inst in enumerate(sets):
        base = m.Desc(gx=inst.gx, gy=inst.gy, gt=inst.gt, hs=40.0, ht=40.0)
        srv.add_set(f"s{k}", torch.from_numpy(inst.points).cuda(), base, m.Tuning(tile_t=16))
        names.append(f"s{k}")
    _say(f"serving workload: {len(sets)} resident sets, n = {[s.points.shape[0] for s in sets]}")
    raw = workloads.config4_requests(32, seed_salt=7)
    reqs = [Request(set=names[r["set"]], gx=r["gx"], gy=r["gy"], gt=r["gt"], ox=int(r["x0"]),
                    oy=int(r["y0"]), ot=int(r["t0"]), hs=r["hs"], ht=r["ht"],
                    flags=m.FLAG_MASS | m.FLAG_KAHAN) for r in raw]
    tks = _serve(torch, srv, ex, reqs)
    st = srv.latency_stats()
    _say(f"served {st['count']} in {st['ticks']} ticks, {st['max_inflight_seen']} in flight at most")
    assert st["count"] == 32 and all(t.done and t.error is None for t in tks)
    assert st["max_inflight_seen"] == 2 and srv.high_water <= srv.budget
    worst = 0.0
    for tk in tks:
        r = tk.req
        pts = sets[names.index(r.set)].points
        _say(f"request {tk.rid}: set {r.set} (n={pts.shape[0]}), window {r.gx}x{r.gy}x{r.gt} at "
             f"({r.ox}, {r.oy}, {r.ot}), hs={r.hs:.3f} ht={r.ht:.3f}")
        assert _check_alone(torch, m, ex, tk), f"request {tk.rid} differs alone"
        g = Grid(gx=r.gx, gy=r.gy, gt=r.gt, hs=r.hs, ht=r.ht, x0=float(r.ox), y0=float(r.oy),
                 t0=float(r.ot))
        ref, _ = oracle.pbsym(pts, g)
        got = tk.out.cpu().numpy()
        if float(np.max(ref)) == 0.0:
            assert not np.any(got), f"request {tk.rid}: nonzero grid where the oracle is zero"
        else:
            s = assert_parity(got, ref, what=f"request {tk.rid}")
            worst = max(worst, s["max_rel"])
        mass = tk.stats.cpu().numpy()[0]
        assert mass == pytest.approx(float(got.astype(np.float64).sum()), rel=1e-9, abs=1e-300)
        del ref
        srv.release(tk)
    _say(f"worst max rel err over the 32 requests {worst:.3e}")
