"""GPU: requests served in a mix over resident sets equal the same requests
run alone (bitwise: same tuning, same set), and match the FP64 oracle on
the window grid with the whole set's points."""
import sys

import numpy as np
import pytest

import oracle
from oracle import Grid

pytestmark = pytest.mark.gpu


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


def test_mix_equals_alone_and_oracle(torch_cuda):
    import paper_1705_09366_amd as m
    from paper_1705_09366_amd.serve import GpuExecutor, Request, Server
    torch = torch_cuda
    rng = np.random.default_rng(21)
    base = m.Desc(gx=128, gy=112, gt=64, hs=8.0, ht=8.0)
    sets = {}
    ex = GpuExecutor()
    srv = Server(executor=ex, max_inflight=2)
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
    tks = [srv.submit(r) for r in reqs]
    srv.drain()
    torch.cuda.synchronize()
    st = srv.latency_stats()
    _say(f"served {st['count']} in {st['ticks']} ticks, p50 {st['p50_ms']:.3f} ms")
    assert st["count"] == 12 and all(t.done for t in tks)
    for tk in tks:
        r = tk.req
        # alone: the same request in a batch of its own
        item = ex.prepare(type(tk)(rid=-1, req=r, t_arrival=0.0))
        b = m.Batch([item])
        b.run()
        torch.cuda.synchronize()
        assert torch.equal(item.out, tk.out), f"request {tk.rid} differs alone"
        b.close()
        g = Grid(gx=r.gx, gy=r.gy, gt=r.gt, hs=r.hs, ht=r.ht, x0=float(r.ox), y0=float(r.oy),
                 t0=float(r.ot))
        ref, _ = oracle.pbsym(sets[r.set], g)
        got = tk.out.cpu().numpy().astype(np.float64)
        scale = max(float(np.max(ref)), 1e-300)
        assert float(np.max(np.abs(got - ref))) <= 1e-5 * scale
        mass = tk.stats.cpu().numpy()[0]
        assert mass == pytest.approx(float(got.sum()), rel=1e-9, abs=1e-300)
