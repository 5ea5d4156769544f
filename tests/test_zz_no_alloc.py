"""GPU: the entry point without allocation (stkde_compute_noalloc) gives the
grid and statistics of stkde_compute with a caller workspace, bit for bit,
and matches the FP64 oracle -- on calls in a row, each smaller than the one
before (the static scratch keeps the previous call's contents), and again
after a larger stkde_compute has run.""" 
import sys

import numpy as np
import pytest

import oracle
import workloads
from oracle import Grid
from parity import assert_parity

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


def _case(torch, m, g, pts, flags):
    desc = m.Desc(flags=flags, **g)
    plan = m.Plan(desc)
    n = pts.shape[0]
    assert plan.workspace_bytes(n) <= m.STATIC_SCRATCH_BYTES
    d = torch.from_numpy(pts).cuda()
    shape = (g["gx"], g["gy"], g["gt"])
    ref = torch.full(shape, float("nan"), dtype=torch.float32, device="cuda")
    got = torch.full(shape, float("nan"), dtype=torch.float32, device="cuda")
    st_ref = torch.zeros(8, dtype=torch.float64, device="cuda")
    st_got = torch.full((8,), float("nan"), dtype=torch.float64, device="cuda")
    plan.compute_into(d, ref, stats=st_ref)
    plan.compute_noalloc(d, got, stats=st_got)
    torch.cuda.synchronize()
    assert torch.equal(got, ref), "noalloc grid differs from stkde_compute"
    assert torch.equal(st_got, st_ref), "noalloc statistics differ from stkde_compute"
    o, _ = oracle.pbsym(pts, Grid(**g))
    s = assert_parity(got.cpu().numpy(), o, what="noalloc")
    plan.close()
    return s


def test_noalloc_matches_compute_two_calls(torch_cuda):
    import paper_1705_09366_amd as m
    torch = torch_cuda
    rng = np.random.default_rng(7100)
    g1 = dict(gx=96, gy=80, gt=48, hs=6.5, ht=4.5, sres=1.0, tres=1.0, x0=0.0, y0=0.0, t0=0.0)
    # uniform events plus a dense pile, so that some tiles take several
    # compensated phases (their running sums live in the scratch)
    p1 = np.concatenate([rng.uniform(0, 1, (26_000, 3)) * [96, 80, 48],
                         np.array([40.0, 30.0, 20.0]) + rng.normal(0, 2.0, (4_000, 3))])
    _say(f"first call: grid 96x80x48, n={p1.shape[0]}, Kahan and mass")
    s1 = _case(torch, m, g1, p1, m.FLAG_KAHAN | m.FLAG_MASS)
    _say(f"first call: max rel err {s1['max_rel']:.2e}")
    inst = workloads.config0()
    g2 = dict(gx=inst.gx, gy=inst.gy, gt=inst.gt, hs=inst.hs, ht=inst.ht, sres=1.0, tres=1.0, x0=0.0, y0=0.0,
              t0=0.0)
    _say(f"second, smaller call: {inst.name}, n={inst.points.shape[0]}, Kahan and mass")
    s2 = _case(torch, m, g2, inst.points, m.FLAG_KAHAN | m.FLAG_MASS)
    _say(f"second call: max rel err {s2['max_rel']:.2e}")
    pts, g3 = workloads.small_random_case(5, max_g=48, max_n=500)
    _say(f"third, smaller call: grid {g3['gx']}x{g3['gy']}x{g3['gt']}, n={pts.shape[0]}")
    s3 = _case(torch, m, g3, pts, m.FLAG_MASS)
    _say(f"third call: max rel err {s3['max_rel']:.2e}")


def test_noalloc_after_larger_compute_and_limit(torch_cuda):
    import paper_1705_09366_amd as m
    torch = torch_cuda
    pts, g = workloads.small_random_case(9, max_g=40, max_n=300)
    _say(f"noalloc after a larger compute: grid {g['gx']}x{g['gy']}x{g['gt']}, n={pts.shape[0]}")
    s = _case(torch, m, g, pts, m.FLAG_KAHAN)
    _say(f"max rel err {s['max_rel']:.2e}")
    # beyond the static scratch: refused on the host, output untouched
    big = m.Plan(m.Desc(gx=1024, gy=1024, gt=256, hs=10.0, ht=7.0))
    n = 4_000_000
    assert big.workspace_bytes(n) > m.STATIC_SCRATCH_BYTES
    x = torch.zeros((n, 3), dtype=torch.float64, device="cuda")
    out = torch.full((4, 4, 4), 7.0, dtype=torch.float32, device="cuda")
    st = m.lib().stkde_compute_noalloc(big.handle, x.data_ptr(), n, out.data_ptr(), None, None)
    assert st == m.STKDE_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
    big.close()
