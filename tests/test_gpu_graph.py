"""GPU: one computation recorded as a HIP graph (stkde_plan_capture /
stkde_plan_replay) gives bitwise the grid of stkde_compute with the same
arguments, on every replay, with the program's own eager work and
synchronisations between replays; a replay reads the point values the input
holds when it runs; and it matches the FP64 oracle."""
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


CASES = [
    ("uniform-10k kahan", lambda: workloads.config0(), 1 | 4, None),
    ("uniform-10k plain 16-row", lambda: workloads.config0(), 4, (16, 0, 0, 0)),
    ("uniform-10k fp32 operands", lambda: workloads.config0(), 1 | 4, (0, 0, 0, 0, 0, 1)),
]


@pytest.mark.parametrize("name,make,flags,tun", CASES, ids=[c[0] for c in CASES])
def test_replay_bitwise_equals_compute(torch_cuda, name, make, flags, tun):
    import paper_1705_09366_amd as m
    torch = torch_cuda
    inst = make()
    _say(f"graph {name}: n={inst.points.shape[0]} grid {inst.gx}x{inst.gy}x{inst.gt}")
    desc = m.Desc(gx=inst.gx, gy=inst.gy, gt=inst.gt, hs=inst.hs, ht=inst.ht, flags=flags)
    plan = m.Plan(desc, m.Tuning(*tun) if tun else None)
    pts = torch.from_numpy(inst.points).cuda()
    eager = torch.full((inst.gx, inst.gy, inst.gt), float("nan"), dtype=torch.float32, device="cuda")
    st_e = torch.zeros(8, dtype=torch.float64, device="cuda")
    plan.compute_into(pts, eager, stats=st_e, workspace=plan.workspace(len(pts)))
    torch.cuda.synchronize()
    out = torch.full_like(eager, float("nan"))
    st = torch.zeros(8, dtype=torch.float64, device="cuda")
    ws = torch.empty(plan.workspace_bytes(len(pts)) + 256, dtype=torch.uint8, device="cuda")
    plan.capture(pts, out, stats=st, workspace=ws)
    torch.cuda.synchronize()
    assert torch.isnan(out).all(), "capture must not run anything"
    for rep in range(4):
        out.fill_(float("nan"))
        st.zero_()
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
        plan.replay()
        torch.cuda.synchronize()
        assert float(junk) == float(junk)
        assert torch.equal(out, eager), f"replay {rep} differs from the eager computation"
        assert torch.equal(st, st_e), f"replay {rep}: statistics differ"
    ref, _ = oracle.pbsym(inst.points, Grid(gx=inst.gx, gy=inst.gy, gt=inst.gt, hs=inst.hs, ht=inst.ht))
    assert_parity(out.cpu().numpy(), ref, what=name)
    plan.close()


def test_replay_reads_the_current_points(torch_cuda):
    import paper_1705_09366_amd as m
    torch = torch_cuda
    rng = np.random.default_rng(5)
    g = dict(gx=77, gy=53, gt=41, hs=4.5, ht=3.5)
    a = rng.uniform(0, 1, (900, 3)) * [77, 53, 41]
    b = rng.uniform(0, 1, (900, 3)) * [77, 53, 41]
    plan = m.Plan(m.Desc(**g, flags=1))
    pts = torch.from_numpy(a).cuda()
    out = torch.empty((77, 53, 41), dtype=torch.float32, device="cuda")
    plan.capture(pts, out)
    for src in (a, b, a):
        pts.copy_(torch.from_numpy(src))
        plan.replay()
        torch.cuda.synchronize()
        ref, _ = oracle.pbsym(src, Grid(**g))
        assert_parity(out.cpu().numpy(), ref, what="replay after new points")
        eager = m.Plan(m.Desc(**g, flags=1))(pts)
        torch.cuda.synchronize()
        assert torch.equal(out, eager)
    plan.close()


def test_capture_checks_arguments(torch_cuda):
    import paper_1705_09366_amd as m
    torch = torch_cuda
    plan = m.Plan(m.Desc(gx=8, gy=8, gt=8, hs=2.0, ht=2.0))
    pts = torch.zeros((10, 3), dtype=torch.float64, device="cuda")
    out = torch.empty((8, 8, 8), dtype=torch.float32, device="cuda")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(m.StkdeError) as e:
        plan.capture(pts, out, workspace=small)
    assert e.value.status == m.STKDE_ERR_WORKSPACE
    with pytest.raises(m.StkdeError) as e:
        plan.replay()  # nothing recorded
    assert e.value.status == m.STKDE_ERR_UNSUPPORTED
    plan.close()
