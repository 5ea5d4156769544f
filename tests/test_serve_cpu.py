"""Scheduling logic of the request server, on the CPU with a fake executor:
first-come-first-served admission against the byte budget (outputs until
released plus the workspaces of ticks on the device, counted before a tick
launches), continuous batching under load, completion and latency
accounting."""
import pytest

from paper_1705_09366_amd.serve import Request, Server


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Each tick takes `per_request` seconds of virtual time per request."""

    def __init__(self, clock, total=10_000, per_request=1.0, ws=10):
        self.clock, self.total, self.per_request, self.ws = clock, total, per_request, ws
        self.launched = []
        self.released = []
        self.planned = 0
        self.discarded_plans = 0
        self.discarded = []
        self.busy_until = 0.0

    def total_memory(self):
        return self.total

    def add_set(self, name, points, base, tuning=None):
        return 1000

    def prepare(self, tk):
        if tk.req.gx <= 0:
            raise ValueError("bad request")
        return ("item", tk.rid)

    def plan_tick(self, items):
        self.planned += 1
        return {"items": list(items)}

    def planned_workspace_bytes(self, planned):
        return self.ws

    def discard_plan(self, planned):
        self.discarded_plans += 1

    def discard(self, item, tk):
        self.discarded.append(tk.rid)

    def launch(self, items, planned=None):
        assert planned is not None and planned["items"] == list(items)
        start = max(self.clock(), self.busy_until)
        self.busy_until = start + self.per_request * len(items)
        tok = {"items": [i[1] for i in items], "end": self.busy_until}
        self.launched.append(tok)
        return tok

    def workspace_bytes(self, token):
        return self.ws

    def done(self, token):
        return self.clock() >= token["end"]

    def release(self, token, items):
        self.released.append(token)


def _req(k, gx=10):
    return Request(set="a", gx=gx, gy=1, gt=1, ox=0, oy=0, ot=0, hs=1.0, ht=1.0)


def _server(clock, **kw):
    ex = FakeExecutor(clock, **{k: kw.pop(k) for k in list(kw) if k in ("total", "per_request", "ws")})
    s = Server(executor=ex, budget_bytes=kw.pop("budget", 10_000), clock=clock, **kw)
    return s, ex


def test_all_requests_complete_in_order_with_latency():
    clock = FakeClock()
    s, ex = _server(clock, max_inflight=1)
    tks = [s.submit(_req(k), t_arrival=0.0) for k in range(5)]
    s.poll()  # one tick with all five
    assert len(ex.launched) == 1 and ex.launched[0]["items"] == [0, 1, 2, 3, 4]
    clock.t = 4.9
    s.poll()
    assert not any(t.done for t in tks)
    clock.t = 5.0
    s.poll()
    assert all(t.done for t in tks) and s.idle()
    assert [t.latency for t in tks] == [5.0] * 5
    st = s.latency_stats()
    assert st["count"] == 5 and st["p50_ms"] == pytest.approx(5000.0)


def _poll_release(s):
    """Poll, hand every finished output back, poll again."""
    s.poll()
    for tk in s.finished:
        if tk.charged:
            s.release(tk)
    s.poll()


def test_admission_respects_the_budget_first_come_first_served():
    clock = FakeClock()
    # each request needs 40 + 64 bytes; the budget fits two (plus a tick workspace)
    s, ex = _server(clock, budget=300, max_inflight=4)
    tks = [s.submit(_req(k), t_arrival=0.0) for k in range(5)]
    s.poll()
    assert ex.launched[-1]["items"] == [0, 1]
    assert s.active_bytes == 2 * 104 + 10 <= s.budget
    s.poll()  # nothing fits until the first tick retires
    assert len(ex.launched) == 1
    clock.t = 2.0
    _poll_release(s)
    assert ex.launched[-1]["items"] == [2, 3]
    clock.t = 4.0
    _poll_release(s)
    assert ex.launched[-1]["items"] == [4]
    clock.t = 5.0
    _poll_release(s)
    assert s.idle() and s.high_water <= s.budget and s.active_bytes == 0
    assert [t.tick for t in tks] == [0, 0, 1, 1, 2]


def test_tick_workspace_is_counted_before_the_launch():
    clock = FakeClock()
    # two outputs (2 x 104) fit the budget of 300, but not with a 100-byte
    # tick workspace: the tick is cut back to one request, the second waits
    s, ex = _server(clock, budget=300, max_inflight=4, ws=100)
    tks = [s.submit(_req(k), t_arrival=0.0) for k in range(3)]
    s.poll()
    assert ex.launched[-1]["items"] == [0]
    assert s.active_bytes == 104 + 100 <= s.budget
    assert ex.discarded == [1] and [t.rid for t in s.waiting] == [1, 2]
    s.poll()  # 204 + 104 + 100 > 300: nothing more until tick 0 retires
    assert len(ex.launched) == 1
    clock.t = 1.0
    _poll_release(s)
    assert ex.launched[-1]["items"] == [1]
    clock.t = 10.0
    while not s.idle():
        _poll_release(s)
        clock.t += 1.0
    assert all(t.done and t.error is None for t in tks)
    assert s.high_water <= s.budget


def test_outputs_stay_charged_until_released():
    clock = FakeClock()
    s, ex = _server(clock, budget=300, max_inflight=4)
    a = s.submit(_req(0), t_arrival=0.0)
    s.poll()
    clock.t = 1.0
    s.poll()
    assert a.done and s.active_bytes == 104  # workspace returned, output held
    with pytest.raises(ValueError):
        s.release(s.submit(_req(1), t_arrival=1.0))  # not finished
    s.release(a)
    assert s.active_bytes == 0 and a.out is None


def test_a_request_that_cannot_fit_with_its_workspace_fails_instead_of_waiting():
    clock = FakeClock()
    s, ex = _server(clock, budget=300, max_inflight=4, ws=250)
    tk = s.submit(_req(0), t_arrival=0.0)  # 104 bytes of output alone fit, 354 with the workspace do not
    s.poll()
    assert tk.done and tk.error and s.failed == [tk] and not ex.launched and s.idle()


def test_batches_grow_under_load():
    clock = FakeClock()
    s, ex = _server(clock, max_inflight=1, per_request=0.1)
    s.submit(_req(0), t_arrival=0.0)
    s.poll()  # tick of one
    for k in range(1, 8):  # arrive while the first tick runs
        clock.t = 0.01 * k
        s.submit(_req(k))
        s.poll()
    assert len(ex.launched) == 1
    clock.t = 0.1
    s.poll()  # retires tick 0, launches the seven waiting together
    assert ex.launched[-1]["items"] == list(range(1, 8))
    clock.t = 10.0
    s.drain()
    assert len(s.finished) == 8


def test_max_batch_caps_a_tick():
    clock = FakeClock()
    s, ex = _server(clock, max_batch=3, max_inflight=8)
    for k in range(7):
        s.submit(_req(k), t_arrival=0.0)
    s.poll()
    s.poll()
    s.poll()
    assert [len(t["items"]) for t in ex.launched] == [3, 3, 1]


def test_oversize_and_bad_requests_are_refused():
    clock = FakeClock()
    s, ex = _server(clock, budget=300)
    with pytest.raises(ValueError):
        s.submit(Request(set="a", gx=100, gy=1, gt=1, ox=0, oy=0, ot=0, hs=1.0, ht=1.0))
    s.submit(_req(1), t_arrival=0.0)
    bad = s.submit(_req(0, gx=0))
    s.submit(_req(2), t_arrival=0.0)
    with pytest.raises(ValueError):
        s.poll()
    # the bad request failed; the good ones went back to the queue in order
    assert bad.done and bad.error and s.failed == [bad]
    assert [t.rid for t in s.waiting] == [0, 2] and ex.discarded == [0]


def test_resident_sets_reduce_the_budget():
    clock = FakeClock()
    s, ex = _server(clock, budget=5000)
    s.add_set("a", None, None)
    assert s.budget == 4000
