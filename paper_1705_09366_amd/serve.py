"""Serving density requests over resident binned point sets.

The paper's motivation is interactive exploration (Sec. 1): an analyst asks
for the density of a region at some bandwidths, looks, and asks again.
Here the point sets stay binned on the device (``BinnedSet``); a request
names a set, a voxel-aligned window of its base grid and a bandwidth pair,
and gets the window of the set's density (the estimate divides by the whole
set's n, so a window is a cut-out of the full grid).

Scheduling is continuous batching: each tick packs every admitted waiting
request into one ``Batch`` (one work list, one persistent gather launch per
tile group, the requests' tiles scheduled together costliest first) and
enqueues it on the next of the executor's streams, so that a new tick's
work starts while the previous one drains; while ``max_inflight`` ticks are
on the device, the next tick collects whatever arrived meanwhile, so
batches grow with the load.  Admission is first come, first served, against a byte
budget: the outputs of admitted requests that the caller has not released
(:meth:`Server.release`) plus the workspaces of the ticks on the device must
fit in the device memory left after the resident sets and a reserve.  A
tick's workspace is known from its plan before anything is launched, so a
tick is cut back (its last requests return to the head of the queue) until
outputs and workspace fit; the budget is never exceeded.  A request completes
when its tick's completion event has been reached; its latency is measured
on the host clock from submission (or a given arrival time) to the poll that
observes completion.

The device side sits behind a small executor interface, so the scheduling
logic is testable without a GPU.
"""
import collections
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

from . import FLAG_MASS, Batch, BinnedSet, Desc, Item, Plan, StkdeError, Tuning
from . import STKDE_ERR_UNSUPPORTED


@dataclass
class Request:
    """A density window: set name, grid size, window origin in base voxels,
    bandwidths in domain units, and flags (only STKDE_FLAG_MASS /
    STKDE_FLAG_KAHAN apply)."""
    set: str
    gx: int
    gy: int
    gt: int
    ox: int
    oy: int
    ot: int
    hs: float
    ht: float
    flags: int = 0

    def nbytes(self) -> int:
        return self.gx * self.gy * self.gt * 4


@dataclass
class Ticket:
    rid: int
    req: Request
    t_arrival: float
    t_admit: float = 0.0
    t_done: float = 0.0
    out: object = None
    stats: object = None
    tick: int = -1
    done: bool = False
    error: Optional[str] = None
    charged: int = 0  # output bytes held against the budget until released

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class GpuExecutor:
    """Runs ticks as Batch launches on round-robin streams; completion by events."""

    def __init__(self, device=None, tuning_cache: Optional[str] = None, streams: int = 2):
        import torch
        self.torch = torch
        self.device = torch.device(device if device is not None else "cuda")
        # default priority on every stream
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(max(1, streams))]
        self.stream = self.streams[0]
        self._next_stream = 0
        self.tuning_cache = tuning_cache
        self.sets: Dict[str, BinnedSet] = {}
        self.base: Dict[str, Desc] = {}

    def total_memory(self) -> int:
        return int(self.torch.cuda.get_device_properties(self.device).total_memory)

    def add_set(self, name: str, points, base: Desc, tuning: Optional[Tuning] = None) -> int:
        s = BinnedSet(base, int(points.shape[0]), tuning)
        with self.torch.cuda.stream(self.stream):
            s.build(points, stream=self.stream)
        self.stream.synchronize()
        s._scratch = None
        self.sets[name] = s
        self.base[name] = base
        return s.set_bytes

    def _plan(self, req: Request, tile_t: Optional[int] = None) -> Plan:
        from . import autotune
        b = self.base[req.set]
        d = Desc(gx=req.gx, gy=req.gy, gt=req.gt, hs=req.hs, ht=req.ht, sres=b.sres, tres=b.tres,
                 x0=b.x0 + req.ox * b.sres, y0=b.y0 + req.oy * b.sres, t0=b.t0 + req.ot * b.tres,
                 flags=req.flags)
        t = autotune.lookup(d, self.sets[req.set].n, self.tuning_cache)
        # the set's bins are fixed: keep only the tile rows and split share
        tt = tile_t if tile_t is not None else (t.tile_t if t else 0)
        return Plan(d, Tuning(tt, 0, 0, t.split_share if t else 0))

    def prepare(self, tk: Ticket):
        """Plan the request and allocate its output (raises on a bad request)."""
        torch = self.torch
        s = self.sets[tk.req.set]
        plan = self._plan(tk.req)
        with torch.cuda.stream(self.streams[self._next_stream]):
            out = torch.empty((tk.req.gx, tk.req.gy, tk.req.gt), dtype=torch.float32, device=self.device)
            stats = torch.empty(8, dtype=torch.float64, device=self.device) \
                if tk.req.flags & FLAG_MASS else None
        item = Item(plan=plan, set=s, out=out, ox=tk.req.ox, oy=tk.req.oy, ot=tk.req.ot, stats=stats)
        try:
            Batch([item], allocate=False).close()
        except StkdeError as e:
            if e.status != STKDE_ERR_UNSUPPORTED:
                raise
            # too many bin rows of this set for the cached tile rows
            plan.close()
            item.plan = self._plan(tk.req, tile_t=16)
            Batch([item], allocate=False).close()
        tk.out, tk.stats = out, stats
        return item

    def plan_tick(self, items: List[Item]):
        """Plan one tick (validation and workspace size, no device memory)."""
        return Batch(items, allocate=False)

    def planned_workspace_bytes(self, planned) -> int:
        return planned.workspace_bytes

    def discard_plan(self, planned):
        planned.close()

    def discard(self, item: Item, tk: Ticket):
        """Undo prepare() for a request that goes back to the queue."""
        item.plan.close()
        tk.out, tk.stats = None, None

    def launch(self, items: List[Item], planned=None):
        """Enqueue one tick on the next stream (its outputs were allocated on
        that stream by prepare)."""
        torch = self.torch
        st = self.streams[self._next_stream]
        self._next_stream = (self._next_stream + 1) % len(self.streams)
        b = planned if planned is not None else Batch(items, allocate=False)
        with torch.cuda.stream(st):
            b.allocate(self.device)
            b.run(stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
        return (b, ev, b.workspace_bytes)

    def workspace_bytes(self, token) -> int:
        return token[2]

    def done(self, token) -> bool:
        return token[1].query()

    def release(self, token, items: List[Item]):
        b, ev, _ = token
        b.close()
        for it in items:
            it.plan.close()


class Server:
    """Continuous-batching server over resident binned sets (see module doc)."""

    def __init__(self, executor=None, budget_bytes: Optional[int] = None, reserve: float = 0.05,
                 max_batch: int = 256, max_inflight: int = 2,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor if executor is not None else GpuExecutor()
        total = self.ex.total_memory()
        self.capacity = int(budget_bytes) if budget_bytes is not None else int(total * (1.0 - reserve))
        self.resident = 0
        self.max_batch = int(max_batch)
        self.max_inflight = int(max_inflight)
        self.clock = clock
        self.waiting: collections.deque = collections.deque()
        self.inflight: List = []  # (token, tickets, items, bytes)
        self.active_bytes = 0
        self.high_water = 0
        self.finished: List[Ticket] = []
        self.failed: List[Ticket] = []
        self.max_inflight_seen = 0
        self._next_id = 0
        self._ticks = 0

    # ---- sets ------------------------------------------------------------
    def add_set(self, name: str, points, base: Desc, tuning: Optional[Tuning] = None):
        self.resident += self.ex.add_set(name, points, base, tuning)

    @property
    def budget(self) -> int:
        """Bytes available to outputs and tick workspaces."""
        return self.capacity - self.resident

    # ---- requests ------------------------------------------------------------
    def submit(self, req: Request, t_arrival: Optional[float] = None) -> Ticket:
        if req.nbytes() > self.budget:
            raise ValueError(f"request of {req.nbytes()} bytes exceeds the budget {self.budget}")
        tk = Ticket(self._next_id, req, self.clock() if t_arrival is None else t_arrival)
        self._next_id += 1
        self.waiting.append(tk)
        return tk

    def _retire(self):
        now = None
        keep = []
        for token, tickets, items, ws in self.inflight:
            if self.ex.done(token):
                now = self.clock() if now is None else now
                for tk in tickets:
                    tk.t_done = now
                    tk.done = True
                    self.finished.append(tk)
                self.ex.release(token, items)
                self.active_bytes -= ws  # outputs stay charged until released
            else:
                keep.append((token, tickets, items, ws))
        self.inflight = keep

    def release(self, tk: Ticket):
        """The caller is done with a finished request's output: its bytes
        return to the budget (the tensors are dropped here)."""
        if not tk.done:
            raise ValueError("release() of a request that has not finished")
        tk.out, tk.stats = None, None
        self.active_bytes -= tk.charged
        tk.charged = 0

    def _admit(self):
        if len(self.inflight) >= self.max_inflight or not self.waiting:
            return
        # the longest first-come-first-served prefix whose outputs fit
        tickets, nbytes = [], 0
        for tk in self.waiting:
            if len(tickets) >= self.max_batch:
                break
            need = tk.req.nbytes() + 64
            if self.active_bytes + nbytes + need > self.budget:
                break  # the head waits until it fits
            tickets.append(tk)
            nbytes += need
        if not tickets:
            return
        for _ in tickets:
            self.waiting.popleft()
        items = []
        try:
            for tk in tickets:
                items.append(self.ex.prepare(tk))
        except Exception as e:
            # the bad request fails; the others go back to the queue in order
            k = len(items)
            for it, tk in zip(items, tickets):
                self.ex.discard(it, tk)
            for tk in reversed(tickets[:k] + tickets[k + 1:]):
                self.waiting.appendleft(tk)
            bad = tickets[k]
            bad.error, bad.done, bad.t_done = str(e), True, self.clock()
            self.failed.append(bad)
            raise
        # cut the tick back until outputs plus its workspace fit
        while True:
            planned = self.ex.plan_tick(items)
            ws = self.ex.planned_workspace_bytes(planned)
            if self.active_bytes + nbytes + ws <= self.budget:
                break
            self.ex.discard_plan(planned)
            tk, it = tickets.pop(), items.pop()
            self.ex.discard(it, tk)
            nbytes -= tk.req.nbytes() + 64
            if not tickets:
                if not self.inflight and self.active_bytes == 0:
                    # alone on an idle device it still does not fit: refuse it
                    tk.error = (f"request needs {tk.req.nbytes() + 64 + ws} bytes with its "
                                f"workspace; the budget is {self.budget}")
                    tk.done = True
                    tk.t_done = self.clock()
                    self.failed.append(tk)
                else:
                    self.waiting.appendleft(tk)
                return
            self.waiting.appendleft(tk)
        now = self.clock()
        for tk in tickets:
            tk.t_admit = now
            tk.tick = self._ticks
            tk.charged = tk.req.nbytes() + 64
        token = self.ex.launch(items, planned)
        self._ticks += 1
        self.active_bytes += nbytes + ws
        self.high_water = max(self.high_water, self.active_bytes)
        self.max_inflight_seen = max(self.max_inflight_seen, len(self.inflight) + 1)
        self.inflight.append((token, tickets, items, ws))

    def poll(self):
        """Retire finished ticks, then launch a tick of admitted requests."""
        self._retire()
        self._admit()

    def idle(self) -> bool:
        return not self.waiting and not self.inflight

    def drain(self, sleep: float = 0.0):
        while not self.idle():
            self.poll()
            if sleep:
                time.sleep(sleep)

    # ---- statistics ------------------------------------------------------------
    def latency_stats(self, tickets: Optional[List[Ticket]] = None) -> Dict[str, float]:
        ts = self.finished if tickets is None else tickets
        lat = sorted(t.latency for t in ts)
        if not lat:
            return {"count": 0}

        def pct(p):
            return lat[min(len(lat) - 1, int(round(p / 100.0 * (len(lat) - 1))))]
        return {"count": len(lat), "p50_ms": pct(50) * 1e3, "p99_ms": pct(99) * 1e3,
                "mean_ms": sum(lat) / len(lat) * 1e3, "ticks": self._ticks,
                "high_water_bytes": self.high_water, "max_inflight_seen": self.max_inflight_seen}
