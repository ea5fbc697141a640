"""Continuous-batching request loop over the resident index.

Requests (a batch of queries with one pool size L and result count K)
arrive over time. A request is admitted as soon as a slot is free and the
queries already on the GPU leave room under the in-flight budget (the number
of queries whose search state fits on chip at once); admitted requests run
on their slot's own stream, so searches of different requests overlap on the
device while new requests keep arriving. Each slot owns pinned host staging
buffers and device buffers sized for the largest request, so the loop
allocates nothing per request.

The scheduler is independent of the device: ``GpuDevice`` launches through
the library, ``FakeDevice`` (tests) completes requests after scripted times.
Nothing here changes a query's result: a request's output is the same alone
and in any mix.
"""

from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float            # seconds from the start of the run
    queries: np.ndarray       # [b, d] float32 (host)
    L: int
    K: int
    # filled by the server
    admitted: float = -1.0
    finished: float = -1.0
    slot: int = -1
    ids: np.ndarray | None = None
    dists: np.ndarray | None = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Scheduler:
    """FIFO admission under a slot count and an in-flight query budget."""

    def __init__(self, device, n_slots: int, inflight_budget: int):
        if n_slots < 1 or inflight_budget < 1:
            raise ValueError("need at least one slot and a positive budget")
        self.dev = device
        self.free = list(range(n_slots))[::-1]
        self.budget = inflight_budget
        self.inflight = 0
        self.running: dict[int, Request] = {}
        self.waiting: collections.deque[Request] = collections.deque()
        self.done: list[Request] = []
        self.max_inflight_seen = 0
        self.max_running_seen = 0

    def submit(self, r: Request):
        self.waiting.append(r)

    def _fits(self, r: Request) -> bool:
        # an oversized request is admitted alone rather than starved
        return self.inflight + len(r.queries) <= self.budget or self.inflight == 0

    def step(self, now: float) -> int:
        """Retire finished requests, then admit waiting ones in arrival order.
        Returns the number of state changes."""
        changes = 0
        for slot, r in list(self.running.items()):
            if self.dev.poll(slot):
                r.ids, r.dists = self.dev.result(slot, len(r.queries), r.K)
                r.finished = self.dev.now() if hasattr(self.dev, "now") else now
                del self.running[slot]
                self.free.append(slot)
                self.inflight -= len(r.queries)
                self.done.append(r)
                changes += 1
        while self.waiting and self.free and self._fits(self.waiting[0]):
            r = self.waiting.popleft()
            slot = self.free.pop()
            r.slot = slot
            r.admitted = now
            self.inflight += len(r.queries)
            self.max_inflight_seen = max(self.max_inflight_seen, self.inflight)
            self.running[slot] = r
            self.max_running_seen = max(self.max_running_seen, len(self.running))
            self.dev.launch(slot, r)
            changes += 1
        return changes

    def idle(self) -> bool:
        return not self.running and not self.waiting


def run(requests: list[Request], scheduler: Scheduler, clock=None, spin_sleep: float = 0.0):
    """Feed requests at their arrival times and run the scheduler until every
    request has finished. ``clock`` returns seconds since the start."""
    if clock is None:
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0  # noqa: E731
    pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
    while pending or not scheduler.idle():
        now = clock()
        while pending and pending[0].arrival <= now:
            scheduler.submit(pending.popleft())
        if scheduler.step(now) == 0 and spin_sleep:
            time.sleep(spin_sleep)
    return scheduler.done


def poisson_requests(rng, n_req: int, rate: float, pool_q: np.ndarray, L_choices, K: int,
                     max_batch: int = 256, min_batch: int = 1):
    """Arrivals of a Poisson process (rate requests/s); batch sizes uniform in
    [min_batch, max_batch]; each request draws its queries from pool_q and one
    pool size from L_choices. Returns (requests, query index per request)."""
    t = 0.0
    reqs, picks = [], []
    for i in range(n_req):
        t += rng.exponential(1.0 / rate)
        b = int(rng.integers(min_batch, max_batch + 1))
        idx = rng.integers(0, len(pool_q), size=b)
        reqs.append(Request(i, t, np.ascontiguousarray(pool_q[idx]), int(rng.choice(L_choices)), K))
        picks.append(idx)
    return reqs, picks


def summarize(done: list[Request]) -> dict:
    lat = np.array([r.latency for r in done])
    nq = sum(len(r.queries) for r in done)
    span = max(r.finished for r in done) - min(r.arrival for r in done)
    return {"requests": len(done), "queries": int(nq), "makespan_s": span, "qps": nq / span,
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3)}


class FakeDevice:
    """Scripted device for scheduler tests: a request finishes ``cost(r)``
    seconds of simulated time after its launch."""

    def __init__(self, cost, clock):
        self.cost, self.clock = cost, clock
        self.end: dict[int, float] = {}
        self.launched: list[tuple[int, int]] = []
        self.req: dict[int, Request] = {}

    def launch(self, slot, r):
        self.end[slot] = self.clock() + self.cost(r)
        self.req[slot] = r
        self.launched.append((slot, r.rid))

    def poll(self, slot):
        return self.clock() >= self.end[slot]

    def result(self, slot, b, K):
        r = self.req.pop(slot)
        return np.tile(np.arange(K, dtype=np.int32), (b, 1)) + r.rid, np.zeros((b, K), np.float32)


class GpuDevice:
    """Slots backed by one stream each, pinned staging buffers and device
    buffers for up to ``max_batch`` queries; searches run in libssg."""

    def __init__(self, base, graph, entry_ids, n_slots: int, max_batch: int, max_K: int,
                 metric: str = "l2", dim_scale=None, base_f32=None, rerank: bool = False):
        import torch

        from .binding import search
        self.torch, self.search = torch, search
        self.index = (base, graph, entry_ids)
        self.metric, self.dim_scale, self.base_f32, self.rerank = metric, dim_scale, base_f32, rerank
        dev = base.device
        d = base.shape[1]
        self.slots = []
        for _ in range(n_slots):
            self.slots.append(dict(
                stream=torch.cuda.Stream(device=dev),  # default priority
                hq=torch.empty((max_batch, d), dtype=torch.float32, pin_memory=True),
                dq=torch.empty((max_batch, d), dtype=torch.float32, device=dev),
                di=torch.empty((max_batch, max_K), dtype=torch.int32, device=dev),
                dd=torch.empty((max_batch, max_K), dtype=torch.float32, device=dev),
                hi=torch.empty((max_batch, max_K), dtype=torch.int32, pin_memory=True),
                hd=torch.empty((max_batch, max_K), dtype=torch.float32, pin_memory=True),
                ev=torch.cuda.Event(), b=0, K=0))

    def launch(self, slot, r: Request):
        torch = self.torch
        s = self.slots[slot]
        b, K = len(r.queries), r.K
        s["hq"][:b].numpy()[:] = r.queries  # the slot's previous copy has completed
        with torch.cuda.stream(s["stream"]):
            q = s["dq"][:b]
            q.copy_(s["hq"][:b], non_blocking=True)
            ids = s["di"].view(-1)[:b * K].view(b, K)
            dd = s["dd"].view(-1)[:b * K].view(b, K)
            kw = dict(base_f32=self.base_f32, rerank_k=K) if self.rerank else {}
            self.search(self.index[0], self.index[1], self.index[2], q, K, r.L, self.metric,
                        dim_scale=self.dim_scale, out=(ids, dd), stream=s["stream"], **kw)
            s["hi"].view(-1)[:b * K].copy_(ids.view(-1), non_blocking=True)
            s["hd"].view(-1)[:b * K].copy_(dd.view(-1), non_blocking=True)
            s["ev"].record(s["stream"])

    def poll(self, slot):
        return self.slots[slot]["ev"].query()

    def result(self, slot, b, K):
        s = self.slots[slot]
        return (s["hi"].view(-1)[:b * K].view(b, K).numpy().copy(),
                s["hd"].view(-1)[:b * K].view(b, K).numpy().copy())
