"""Continuous-batching request loop over the resident index.

Requests (a batch of queries with one pool size L and result count K)
arrive over time. A request is admitted as soon as a slot is free and the
queries already on the GPU leave room under the in-flight budget (the number
of queries whose search state fits on chip at once); admitted requests run
on their slot's own stream, so searches of different requests overlap on the
device while new requests keep arriving. Each slot owns pinned host staging
buffers and device buffers sized for the largest request, so the loop
allocates nothing per request.

Two ways to put requests on the device:

* ``Scheduler`` + ``GpuDevice``: one launch per request, requests overlap on
  per-slot streams;
* ``BatchScheduler`` + ``GpuBatchDevice`` (continuous batching): whenever a
  batch slot is free, the waiting requests that fit the device budget (FIFO)
  are launched together as one mixed batch through the batched entry point
  (``ssg_search_batched``: one launch per L bucket, one wavefront per query),
  each query with its own request's pool size L and result count K.
  This keeps the device full with a few launches at a time instead of one
  launch per request.

Admission budget (``DeviceBudget``): a query in flight holds on-chip state
(LDS: its pool, merge stage and visited set, sized by its L bucket; the
library reports the bytes) and HBM staging (its query row, L and K, and its
K output rows). A batch is admitted only while the in-flight totals stay
within the budget: the LDS budget is the bytes of the searches the GPU holds
at once, times an oversubscription factor (queued waves start as soon as
resident ones finish); the HBM budget is the staging and output memory the
device preallocated. A request that can never fit (more queries or a larger
K than a slot holds, or more bytes than the whole budget) is finished at once
with an error instead of stalling the queue.

The schedulers are independent of the device: the GPU devices launch through
the library, the fake devices (tests) complete work after scripted times.
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
    error: str | None = None

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
        cap = getattr(self.dev, "max_queries", None)
        kmax = getattr(self.dev, "max_K", None)
        if (cap is not None and len(r.queries) > cap) or (kmax is not None and r.K > kmax):
            _reject(r, f"request of {len(r.queries)} queries with K = {r.K} exceeds a slot "
                       f"({cap} queries, K <= {kmax})", self.done)
            return
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


def _reject(r: Request, msg: str, done: list):
    r.error = msg
    r.admitted = r.finished = r.arrival
    done.append(r)


class DeviceBudget:
    """Byte budget for the queries in flight on one device.

    lds_bytes:  on-chip bytes the in-flight searches may hold together
    hbm_bytes:  staging + output bytes they may hold together
    lds_of:     L -> LDS bytes of one search of pool size L
    hbm_of:     K -> HBM bytes of one query with K results
    """

    def __init__(self, lds_bytes: int, hbm_bytes: int, lds_of, hbm_of):
        if lds_bytes < 1 or hbm_bytes < 1:
            raise ValueError("budgets must be positive")
        self.lds_bytes, self.hbm_bytes = int(lds_bytes), int(hbm_bytes)
        self.lds_of, self.hbm_of = lds_of, hbm_of

    def cost(self, r: Request) -> tuple[int, int]:
        b = len(r.queries)
        return b * int(self.lds_of(r.L)), b * int(self.hbm_of(r.K))


class BatchScheduler:
    """Continuous batching: whenever one of ``n_slots`` batch slots is free,
    the waiting requests are taken in arrival order while their queries fit
    ``max_batch`` and the bytes of everything in flight fit ``budget`` (a
    ``DeviceBudget``; None = queries alone), and launched as one batch. A
    request waits while the budget is taken (FIFO: later requests wait behind
    it) and is rejected if it could never fit."""

    def __init__(self, device, n_slots: int, max_batch: int, budget: DeviceBudget | None = None):
        if n_slots < 1 or max_batch < 1:
            raise ValueError("need at least one slot and a positive batch size")
        self.dev = device
        self.free = list(range(n_slots))[::-1]
        cap = getattr(device, "max_queries", None)
        self.max_batch = min(max_batch, cap) if cap else max_batch
        self.max_K = getattr(device, "max_K", None)
        self.budget = budget
        self.inflight = [0, 0]  # LDS, HBM bytes of admitted, unfinished batches
        self.batch_cost: dict[int, tuple[int, int]] = {}
        self.running: dict[int, list[Request]] = {}
        self.waiting: collections.deque[Request] = collections.deque()
        self.done: list[Request] = []
        self.batches = 0
        self.max_running_seen = 0
        self.max_batch_seen = 0
        self.max_inflight_seen = [0, 0]
        self.budget_waits = 0  # steps where a free slot idled because the budget was taken

    def submit(self, r: Request):
        if len(r.queries) > self.max_batch or (self.max_K is not None and r.K > self.max_K):
            _reject(r, f"request of {len(r.queries)} queries with K = {r.K} exceeds a batch "
                       f"({self.max_batch} queries, K <= {self.max_K})", self.done)
            return
        if self.budget is not None:
            c = self.budget.cost(r)
            if c[0] > self.budget.lds_bytes or c[1] > self.budget.hbm_bytes:
                _reject(r, f"request needs {c[0]} LDS / {c[1]} HBM bytes, over the whole budget "
                           f"({self.budget.lds_bytes} / {self.budget.hbm_bytes})", self.done)
                return
        self.waiting.append(r)

    def _cost(self, r: Request) -> tuple[int, int]:
        return self.budget.cost(r) if self.budget is not None else (0, 0)

    def _fits(self, used, c) -> bool:
        if self.budget is None:
            return True
        return used[0] + c[0] <= self.budget.lds_bytes and used[1] + c[1] <= self.budget.hbm_bytes

    def step(self, now: float) -> int:
        changes = 0
        for slot, reqs in list(self.running.items()):
            if self.dev.poll(slot):
                outs = self.dev.results(slot, reqs)
                t = self.dev.now() if hasattr(self.dev, "now") else now
                for r, (ids, dd) in zip(reqs, outs):
                    r.ids, r.dists, r.finished = ids, dd, t
                    self.done.append(r)
                del self.running[slot]
                c = self.batch_cost.pop(slot)
                self.inflight = [self.inflight[0] - c[0], self.inflight[1] - c[1]]
                self.free.append(slot)
                changes += 1
        while self.waiting and self.free:
            used = list(self.inflight)
            c = self._cost(self.waiting[0])
            if not self._fits(used, c):
                self.budget_waits += 1
                break  # the head waits for bytes to free up; FIFO keeps the rest behind it
            batch = [self.waiting.popleft()]
            used = [used[0] + c[0], used[1] + c[1]]
            total = len(batch[0].queries)
            while self.waiting and total + len(self.waiting[0].queries) <= self.max_batch:
                c = self._cost(self.waiting[0])
                if not self._fits(used, c):
                    break
                r = self.waiting.popleft()
                batch.append(r)
                used = [used[0] + c[0], used[1] + c[1]]
                total += len(r.queries)
            slot = self.free.pop()
            for r in batch:
                r.slot, r.admitted = slot, now
            self.batch_cost[slot] = (used[0] - self.inflight[0], used[1] - self.inflight[1])
            self.inflight = used
            self.max_inflight_seen = [max(a, b) for a, b in zip(self.max_inflight_seen, used)]
            self.running[slot] = batch
            self.batches += 1
            self.max_running_seen = max(self.max_running_seen, len(self.running))
            self.max_batch_seen = max(self.max_batch_seen, total)
            self.dev.launch_batch(slot, batch)
            changes += 1
        return changes

    def idle(self) -> bool:
        return not self.running and not self.waiting


def run(requests: list[Request], scheduler, clock=None, spin_sleep: float = 0.0):
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
    ok = [r for r in done if r.error is None]
    lat = np.array([r.latency for r in ok])
    nq = sum(len(r.queries) for r in ok)
    span = max(r.finished for r in ok) - min(r.arrival for r in ok)
    return {"requests": len(ok), "rejected": len(done) - len(ok), "queries": int(nq),
            "makespan_s": span, "qps": nq / span,
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


class FakeBatchDevice:
    """Scripted batch device for scheduler tests: a batch finishes
    ``cost(batch)`` seconds of simulated time after its launch."""

    def __init__(self, cost, clock):
        self.cost, self.clock = cost, clock
        self.end: dict[int, float] = {}
        self.launched: list[tuple[int, list[int]]] = []

    def launch_batch(self, slot, reqs):
        self.end[slot] = self.clock() + self.cost(reqs)
        self.launched.append((slot, [r.rid for r in reqs]))

    def poll(self, slot):
        return self.clock() >= self.end[slot]

    def results(self, slot, reqs):
        return [(np.tile(np.arange(r.K, dtype=np.int32), (len(r.queries), 1)) + r.rid,
                 np.zeros((len(r.queries), r.K), np.float32)) for r in reqs]


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
        self.max_queries, self.max_K = max_batch, max_K
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


class GpuBatchDevice:
    """Batch slots for ``BatchScheduler``: each slot owns a stream, pinned
    staging buffers and device buffers for up to ``max_batch`` queries, and
    runs a batch through the batched entry point (``ssg_search_batched``)
    with every query's own L and K; nothing is allocated per batch."""

    def __init__(self, base, graph, entry_ids, n_slots: int, max_batch: int, max_K: int,
                 metric: str = "l2", dim_scale=None, base_f32=None, rerank: bool = False,
                 shapes=None):
        import ctypes

        import torch

        from . import _lib
        from .batched import BUCKET_BOUNDS
        from .binding import _DTYPES, _METRICS, _VISITED
        self.torch, self.ctypes, self.lib_mod = torch, ctypes, _lib
        self.visited_map = _VISITED
        self.bounds = BUCKET_BOUNDS
        self.index = (base, graph, entry_ids, dim_scale, base_f32)
        self.dtype, self.metric = _DTYPES[base.dtype], _METRICS[metric]
        self.rerank = -1 if rerank else 0
        self.max_K, self.shapes = max_K, shapes or {}
        self.max_queries, self.n_slots = max_batch, n_slots
        dev = base.device
        d = base.shape[1]
        nbmax = len(BUCKET_BOUNDS)
        wsb = _lib.lib().ssg_batch_workspace_bytes(nbmax)
        self.slots = []
        for _ in range(n_slots):
            ws = torch.empty(wsb + 256, dtype=torch.uint8, device=dev)
            self.slots.append(dict(
                stream=torch.cuda.Stream(device=dev),  # default priority
                hq=torch.empty((max_batch, d), dtype=torch.float32, pin_memory=True),
                hLK=torch.empty((3, max_batch), dtype=torch.int32, pin_memory=True),
                dq=torch.empty((max_batch, d), dtype=torch.float32, device=dev),
                dLK=torch.empty((3, max_batch), dtype=torch.int32, device=dev),
                di=torch.empty((max_batch, max_K), dtype=torch.int32, device=dev),
                dd=torch.empty((max_batch, max_K), dtype=torch.float32, device=dev),
                hi=torch.empty((max_batch, max_K), dtype=torch.int32, pin_memory=True),
                hd=torch.empty((max_batch, max_K), dtype=torch.float32, pin_memory=True),
                ws=ws, wsp=(ws.data_ptr() + 255) & ~255, wsb=wsb,
                ev=torch.cuda.Event(), b=0))

    def launch_batch(self, slot, reqs):
        from .batched import plan_buckets
        torch, ctypes, _lib = self.torch, self.ctypes, self.lib_mod
        s = self.slots[slot]
        b = sum(len(r.queries) for r in reqs)
        if b > s["hq"].shape[0] or any(r.K > self.max_K for r in reqs):
            raise ValueError("batch larger than the slot buffers")
        hq = s["hq"].numpy()
        hLK = s["hLK"].numpy()
        o = 0
        for r in reqs:  # the slot's previous batch has completed (polled)
            m = len(r.queries)
            hq[o:o + m] = r.queries
            hLK[0, o:o + m] = r.L
            hLK[1, o:o + m] = r.K
            o += m
        plan = plan_buckets(hLK[0, :b], self.bounds)
        o = 0
        offs = []
        for _, qi in plan:  # the bucket query lists share row 2
            hLK[2, o:o + len(qi)] = qi
            offs.append(o)
            o += len(qi)
        base, graph, entry, scale, bf32 = self.index
        with torch.cuda.stream(s["stream"]):
            s["dq"][:b].copy_(s["hq"][:b], non_blocking=True)
            for k in range(3):
                s["dLK"][k, :b].copy_(s["hLK"][k, :b], non_blocking=True)
            dLK = s["dLK"]
            desc = _lib.BatchDesc(
                base.data_ptr(), base.shape[0], base.shape[1], self.dtype, self.metric,
                None if scale is None else scale.data_ptr(),
                None if bf32 is None else bf32.data_ptr(), self.rerank, graph.data_ptr(),
                graph.shape[1], entry.data_ptr(), entry.numel(), s["dq"].data_ptr(), b,
                dLK[0].data_ptr(), dLK[1].data_ptr(), self.max_K, s["di"].data_ptr(),
                s["dd"].data_ptr(), None, None)
            arr = (_lib.Bucket * len(plan))()
            for i, ((mL, qi), off) in enumerate(zip(plan, offs)):
                cap = next(x for x in self.bounds if mL <= x)
                sh = self.shapes.get(cap, {})
                arr[i] = _lib.Bucket(dLK[2].data_ptr() + 4 * off, len(qi), mL,
                                     sh.get("gather_variant", 0), sh.get("hash_log2", 0),
                                     sh.get("waves_per_block", 0), sh.get("blocks", 0),
                                     self.visited_map[sh.get("visited", "auto")],
                                     sh.get("queries_per_wave", 0))
            _lib.check(_lib.lib().ssg_search_batched(ctypes.byref(desc), arr, len(plan),
                                                     ctypes.c_void_p(s["wsp"]), s["wsb"],
                                                     ctypes.c_void_p(s["stream"].cuda_stream)))
            s["hi"][:b].copy_(s["di"][:b], non_blocking=True)
            s["hd"][:b].copy_(s["dd"][:b], non_blocking=True)
            s["ev"].record(s["stream"])
        s["b"] = b

    def poll(self, slot):
        return self.slots[slot]["ev"].query()

    def budget(self, oversubscribe: float = 2.0) -> DeviceBudget:
        """The device's byte budget: LDS = compute units x LDS per unit x
        ``oversubscribe`` (searches beyond what the chip holds at once wait
        on the device for a resident one to finish); HBM = the staging and
        output buffers of every slot. Per query: the library's LDS bytes for
        its L, and d * 4 + 12 + K * 8 bytes of staging and output."""
        torch, _lib = self.torch, self.lib_mod
        base, graph = self.index[0], self.index[1]
        props = torch.cuda.get_device_properties(base.device)
        per_cu = getattr(props, "shared_memory_per_multiprocessor", 0) or 160 * 1024
        n, d = base.shape
        R = graph.shape[1]
        memo = {}

        def lds_of(L):
            if L not in memo:
                memo[L] = int(_lib.lib().ssg_query_lds_bytes(L, R, d, self.dtype, n, self.rerank, 0))
                if memo[L] == 0:
                    raise ValueError(f"no search of pool size {L} fits this index")
            return memo[L]

        def hbm_of(K):
            return d * 4 + 12 + K * 8
        return DeviceBudget(int(props.multi_processor_count * per_cu * oversubscribe),
                            self.n_slots * self.max_queries * hbm_of(self.max_K), lds_of, hbm_of)

    def results(self, slot, reqs):
        s = self.slots[slot]
        hi, hd = s["hi"].numpy(), s["hd"].numpy()
        out, o = [], 0
        for r in reqs:
            m = len(r.queries)
            out.append((hi[o:o + m, :r.K].copy(), hd[o:o + m, :r.K].copy()))
            o += m
        return out
