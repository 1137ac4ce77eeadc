"""Continuous-batching server for the QTAM forward + inverse transform.

Requests (one segment each) arrive with their own sample rate, length, Q and
row count. The server keeps, per shape bucket, a resident plan and slot
buffers on the device; a request waits in its bucket's queue and is launched,
together with whatever else of that bucket is waiting, as soon as the bucket's
slot buffers are free and a stream is free. Different buckets run on
different streams at the same time, so requests that arrive while others are
on the GPU are admitted as slots and memory free up. A bucket holds two slot
sets (the executor's ``sets_per_bucket``), so arrivals to a bucket whose
launch is in flight go out on the other set without waiting for it. A
bucket's batch runs as a replay of a captured graph (forward + inverse over
the slot count rounded up to a power of two). Device memory is admitted by
footprint: a bucket's resources are created only if they fit the budget,
evicting idle buckets (least recently used) when needed.

Payloads: a request's samples may be a pinned host tensor (then the executor
copies it to its slot with one asynchronous DMA, no host copy) or any array
(staged through the bucket's pinned buffer). Results come back to the host
by DMA into pinned memory; only requests with ``keep_result`` get a host
copy of theirs.

The scheduler (``Server``) is independent of the device: it drives an
executor with ``footprint / prepare / release / launch / poll``. ``GpuExecutor``
is the MI355X one; tests drive the scheduler with a simulated executor.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Any, Callable, Deque, Dict, List, Optional


class Unsupported(RuntimeError):
    """Raised by an executor's prepare() for a shape its device path cannot run."""


@dataclasses.dataclass(frozen=True)
class BucketKey:
    fs: float
    n: int
    q: float
    rows: int
    f_min: float
    f_max: float
    precision: str = "fp32"


@dataclasses.dataclass
class Request:
    rid: int
    key: BucketKey
    data: Any                          # host array of n samples
    arrival: float = 0.0               # seconds on the server clock
    deadline: Optional[float] = None   # drop if not launched by then
    status: str = "queued"             # queued | running | done | rejected | timeout
    launched: Optional[float] = None
    finished: Optional[float] = None
    result: Any = None                 # reconstruction (host), set by the executor
    coeffs: Any = None                 # envelopes (host), if the executor keeps them
    keep_result: bool = True           # False: latency only, no host copy of the result

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


def slot_count(n: int, max_slots: int = 64, target_samples: int = 1 << 23) -> int:
    """Slots per bucket: about target_samples per launch, a power of two."""
    s = max(1, min(max_slots, target_samples // max(n, 1)))
    return 1 << int(math.floor(math.log2(s)))


class Server:
    """Scheduler: bucket queues, HBM admission, stream assignment."""

    def __init__(self, executor, hbm_budget: int, streams: int = 4, max_slots: int = 64,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.streams = int(streams)
        self.max_slots = int(max_slots)
        self.clock = clock
        self.queues: Dict[BucketKey, Deque[Request]] = collections.OrderedDict()
        self.resources: Dict[BucketKey, Any] = {}      # prepared bucket -> executor handle
        self.footprints: Dict[BucketKey, int] = {}
        self.last_use: Dict[BucketKey, float] = {}
        self.busy: Dict[BucketKey, List[Any]] = {}     # bucket -> its launches in flight
        self.sets = max(1, int(getattr(executor, "sets_per_bucket", 1)))
        self.stream_busy = [None] * self.streams       # stream -> bucket in flight
        self.used = 0
        self.peak_used = 0
        self.done: List[Request] = []
        self.launches = 0
        self.evictions = 0

    # -- submission --------------------------------------------------------
    def submit(self, req: Request) -> Request:
        fp = self.ex.footprint(req.key, slot_count(req.key.n, self.max_slots))
        if fp > self.budget:
            req.status = "rejected"
            req.finished = self.clock()
            self.done.append(req)
            return req
        self.queues.setdefault(req.key, collections.deque()).append(req)
        return req

    def pending(self) -> int:
        return sum(len(q) for q in self.queues.values()) + sum(len(t) for t in self.busy.values())

    # -- one scheduling pass -----------------------------------------------
    def step(self) -> int:
        """Retire finished launches, drop expired requests, admit and launch.
        Returns the number of launches started."""
        now = self.clock()
        for key, toks in list(self.busy.items()):
            for tok in list(toks):
                if self.ex.poll(tok):
                    t = self.clock()
                    for r in tok.requests:
                        r.status = "done"
                        r.finished = t
                        self.done.append(r)
                    self.stream_busy[tok.stream] = None
                    toks.remove(tok)
                    self.last_use[key] = t
            if not toks:
                del self.busy[key]
        for key, q in self.queues.items():
            while q and q[0].deadline is not None and q[0].deadline < now:
                r = q.popleft()
                r.status = "timeout"
                r.finished = now
                self.done.append(r)
        started = 0
        # oldest waiting request first
        order = sorted(((q[0].arrival, i, key) for i, (key, q) in enumerate(self.queues.items())
                        if q and len(self.busy.get(key, ())) < self.sets), key=lambda e: (e[0], e[1]))
        for _, _, key in order:
            free = [i for i, b in enumerate(self.stream_busy) if b is None]
            if not free:
                break
            if key not in self.resources:
                try:
                    admitted = self._admit(key)
                except Unsupported as e:        # the device path cannot run this shape
                    for r in self.queues.pop(key):
                        r.status = "rejected"
                        r.result = repr(e)
                        r.finished = self.clock()
                        self.done.append(r)
                    continue
                if not admitted:
                    continue
            q = self.queues[key]
            slots = slot_count(key.n, self.max_slots)
            batch = [q.popleft() for _ in range(min(slots, len(q)))]
            t = self.clock()
            for r in batch:
                r.status = "running"
                r.launched = t
            tok = self.ex.launch(self.resources[key], batch, free[0])
            tok.requests = batch
            tok.stream = free[0]
            self.busy.setdefault(key, []).append(tok)
            self.stream_busy[free[0]] = key
            self.last_use[key] = t
            self.launches += 1
            started += 1
        return started

    def _admit(self, key: BucketKey) -> bool:
        slots = slot_count(key.n, self.max_slots)
        need = self.ex.footprint(key, slots)
        if self.used + need > self.budget:
            idle = sorted((k for k in self.resources if k not in self.busy and not self.queues.get(k)),
                          key=lambda k: self.last_use.get(k, 0.0))
            for k in idle:
                if self.used + need <= self.budget:
                    break
                self.ex.release(self.resources.pop(k))
                self.used -= self.footprints.pop(k)
                self.evictions += 1
            if self.used + need > self.budget:
                return False
        self.resources[key] = self.ex.prepare(key, slots)
        self.footprints[key] = need
        self.used += need
        self.peak_used = max(self.peak_used, self.used)
        return True

    # -- driving ------------------------------------------------------------
    def drain(self, timeout: float = 60.0):
        t0 = self.clock()
        while self.pending() and self.clock() - t0 < timeout:
            if not self.step():
                self.ex.idle()

    def run_stream(self, arrivals, make_request: Callable[[Any], Request], timeout: float = 120.0):
        """Replay arrivals (objects with .arrival seconds) in real time."""
        t0 = self.clock()
        i = 0
        items = sorted(arrivals, key=lambda a: a.arrival)
        while i < len(items) or self.pending():
            now = self.clock() - t0
            while i < len(items) and items[i].arrival <= now:
                r = make_request(items[i])
                r.arrival = t0 + items[i].arrival
                self.submit(r)
                i += 1
            if not self.step():
                self.ex.idle()
            if now > timeout + (items[-1].arrival if items else 0.0):
                break

    def shutdown(self):
        for key in list(self.resources):
            for tok in self.busy.pop(key, []):
                while not self.ex.poll(tok):
                    self.ex.idle()
            self.ex.release(self.resources.pop(key))
        self.used = 0

    # -- statistics ---------------------------------------------------------
    def stats(self) -> dict:
        done = [r for r in self.done if r.status == "done"]
        lat = sorted(r.latency for r in done)
        if not lat:
            return dict(completed=0)
        span = max(r.finished for r in done) - min(r.arrival for r in done)
        samples = sum(r.key.n for r in done)

        def pct(p):
            return lat[min(len(lat) - 1, int(math.ceil(p / 100.0 * len(lat))) - 1)]

        return dict(completed=len(done), rejected=sum(r.status == "rejected" for r in self.done),
                    timeouts=sum(r.status == "timeout" for r in self.done),
                    p50_ms=1e3 * pct(50), p99_ms=1e3 * pct(99), max_ms=1e3 * lat[-1],
                    samples_per_s=samples / span if span > 0 else float("nan"),
                    launches=self.launches, buckets=len(self.footprints) + self.evictions,
                    evictions=self.evictions, peak_hbm_bytes=self.peak_used)


class _Token:
    """One launch in flight: set by the executor (event, buffers) and the
    server (requests, stream)."""


class GpuExecutor:
    """MI355X executor: plans resident per bucket and ``sets_per_bucket`` slot
    sets (device buffers, workspace, pinned host staging) per bucket, one
    captured graph of forward + inverse per (slot set, power-of-two slot
    count), one HIP stream per server stream."""

    def __init__(self, streams: int = 4, keep_coeffs: bool = False, device: str = "cuda", sets_per_bucket: int = 2):
        import torch
        from .binding import Plan
        self.torch = torch
        self.Plan = Plan
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(streams)]
        self.keep_coeffs = keep_coeffs
        self.sets_per_bucket = max(1, int(sets_per_bucket))
        self.plans: Dict[BucketKey, Any] = {}

    def _plan(self, key: BucketKey):
        p = self.plans.get(key)
        if p is None:
            p = self.Plan(key.fs, key.n, key.q, key.f_min, key.f_max, key.rows, precision=key.precision)
            self.plans[key] = p
        return p

    def footprint(self, key: BucketKey, slots: int) -> int:
        from .binding import Plan
        p = self.plans.get(key) or Plan(key.fs, key.n, key.q, key.f_min, key.f_max, key.rows,
                                        precision=key.precision, host_only=True)
        b = 8 if key.precision == "fp64" else 4
        per = 2 * b * key.n + 2 * b * p.R * p.N_out
        return self.sets_per_bucket * (slots * per + p.workspace_bytes(slots)) + 32 * p.info.sum_len + 16 * p.info.n_bins

    def prepare(self, key: BucketKey, slots: int):
        from .binding import QtamError, QTAM_ERR_UNSUPPORTED
        torch = self.torch
        try:
            p = self._plan(key)
        except QtamError as e:
            if e.status == QTAM_ERR_UNSUPPORTED:
                raise Unsupported(str(e)) from e
            raise
        rdt = torch.float64 if p.fp64 else torch.float32
        cdt = torch.complex128 if p.fp64 else torch.complex64

        def slot_set():
            return dict(x=torch.zeros(slots, key.n, dtype=rdt, device=self.device),
                        y=torch.zeros(slots, p.R, p.N_out, dtype=cdt, device=self.device),
                        xr=torch.zeros(slots, key.n, dtype=rdt, device=self.device),
                        ws=torch.empty(p.workspace_bytes(slots), dtype=torch.uint8, device=self.device),
                        hin=torch.zeros(slots, key.n, dtype=rdt, pin_memory=True),
                        hout=torch.zeros(slots, key.n, dtype=rdt, pin_memory=True),
                        graphs={}, in_use=False)

        return dict(plan=p, slots=slots, dtype=rdt, sets=[slot_set() for _ in range(self.sets_per_bucket)])

    def warm(self, res):
        """Capture every graph of every slot set of a prepared bucket."""
        for ss in res["sets"]:
            n = 1
            while n <= res["slots"]:
                self._graph(res, ss, n)
                n *= 2

    def _graph(self, res, ss, count: int):
        torch = self.torch
        k = 1 << max(0, math.ceil(math.log2(max(count, 1))))
        k = min(k, res["slots"])
        g = ss["graphs"].get(k)
        if g is None:
            p = res["plan"]
            x, y, xr, ws = ss["x"][:k], ss["y"][:k], ss["xr"][:k], ss["ws"]
            s = torch.cuda.Stream(device=self.device)
            s.wait_stream(torch.cuda.current_stream(self.device))
            with torch.cuda.stream(s):      # warm-up outside capture
                p.forward(x, out=y, ws=ws, stream=s)
                p.inverse(y, out=xr, ws=ws, stream=s)
            s.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=s):
                cs = torch.cuda.current_stream(self.device)
                p.forward(x, out=y, ws=ws, stream=cs)
                p.inverse(y, out=xr, ws=ws, stream=cs)
            torch.cuda.synchronize(self.device)
            ss["graphs"][k] = g
        return g, k

    def release(self, res):
        res.clear()

    def launch(self, res, batch: List[Request], stream_idx: int):
        torch = self.torch
        s = self.streams[stream_idx]
        n = len(batch)
        ss = next(x for x in res["sets"] if not x["in_use"])
        g, k = self._graph(res, ss, n)
        tok = _Token()
        with torch.cuda.stream(s):
            for i, r in enumerate(batch):
                d = r.data
                if isinstance(d, torch.Tensor) and d.is_pinned() and d.dtype == res["dtype"]:
                    ss["x"][i].copy_(d, non_blocking=True)           # DMA from the request's pinned payload
                else:
                    ss["hin"][i].copy_(torch.as_tensor(d, dtype=res["dtype"]))
                    ss["x"][i].copy_(ss["hin"][i], non_blocking=True)
            g.replay()
            tok.event = torch.cuda.Event()
            tok.event.record(s)
            ss["hout"][:n].copy_(ss["xr"][:n], non_blocking=True)
            if self.keep_coeffs:
                tok.coeffs = ss["y"][:n].clone()
            tok.copied = torch.cuda.Event()
            tok.copied.record(s)
        ss["in_use"] = True
        tok.set = ss
        tok.count = n
        return tok

    def poll(self, tok) -> bool:
        if not tok.copied.query():
            return False
        for i, r in enumerate(tok.requests):
            if r.keep_result:
                r.result = tok.set["hout"][i].numpy().copy()
            if self.keep_coeffs:
                r.coeffs = tok.coeffs[i].cpu().numpy()
        tok.set["in_use"] = False
        return True

    def idle(self):
        time.sleep(20e-6)


def plain_run(requests: List[Request], plans: Optional[dict] = None, device: str = "cuda"):
    """The plain form: one segment per launch, no graph, synchronous, in
    arrival order. Returns elapsed seconds; fills r.result."""
    import torch
    from .binding import Plan
    plans = {} if plans is None else plans
    t0 = time.perf_counter()
    for r in requests:
        key = r.key
        p = plans.get(key)
        if p is None:
            p = plans[key] = Plan(key.fs, key.n, key.q, key.f_min, key.f_max, key.rows, precision=key.precision)
        rdt = torch.float64 if p.fp64 else torch.float32
        x = torch.as_tensor(r.data, dtype=rdt).to(device)
        xr = p.inverse(p.forward(x))
        r.result = xr.cpu().numpy()
        r.status = "done"
    torch.cuda.synchronize()
    return time.perf_counter() - t0
