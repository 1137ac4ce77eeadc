"""Scheduler logic of the continuous-batching server, driven by a simulated
executor on a manual clock (no GPU)."""
import math

import pytest

from paper_2603_29785_amd.serving import BucketKey, Request, Server, Unsupported, slot_count


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Launches take 1 ms + 1 ns per sample; memory is counted, not used."""

    def __init__(self, clock, fail_shapes=()):
        self.clock = clock
        self.prepared = {}
        self.live = 0
        self.max_live = 0
        self.in_flight = 0
        self.max_in_flight = 0
        self.launch_log = []
        self.fail_shapes = set(fail_shapes)

    def footprint(self, key, slots):
        return slots * key.n * 16 + 1000

    def prepare(self, key, slots):
        if key.n in self.fail_shapes:
            raise Unsupported("shape not on the device path")
        h = object()
        self.prepared[h] = key
        self.live += 1
        self.max_live = max(self.max_live, self.live)
        return h

    def release(self, h):
        del self.prepared[h]
        self.live -= 1

    def launch(self, h, batch, stream):
        class Tok:
            pass
        tok = Tok()
        tok.end = self.clock() + 1e-3 + 1e-9 * sum(r.key.n for r in batch)
        self.in_flight += 1
        self.max_in_flight = max(self.max_in_flight, self.in_flight)
        self.launch_log.append((self.prepared[h], len(batch), stream, self.clock()))
        return tok

    def poll(self, tok):
        if self.clock() >= tok.end and not getattr(tok, "seen", False):
            tok.seen = True
            self.in_flight -= 1
            for r in tok.requests:
                r.result = r.data
            return True
        return getattr(tok, "seen", False)

    def idle(self):
        self.clock.t += 1e-4


def key(n, q=8.0, rows=64):
    return BucketKey(4096.0, n, q, rows, 10.0, 2048.0)


def make(rid, k, t=0.0, deadline=None):
    return Request(rid, k, data=rid, arrival=t, deadline=deadline)


def test_slot_count_powers_of_two():
    assert slot_count(4096) == 64 and slot_count(1 << 20) == 8 and slot_count(1 << 24) == 1
    for n in (4096, 16384, 65536, 1 << 18, 1 << 20):
        s = slot_count(n)
        assert s & (s - 1) == 0


def test_same_bucket_batches_and_fifo():
    c = Clock()
    ex = FakeExecutor(c)
    srv = Server(ex, hbm_budget=1 << 40, streams=2, max_slots=4, clock=c)
    k = key(1 << 20)
    for i in range(10):
        srv.submit(make(i, k))
    srv.drain()
    assert [r.rid for r in srv.done] == list(range(10))        # FIFO within a bucket
    sizes = [b for (_, b, _, _) in ex.launch_log]
    assert sizes == [4, 4, 2]                                   # slots fill, then the rest
    assert all(r.result == r.rid for r in srv.done)


def test_buckets_overlap_on_streams():
    c = Clock()
    ex = FakeExecutor(c)
    srv = Server(ex, hbm_budget=1 << 40, streams=4, clock=c)
    for i, n in enumerate([4096, 16384, 65536, 1 << 18, 4096, 16384]):
        srv.submit(make(i, key(n)))
    srv.drain()
    assert ex.max_in_flight >= 3
    assert len(srv.done) == 6 and all(r.status == "done" for r in srv.done)


def test_hbm_admission_evicts_idle_and_waits():
    c = Clock()
    ex = FakeExecutor(c)
    k1, k2, k3 = key(1 << 18, 4), key(1 << 18, 8), key(1 << 18, 16)
    one = ex.footprint(k1, slot_count(k1.n))
    srv = Server(ex, hbm_budget=2 * one, streams=4, clock=c)
    for i, k in enumerate([k1, k2, k3]):
        srv.submit(make(i, k))
    srv.step()
    assert ex.live == 2 and srv.used <= srv.budget                # third waits for memory
    srv.drain()
    assert len(srv.done) == 3 and srv.evictions >= 1
    assert srv.peak_used <= srv.budget and ex.max_live <= 2


def test_oversized_rejected_and_unsupported_reported():
    c = Clock()
    ex = FakeExecutor(c, fail_shapes={1 << 16})
    srv = Server(ex, hbm_budget=10 ** 8, clock=c)
    r = srv.submit(make(0, key(1 << 20)))
    assert r.status == "rejected"
    srv.submit(make(1, key(1 << 16)))
    srv.submit(make(2, key(4096)))
    srv.drain()
    st = {x.rid: x.status for x in srv.done}
    assert st == {0: "rejected", 1: "rejected", 2: "done"}


def test_deadline_timeout():
    c = Clock()
    ex = FakeExecutor(c)
    srv = Server(ex, hbm_budget=1 << 40, streams=1, max_slots=1, clock=c)
    k = key(1 << 20)
    srv.submit(make(0, k))
    srv.submit(make(1, k, deadline=0.0005))   # can only start after request 0 (~2 ms)
    srv.drain()
    st = {x.rid: x.status for x in srv.done}
    assert st == {0: "done", 1: "timeout"}


def test_continuous_arrivals_and_stats():
    c = Clock()
    ex = FakeExecutor(c)
    srv = Server(ex, hbm_budget=1 << 40, streams=4, clock=c)
    k_a, k_b = key(16384), key(65536, 16, 128)

    class A:
        def __init__(self, t, k):
            self.arrival, self.k = t, k

    arr = [A(0.0002 * i, k_a if i % 3 else k_b) for i in range(60)]
    srv.run_stream(arr, lambda a: make(id(a), a.k))
    s = srv.stats()
    assert s["completed"] == 60 and s["p50_ms"] <= s["p99_ms"] <= s["max_ms"]
    # requests that arrived while others ran were batched into later launches
    assert srv.launches < 60
    assert math.isfinite(s["samples_per_s"])


def test_two_slot_sets_let_a_busy_bucket_launch_again():
    """With two slot sets per bucket, requests arriving while the bucket's
    first launch runs go out at once on the second set (and overlap it on
    another stream); a third launch waits until one of them retires."""
    c = Clock()
    ex = FakeExecutor(c)
    ex.sets_per_bucket = 2
    srv = Server(ex, hbm_budget=1 << 40, streams=4, max_slots=2, clock=c)
    k = key(1 << 20)
    srv.submit(make(0, k))
    srv.step()
    srv.submit(make(1, k))
    srv.submit(make(2, k))
    srv.step()
    assert len(ex.launch_log) == 2 and ex.in_flight == 2            # second set in flight beside the first
    assert {s for (_, _, s, _) in ex.launch_log} == {0, 1}
    srv.submit(make(3, k))
    srv.step()
    assert len(ex.launch_log) == 2                                  # both sets busy: request 3 waits
    srv.drain()
    assert [b for (_, b, _, _) in ex.launch_log] == [1, 2, 1]
    assert sorted(r.rid for r in srv.done) == [0, 1, 2, 3] and all(r.status == "done" for r in srv.done)
    # one set: the second launch waits for the first
    c2 = Clock()
    ex1 = FakeExecutor(c2)
    srv1 = Server(ex1, hbm_budget=1 << 40, streams=4, max_slots=2, clock=c2)
    srv1.submit(make(0, k))
    srv1.step()
    srv1.submit(make(1, k))
    srv1.step()
    assert len(ex1.launch_log) == 1
