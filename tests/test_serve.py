"""CPU tests of the serving loop's scheduler (admission by bytes, continuous
batching, FIFO order per kind, failure isolation) with a fake backend that
sleeps instead of running kernels.  The GPU test of the real backend is in
test_gpu_serve.py."""
from __future__ import annotations

import threading
import time

import pytest

from paper_2311_12133_amd.serve import Request, Server, summarize


class FakeBackend:
    def __init__(self, per_item=0.004):
        self.per_item = per_item
        self.lock = threading.Lock()
        self.inflight = 0
        self.peak = 0
        self.batches = []

    def make_slot(self, i):
        return dict(id=i)

    def close_slot(self, slot):
        pass

    def prepare(self, r):
        r.mem = r.data["mem"]
        r.in_bytes = 100

    def run(self, batch, slot):
        mem = sum(r.mem for r in batch)
        with self.lock:
            self.inflight += mem
            self.peak = max(self.peak, self.inflight)
            self.batches.append([r.rid for r in batch])
        try:
            if any(r.data.get("raise") for r in batch):
                raise RuntimeError("device error")
            time.sleep(self.per_item * len(batch))
            for r in batch:
                if r.data.get("fail"):
                    r.error = -2
                else:
                    r.result = ("ok", r.rid)
        finally:
            with self.lock:
                self.inflight -= mem


def reqs(n, gap, mem=10, op_cycle=("compress", "decompress"), extra=None):
    out = []
    for i in range(n):
        d = dict(mem=mem)
        d.update((extra or {}).get(i, {}))
        r = Request(rid=i, op=op_cycle[i % len(op_cycle)], arrival=i * gap, data=d)
        r.out_bytes = 100
        out.append(r)
    return out


def test_all_complete_and_stats():
    be = FakeBackend()
    srv = Server(slots=3, hbm_budget=1000, max_batch=4, backend=be)
    rs = reqs(40, 0.001)
    st = srv.run(rs)
    assert st["completed"] == 40 and st["failed"] == 0
    for r in rs:
        assert r.result == ("ok", r.rid)
        assert r.arrival <= r.admitted + 1e-6 <= r.done + 2e-6
    assert st["p50_ms"] <= st["p99_ms"]
    assert st["compress"]["n"] == 20 and st["decompress"]["n"] == 20


def test_budget_is_never_exceeded():
    be = FakeBackend(per_item=0.003)
    srv = Server(slots=4, hbm_budget=100, max_batch=8, backend=be)
    rs = reqs(30, 0.0005, mem=30)
    st = srv.run(rs)
    assert st["completed"] == 30
    assert be.peak <= 100
    assert max(len(b) for b in be.batches) <= 3


def test_continuous_batching_joins_waiting_requests():
    be = FakeBackend(per_item=0.01)
    srv = Server(slots=1, hbm_budget=10_000, max_batch=16, backend=be)
    # one kind only: while the first batch runs, the rest queue up and go together
    rs = reqs(12, 0.001, op_cycle=("compress",))
    st = srv.run(rs)
    assert st["completed"] == 12
    assert len(be.batches) < 12
    assert st["mean_batch"] > 1


def test_fifo_within_a_kind():
    be = FakeBackend(per_item=0.002)
    srv = Server(slots=2, hbm_budget=10_000, max_batch=3, backend=be)
    rs = reqs(30, 0.0003)
    srv.run(rs)
    order = [rid for b in be.batches for rid in b]
    for op in ("compress", "decompress"):
        ids = [i for i in order if rs[i].op == op]
        assert ids == sorted(ids)


def test_failures_are_isolated():
    be = FakeBackend()
    srv = Server(slots=2, hbm_budget=100, max_batch=4, backend=be)
    rs = reqs(12, 0.001, mem=10, extra={3: dict(fail=True), 5: dict(mem=500), 8: dict(raise_=1)})
    rs[8].data["raise"] = True
    st = srv.run(rs)
    assert rs[3].error == -2 and rs[3].result is None
    assert rs[5].error == -2  # larger than the whole budget
    assert rs[8].error != 0
    bad = {3, 5, 8}
    # the batch that raised fails as a whole; every other request completes
    raised = next(b for b in be.batches if 8 in b)
    for r in rs:
        if r.rid not in bad and r.rid not in raised:
            assert r.error == 0 and r.result == ("ok", r.rid)
    assert st["failed"] >= 3


def test_summary_percentiles():
    rs = []
    for i in range(100):
        r = Request(rid=i, op="compress", arrival=0.0, data=None)
        r.done = (i + 1) / 1000.0
        r.in_bytes = 4
        rs.append(r)
    st = summarize(rs)
    assert st["p50_ms"] == pytest.approx(50.0)
    assert st["p99_ms"] == pytest.approx(99.0)


class HoldingBackend(FakeBackend):
    """Results stay on the device: each successful request holds
    data["result_bytes"] until the caller releases it."""

    def __init__(self, per_item=0.002, keep=0):
        super().__init__(per_item)
        self.keep = keep
        self.held = 0
        self.peak_charged = 0
        self.srv = None

    def reserved_bytes(self, slots):
        return slots * self.keep

    def result_bytes(self, r):
        return r.data.get("result_bytes", 0) if r.result is not None else 0

    def run(self, batch, slot):
        with self.lock:
            # everything the server has charged while this batch starts
            self.peak_charged = max(self.peak_charged, self.srv.charged)
        super().run(batch, slot)


def test_held_results_and_reserve_are_charged():
    be = HoldingBackend(keep=50)
    srv = Server(slots=2, hbm_budget=400, max_batch=4, backend=be)
    be.srv = srv
    assert srv.charged == 100  # the two slots' kept workspace
    rs = reqs(40, 0.0005, mem=60, extra={i: dict(result_bytes=20) for i in range(40)})
    kept = []

    def on_done(r):
        kept.append(r)
        if len(kept) > 5:  # the caller keeps the last five results
            srv.release(kept.pop(0))

    st = srv.run(rs, on_done=on_done)
    assert st["completed"] == 40
    assert be.peak_charged <= 400
    # the five kept results are still charged, the rest returned
    assert srv.charged == 100 + 5 * 20
    for r in kept:
        srv.release(r)
    assert srv.charged == 100


def test_unreleased_results_cannot_stall_the_server():
    # the caller never releases: once results fill the budget, requests that
    # cannot fit fail instead of waiting forever
    be = HoldingBackend()
    srv = Server(slots=2, hbm_budget=200, max_batch=2, backend=be)
    be.srv = srv
    rs = reqs(20, 0.001, mem=50, extra={i: dict(result_bytes=40) for i in range(20)})
    st = srv.run(rs)
    assert st["completed"] + st["failed"] == 20
    assert st["failed"] > 0
    assert all(r.error == -2 for r in rs if r.error)


def test_reserve_larger_than_budget_rejected():
    with pytest.raises(ValueError):
        Server(slots=4, hbm_budget=100, backend=HoldingBackend(keep=30))
