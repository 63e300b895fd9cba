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
