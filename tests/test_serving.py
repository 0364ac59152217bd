"""Serving loop scheduling logic on the CPU: a fake executor (the oracle as
backend, a simulated device-memory budget, completions after a few polls)
exercises admission, back-pressure, ordering and the allocator."""
import numpy as np
import pytest

import oracle
from paper_1912_03732_amd import inputs
from paper_1912_03732_amd.serving import FirstFit, Request, Server, request_bytes, run_open_loop


class FakeExecutor:
    def __init__(self, budget, polls_to_finish=2):
        self.alloc = FirstFit(budget)
        self.polls_to_finish = polls_to_finish
        self.launched = []
        self.peak_used = 0

    def capacity(self):
        return self.alloc.size

    def footprint(self, reqs):
        return 512 + sum(request_bytes(r.n, r.m) for r in reqs)

    def try_launch(self, reqs):
        total = self.footprint(reqs)
        off = self.alloc.alloc(total)
        if off is None:
            return None
        self.peak_used = max(self.peak_used, self.alloc.used)
        self.launched.append([r.rid for r in reqs])
        res = [oracle.walsh_nl(r.table, r.n, r.m) for r in reqs]
        return {"off": off, "total": total, "reqs": list(reqs), "res": res, "polls": 0}

    def poll(self, h):
        h["polls"] += 1
        return h["polls"] >= self.polls_to_finish

    def finish(self, h):
        self.alloc.release(h["off"], h["total"])
        return h["res"]


def _reqs(count, seed=1, sizes=(4, 6, 8)):
    g = inputs.rng(seed)
    out = []
    for i in range(count):
        n = int(g.choice(sizes))
        out.append(Request(i, n, n, inputs.permutation(n, g)))
    return out


def test_first_fit_allocator_coalesces():
    a = FirstFit(4096)
    x = a.alloc(1000)
    y = a.alloc(1000)
    z = a.alloc(1000)
    assert (x, y, z) == (0, 1024, 2048)
    assert a.alloc(2000) is None
    a.release(y, 1000)
    a.release(x, 1000)
    assert a.largest() == 2048 and a.used == 1024
    a.release(z, 1000)
    assert a.free == [[0, 4096]] and a.used == 0


def test_all_requests_complete_with_oracle_results_in_fifo_order():
    ex = FakeExecutor(budget=1 << 20)
    srv = Server(ex, max_batch=5)
    reqs = _reqs(23)
    for r in reqs:
        assert srv.submit(r)
    srv.drain()
    assert len(srv.done) == 23 and not srv.rejected
    launched = [rid for b in ex.launched for rid in b]
    assert launched == list(range(23))  # admitted in arrival order
    assert max(len(b) for b in ex.launched) <= 5
    for r in reqs:
        nl, mx = oracle.walsh_nl(r.table, r.n, r.m)
        assert r.nl == nl and np.array_equal(r.maxabs, mx) and r.status == "done"


def test_memory_budget_bounds_in_flight_work():
    one = 512 + request_bytes(8, 8)
    ex = FakeExecutor(budget=3 * one + 256, polls_to_finish=3)
    srv = Server(ex, max_batch=64, max_inflight=8)
    for r in _reqs(12, sizes=(8,)):
        srv.submit(r)
    srv.drain()
    assert len(srv.done) == 12
    assert ex.peak_used <= ex.capacity()
    assert max(len(b) for b in ex.launched) <= 3


def test_backpressure_rejects_when_queue_full_and_oversize():
    ex = FakeExecutor(budget=1 << 16)
    srv = Server(ex, max_waiting=4)
    reqs = _reqs(6, sizes=(4,))
    ok = [srv.submit(r) for r in reqs]
    assert ok == [True] * 4 + [False] * 2
    assert all(r.status == "rejected" for r in reqs[4:])
    big = Request(99, 14, 14, inputs.permutation(14, inputs.rng(3)))
    assert not srv.submit(big) and big.error == "larger than the device arena"
    srv.drain()
    assert len(srv.done) == 4 and len(srv.rejected) == 3


def test_open_loop_trace_summary():
    ex = FakeExecutor(budget=1 << 22)
    srv = Server(ex)
    reqs = _reqs(30, sizes=(5, 6))
    arrivals = np.linspace(0.0, 0.01, 30)
    stats = run_open_loop(srv, arrivals, reqs)
    assert stats["completed"] == 30 and stats["rejected"] == 0
    assert stats["p99_ms"] >= stats["p50_ms"] >= 0.0
    assert all(r.t_done >= r.t_arrival for r in reqs)
