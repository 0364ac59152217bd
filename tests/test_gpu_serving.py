"""Serving on the GPU: requests that overlap on the device give exactly the
results they give alone."""
import numpy as np
import pytest

import oracle
from paper_1912_03732_amd import binding as B
from paper_1912_03732_amd import inputs
from paper_1912_03732_amd.serving import GpuExecutor, Request, Server, run_open_loop

pytestmark = pytest.mark.gpu


def test_each_result_same_alone_and_in_the_mix():
    t, ns, pick, pools = inputs.workload_serving(4000.0, count=300, pool=8)
    reqs = [Request(i, int(n), int(n), pools[int(n)][int(p)]) for i, (n, p) in enumerate(zip(ns, pick))]
    ex = GpuExecutor(arena_bytes=64 << 20, streams=2)
    srv = Server(ex, max_batch=64)
    stats = run_open_loop(srv, t, reqs)
    assert stats["completed"] == 300 and stats["rejected"] == 0
    alone = {}
    for r in reqs:
        key = (r.n, int(pick[r.rid]))
        if key not in alone:
            nl, mx, _ = B.walsh_nl(B.table_to_device(r.table, r.m), r.n, r.m)
            alone[key] = (nl, mx.cpu().numpy())
        nl, mx = alone[key]
        assert r.nl == nl and np.array_equal(r.maxabs, mx), r.rid
    # and the oracle on one box of each size
    for n in (8, 12, 16):
        r = next(q for q in reqs if q.n == n)
        assert r.nl == oracle.walsh_nl(r.table, n, n, nthreads=16)[0]


def test_small_arena_forces_many_batches():
    g = inputs.rng(77)
    reqs = [Request(i, 12, 12, inputs.permutation(12, g)) for i in range(40)]
    ex = GpuExecutor(arena_bytes=1 << 18, streams=3)
    srv = Server(ex)
    for r in reqs:
        srv.submit(r)
    srv.drain()
    assert len(srv.done) == 40 and srv.batches >= 4
    for r in reqs[:5]:
        assert r.nl == oracle.walsh_nl(r.table, 12, 12)[0]
