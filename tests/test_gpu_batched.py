"""Batched launches: every box of a mixed batch equals the same box alone
(bit-exact), plans replay identically, also inside a captured HIP graph."""
import numpy as np
import pytest

import oracle
from paper_1912_03732_amd import binding as B
from paper_1912_03732_amd import inputs
from tests.gpu_util import dev_table, table

pytestmark = pytest.mark.gpu


def _mixed(count, seed, sizes):
    g = inputs.rng(seed)
    boxes = []
    for i in range(count):
        n = int(g.choice(sizes))
        m = int(g.integers(1, 13))
        boxes.append((n, m, inputs.random_function(n, m, g)))
    return boxes


def test_batched_mixed_sizes_equal_oracle():
    boxes = _mixed(60, 10001, list(range(1, 17)))
    tabs = [dev_table(S, m) for n, m, S in boxes]
    nl, mxs = B.walsh_nl_batched(tabs, [b[0] for b in boxes], [b[1] for b in boxes])
    nl = nl.cpu().numpy()
    for i, (n, m, S) in enumerate(boxes):
        onl, omx = oracle.walsh_nl(S, n, m, nthreads=8)
        assert nl[i] == onl, (i, n, m)
        assert np.array_equal(mxs[i].cpu().numpy(), omx), (i, n, m)


def test_batched_workload_mix_equals_single_calls():
    batch = inputs.workload_batched(count=200)
    tabs = [dev_table(S, n) for n, S in batch]
    ns = [n for n, _ in batch]
    nl, mxs = B.walsh_nl_batched(tabs, ns, ns)
    nl = nl.cpu().numpy()
    for i, (n, S) in enumerate(batch):
        snl, smx, _ = B.walsh_nl(tabs[i], n, n)
        assert nl[i] == snl
        assert np.array_equal(mxs[i].cpu().numpy(), smx.cpu().numpy())
    # and a sample against the oracle
    for i in range(0, 200, 23):
        n, S = batch[i]
        assert nl[i] == oracle.walsh_nl(S, n, n)[0]


def test_plan_replay_and_graph_capture():
    import torch
    batch = inputs.workload_batched(count=64, seed=123)
    tabs = [dev_table(S, n) for n, S in batch]
    ns = [n for n, _ in batch]
    plan = B.Plan(tabs, ns, ns)
    plan.launch()
    torch.cuda.synchronize()
    ref_nl = plan.nl.cpu().numpy().copy()
    ref_mx = [m.cpu().numpy().copy() for m in plan.maxabs]
    for i, (n, S) in enumerate(batch[:8]):
        assert ref_nl[i] == oracle.walsh_nl(S, n, n)[0]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        plan.launch(stream=s)  # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        plan.launch()
    for rep in range(4):
        plan.nl.fill_(-1)
        for m in plan.maxabs:
            m.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(plan.nl.cpu().numpy(), ref_nl), rep
        for a, b in zip(plan.maxabs, ref_mx):
            assert np.array_equal(a.cpu().numpy(), b), rep
    # the graph reads the tables at replay time
    new = inputs.permutation(ns[0], inputs.rng(999))
    tabs[0].copy_(dev_table(new, ns[0]))
    g.replay()
    torch.cuda.synchronize()
    assert int(plan.nl[0].item()) == oracle.walsh_nl(new, ns[0], ns[0])[0]
    plan.close()


def test_batched_with_spectra_and_edge_boxes():
    import torch
    specs = []
    boxes = [(1, 1), (2, 3), (4, 4), (5, 2), (6, 6), (9, 3), (12, 2)]
    tabs, outs_nl, outs_mx, layouts, Ss = [], [], [], [], []
    for i, (n, m) in enumerate(boxes):
        S = table(n, m, 11000 + i)
        Ss.append(S)
        tabs.append(dev_table(S, m))
        outs_nl.append(torch.empty(1, dtype=torch.int32, device="cuda"))
        outs_mx.append(torch.empty(1 << m, dtype=torch.int32, device="cuda"))
        lay = [1, 2, 0x11, 0x12][i % 4]
        layouts.append(lay)
        specs.append(torch.empty(1 << (n + m), dtype=torch.int32, device="cuda"))
    jobs = B.make_jobs(tabs, [b[0] for b in boxes], [b[1] for b in boxes], outs_nl, outs_mx, layouts, specs)
    need = B.sbox_batched_workspace_bytes(jobs, len(boxes))
    ws = B.Workspace(need)
    st = B.sbox_walsh_nl_batched(jobs, len(boxes), ws.ptr, ws.nbytes, int(torch.cuda.current_stream().cuda_stream))
    assert st == 0, B.last_error()
    torch.cuda.synchronize()
    for i, (n, m) in enumerate(boxes):
        lay = oracle.B_MAJOR if (layouts[i] & 3) == 1 else oracle.A_MAJOR
        ref = oracle.spectrum(Ss[i], n, m, lay).reshape(-1)
        if layouts[i] & 0x10:
            ref = ref // 2
        assert np.array_equal(specs[i].cpu().numpy(), ref), (n, m, layouts[i])
        assert int(outs_nl[i].item()) == oracle.walsh_nl(Ss[i], n, m)[0]


def test_empty_batch():
    assert B.sbox_walsh_nl_batched(None, 0, 0, 0, 0) == B.SBOX_OK


@pytest.mark.parametrize("variant", [1, 2])
def test_batched_n16_boxes_both_engines(variant):
    """n = 16 boxes in a mixed batch (matrix-core and VALU engines) equal the oracle."""
    import torch
    g = inputs.rng(10051)
    boxes = [(16, 16, inputs.permutation(16, g)), (16, 3, inputs.random_function(16, 3, g)),
             (12, 9, inputs.random_function(12, 9, g)), (16, 7, inputs.random_function(16, 7, g)),
             (5, 5, inputs.permutation(5, g))]
    tabs = [dev_table(S, m) for n, m, S in boxes]
    plan = B.Plan(tabs, [b[0] for b in boxes], [b[1] for b in boxes], tuning=B.sbox_tuning(0, 0, 0, variant))
    for _ in range(2):
        plan.launch()
        torch.cuda.synchronize()
        nl = plan.nl.cpu().numpy()
        for i, (n, m, S) in enumerate(boxes):
            onl, omx = oracle.walsh_nl(S, n, m, nthreads=8)
            assert nl[i] == onl, (variant, i, n, m)
            assert np.array_equal(plan.maxabs[i].cpu().numpy(), omx), (variant, i, n, m)
    plan.close()
