"""Calls on several streams: the short form keeps one scratch reservation
per (device, stream), so overlapping calls on two streams stay exact; the
batched call stages its descriptors per call (no host wait on another
stream's work) and refuses graph capture, where a plan is the capturable
form."""
import os
import time

import numpy as np
import pytest

import oracle
from paper_1912_03732_amd import binding as B
from paper_1912_03732_amd import inputs
from tests.gpu_util import dev_table, first_diff

pytestmark = pytest.mark.gpu

NT = min(16, os.cpu_count() or 1)


def test_short_form_two_streams_overlapping():
    import torch
    boxes = [(16, 16, inputs.workload_16x16()["perm"]), (12, 12, inputs.permutation(12, inputs.rng(10901))),
             (16, 9, inputs.random_function(16, 9, inputs.rng(10902))), (10, 14, inputs.random_function(10, 14, inputs.rng(10903)))]
    refs = [oracle.walsh_nl(S, n, m, nthreads=NT) for n, m, S in boxes]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for s in streams:
        assert B.sbox_scratch_reserve(16, 16, int(s.cuda_stream)) == B.SBOX_OK, B.last_error()
    tabs = [dev_table(S, m) for n, m, S in boxes]
    outs = [(torch.full((1,), -1, dtype=torch.int32, device="cuda"),
             torch.zeros(1 << m, dtype=torch.int32, device="cuda")) for n, m, S in boxes]
    torch.cuda.synchronize()
    for rep in range(3):
        # boxes 0, 2 on stream 0 and 1, 3 on stream 1, interleaved on the host
        for i in (0, 1, 2, 3):
            n, m, _ = boxes[i]
            s = streams[i % 2]
            st = B.sbox_walsh_nl(tabs[i].data_ptr(), n, m, outs[i][1].data_ptr(), outs[i][0].data_ptr(),
                                 int(s.cuda_stream))
            assert st == B.SBOX_OK, B.last_error()
        torch.cuda.synchronize()
        for i, (n, m, _) in enumerate(boxes):
            onl, omx = refs[i]
            mx = outs[i][1].cpu().numpy()
            assert int(outs[i][0].item()) == onl, (rep, i)
            assert np.array_equal(mx, omx), (rep, i, first_diff(mx, omx))
            outs[i][0].fill_(-1)
            outs[i][1].zero_()
        torch.cuda.synchronize()
    for s in streams:
        assert B.sbox_scratch_release(int(s.cuda_stream)) == B.SBOX_OK


def _batch(tabs, ns, ms):
    import torch
    count = len(tabs)
    nl = torch.full((count,), -1, dtype=torch.int32, device="cuda")
    mxs = [torch.zeros(1 << m, dtype=torch.int32, device="cuda") for m in ms]
    jobs = B.make_jobs(tabs, ns, ms, [nl[i:i + 1] for i in range(count)], mxs)
    ws = B.Workspace(B.sbox_batched_workspace_bytes(jobs, count))
    return jobs, nl, mxs, ws


def test_batched_calls_on_two_streams_do_not_wait_on_the_host():
    """A batched call on stream 1 returns while stream 0 still runs long
    batched work queued before it (its descriptors are staged in a block of
    its own), and every result is exact."""
    import torch
    long_S = [inputs.permutation(16, inputs.rng(10910 + k)) for k in range(2)]
    long_tabs = [dev_table(S, 16) for S in long_S]
    small = [(12, inputs.permutation(12, inputs.rng(10920 + k))) for k in range(8)]
    small_tabs = [dev_table(S, 12) for _, S in small]
    s0, s1 = torch.cuda.Stream(), torch.cuda.Stream()
    A = _batch(long_tabs * 8, [16] * 16, [16] * 16)   # about 16 x 0.6 ms of work
    A2 = _batch(long_tabs, [16] * 2, [16] * 2)
    C = _batch(small_tabs, [12] * 8, [12] * 8)
    # once untimed, so that the staging pool holds a block for each call
    for jobs, cnt, ws, s in ((A[0], 16, A[3], s0), (A2[0], 2, A2[3], s0), (C[0], 8, C[3], s1)):
        assert B.sbox_walsh_nl_batched(jobs, cnt, ws.ptr, ws.nbytes, int(s.cuda_stream)) == B.SBOX_OK
    torch.cuda.synchronize()
    assert B.sbox_walsh_nl_batched(A[0], 16, A[3].ptr, A[3].nbytes, int(s0.cuda_stream)) == B.SBOX_OK
    assert B.sbox_walsh_nl_batched(A2[0], 2, A2[3].ptr, A2[3].nbytes, int(s0.cuda_stream)) == B.SBOX_OK
    t0 = time.perf_counter()
    st = B.sbox_walsh_nl_batched(C[0], 8, C[3].ptr, C[3].nbytes, int(s1.cuda_stream))
    dt_submit = time.perf_counter() - t0
    assert st == B.SBOX_OK, B.last_error()
    t1 = time.perf_counter()
    s0.synchronize()
    dt_rest = time.perf_counter() - t1
    torch.cuda.synchronize()
    # the submission on stream 1 did not wait for stream 0's queued work
    assert dt_submit < 0.5 * (dt_submit + dt_rest), (dt_submit, dt_rest)
    for k, S in enumerate(long_S):
        onl, omx = oracle.walsh_nl(S, 16, 16, nthreads=NT)
        for i in range(k, 16, 2):
            assert int(A[1][i].item()) == onl and np.array_equal(A[2][i].cpu().numpy(), omx), i
        assert int(A2[1][k].item()) == onl and np.array_equal(A2[2][k].cpu().numpy(), omx)
    for i, (n, S) in enumerate(small):
        onl, omx = oracle.walsh_nl(S, n, n, nthreads=NT)
        assert int(C[1][i].item()) == onl and np.array_equal(C[2][i].cpu().numpy(), omx), i


def test_batched_call_refuses_capture_plan_captures():
    import torch
    batch = inputs.workload_batched(count=16, seed=10930)
    tabs = [dev_table(S, n) for n, S in batch]
    ns = [n for n, _ in batch]
    jobs, nl, mxs, ws = _batch(tabs, ns, ns)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        st = B.sbox_walsh_nl_batched(jobs, len(tabs), ws.ptr, ws.nbytes, int(s.cuda_stream))
        nl.fill_(3)
    assert st == B.SBOX_ERR_INVALID_ARG and "captured" in B.last_error()
    g.replay()  # the capture stayed valid: it holds only the fill
    torch.cuda.synchronize()
    assert bool((nl == 3).all())
    assert B.sbox_walsh_nl_batched(jobs, len(tabs), ws.ptr, ws.nbytes, int(s.cuda_stream)) == B.SBOX_OK
    s.synchronize()
    for i, (n, S) in enumerate(batch):
        assert int(nl[i].item()) == oracle.walsh_nl(S, n, n)[0]
