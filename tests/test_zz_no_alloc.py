"""The entry point for callers that cannot allocate (sbox_walsh_nl_static):
through the C ABI, against sbox_walsh_nl_ex with a caller workspace and
against the oracle, on two calls in a row, the second on a smaller box;
sizes beyond the static array are refused before anything is enqueued."""
import numpy as np
import pytest

import oracle
from paper_1912_03732_amd import binding as B
from paper_1912_03732_amd import inputs
from tests.gpu_util import dev_table, first_diff

pytestmark = pytest.mark.gpu


def _outputs(torch, n, m, layout):
    nl = torch.full((1,), -9, dtype=torch.int32, device="cuda")
    mx = torch.full((1 << m,), -9, dtype=torch.int32, device="cuda")
    spec = torch.full((1 << (n + m),), -9, dtype=torch.int32, device="cuda") if layout else None
    return nl, mx, spec


def _run_both(n, m, S, layout=0, full_oracle=True):
    import torch
    t = dev_table(S, m)
    sp = int(torch.cuda.current_stream().cuda_stream)
    nl_s, mx_s, sp_s = _outputs(torch, n, m, layout)
    st = B.sbox_walsh_nl_static(t.data_ptr(), n, m, t.element_size(), mx_s.data_ptr(), nl_s.data_ptr(),
                                sp_s.data_ptr() if sp_s is not None else 0, layout, sp)
    assert st == B.SBOX_OK, B.last_error()
    nl_e, mx_e, sp_e = _outputs(torch, n, m, layout)
    ws = B.Workspace(B.sbox_walsh_nl_workspace_bytes(n, m, layout))
    st = B.sbox_walsh_nl_ex(t.data_ptr(), n, m, t.element_size(), mx_e.data_ptr(), nl_e.data_ptr(),
                            sp_e.data_ptr() if sp_e is not None else 0, layout, ws.ptr, ws.nbytes, None, sp)
    assert st == B.SBOX_OK, B.last_error()
    torch.cuda.synchronize()
    a, b = mx_s.cpu().numpy(), mx_e.cpu().numpy()
    assert np.array_equal(a, b), (n, m, first_diff(a, b))
    assert int(nl_s.item()) == int(nl_e.item())
    if layout:
        assert np.array_equal(sp_s.cpu().numpy(), sp_e.cpu().numpy()), (n, m, layout)
    if full_oracle:
        onl, omx = oracle.walsh_nl(S, n, m, nthreads=8)
        assert int(nl_s.item()) == onl and np.array_equal(a, omx), (n, m)
    else:  # 2^m masks too many for the oracle here: a sample, and NL from the maxima
        g = inputs.rng(11010)
        masks = np.unique(np.concatenate([[1, (1 << m) - 1], g.integers(1, 1 << m, size=64)]))
        assert np.array_equal(a[masks], oracle.maxabs_for_masks(S, n, m, masks, nthreads=8))
        assert int(nl_s.item()) == (1 << (n - 1)) - int(a[1:].max()) // 2
    return int(nl_s.item())


def test_static_scratch_matches_workspace_form_two_calls():
    # the largest box the array serves first, then a smaller one that reuses it
    assert _run_both(16, 16, inputs.workload_16x16()["perm"]) == 31960
    _run_both(12, 10, inputs.random_function(12, 10, inputs.rng(11001)))
    # and a spectrum, then the fused form again
    _run_both(8, 8, inputs.workload_8x8()["perm"], layout=B.SPECTRUM_B_MAJOR)
    # the most scratch the array serves (m = 24 bit-sliced slices at n = 16)
    assert _run_both(16, 24, inputs.random_function(16, 24, inputs.rng(11002)), full_oracle=False) > 0


def test_static_scratch_refuses_sizes_beyond_the_array():
    import torch
    assert B.sbox_walsh_nl_static_max_bytes() == 256 << 10
    nl = torch.full((1,), -9, dtype=torch.int32, device="cuda")
    t = dev_table(inputs.random_function(17, 4, inputs.rng(11003)), 4)
    sp = int(torch.cuda.current_stream().cuda_stream)
    assert B.sbox_walsh_nl_static(t.data_ptr(), 17, 4, 1, 0, nl.data_ptr(), 0, 0, sp) == B.SBOX_ERR_WORKSPACE
    assert "static array" in B.last_error()
    spec_ptr = 1 << 20  # never dereferenced: refused before anything is enqueued
    assert B.sbox_walsh_nl_static(t.data_ptr(), 16, 16, 2, 0, nl.data_ptr(), spec_ptr, B.SPECTRUM_A_MAJOR,
                                  sp) == B.SBOX_ERR_WORKSPACE
    assert B.sbox_walsh_nl_static(t.data_ptr(), 0, 4, 1, 0, nl.data_ptr(), 0, 0, sp) == B.SBOX_ERR_UNSUPPORTED
    assert B.sbox_walsh_nl_static(t.data_ptr(), 8, 8, 1, 0, nl.data_ptr(), 0, 5, sp) == B.SBOX_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert int(nl.item()) == -9
