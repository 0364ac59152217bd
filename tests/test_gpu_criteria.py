"""GPU parity of the component criteria kernel against the oracle."""
import numpy as np
import pytest

import oracle
from paper_1912_03732_amd import binding as B
from paper_1912_03732_amd import inputs
from tests.gpu_util import dev_table, table

pytestmark = pytest.mark.gpu


def _check(S, n, m, ws=True):
    """ws selects the register-blocked kernel (5 <= n <= 14) over the LDS one."""
    summ, per = B.criteria(dev_table(S, m), n, m, workspace=ws)
    osumm, oper = oracle.criteria(S, n, m, nthreads=16)
    assert summ == osumm
    for k in ("w0", "minwt", "acmax", "pcwt"):
        got = per[k].cpu().numpy()
        bad = np.nonzero(got != oper[k])[0]
        assert bad.size == 0, (k, bad[:6], got[bad[:6]], oper[k][bad[:6]])


@pytest.mark.parametrize("ws", [True, False])
@pytest.mark.parametrize("n,m", [(1, 1), (2, 3), (3, 3), (4, 4), (5, 2), (6, 6), (7, 5), (8, 8), (9, 4),
                                 (10, 3), (11, 2), (12, 2), (13, 1), (14, 1)])
def test_criteria_random(n, m, ws):
    _check(table(n, m, 12000 + n * m), n, m, ws)


@pytest.mark.parametrize("n,m", [(5, 20), (6, 18), (7, 17), (8, 16), (9, 11), (10, 10), (11, 9), (12, 7),
                                 (13, 5), (14, 3)])
def test_criteria_register_kernel_many_masks(n, m):
    """Up to n = 8 these shapes give every group of the register-blocked
    kernel several masks to walk in Gray order, the last groups stopping
    part-way; the larger n cover each shape of its lane groups (the 12 x 12
    and 14 x 14 workloads below walk several masks per group at those n)."""
    _check(table(n, m, 12300 + n * m), n, m)


def test_criteria_workload_12x12_full():
    """The 12 x 12 permutation that bench.py times, every mask."""
    _check(inputs.permutation(12, inputs.rng(inputs.SEED_BASE + 6)), 12, 12)


@pytest.mark.parametrize("ws", [True, False])
def test_criteria_workload_14x14_sampled(ws):
    """The 14 x 14 permutation that bench.py times: the oracle sums the
    autocorrelation from its definition (4^14 terms a mask), so the per-mask
    values are checked on sampled masks (transform column and definition),
    NL against the fused path, and the summary against the per-mask arrays."""
    n = 14
    S = inputs.permutation(n, inputs.rng(inputs.SEED_BASE + 6))
    Sd = dev_table(S, n)
    summ, per = B.criteria(Sd, n, n, workspace=ws)
    per = {k: v.cpu().numpy() for k, v in per.items()}
    assert summ["nl"] == B.walsh_nl(Sd, n, n)[0]
    assert summ["unbalanced"] == 0 and np.all(per["w0"][1:] == 0)
    assert summ["abs_indicator"] == int(per["acmax"][1:].max())
    assert summ["ci_order"] == int(per["minwt"][1:].min()) - 1
    assert summ["pc_order"] == int(per["pcwt"][1:].min()) - 1
    wts = np.bitwise_count(np.arange(1 << n).astype(np.uint64))
    for b in [1, 0x2000, 0x3FFF, int(inputs.rng(12700).integers(1, 1 << n))]:
        col = oracle.walsh_column(S, n, n, b)
        assert per["w0"][b] == col[0]
        assert per["minwt"][b] == int(wts[1:][col[1:] != 0].min())
        r = oracle.autocorrelation(S, n, n, b)
        assert per["acmax"][b] == int(np.abs(r[1:]).max())
        assert per["pcwt"][b] == int(wts[1:][r[1:] != 0].min())


@pytest.mark.parametrize("ws", [True, False])
def test_criteria_structured_boxes(ws):
    _check(inputs.aes_sbox(), 8, 8, ws)
    _check(inputs.gf_inversion(6), 6, 6, ws)
    x = np.arange(1 << 10)
    _check(np.bitwise_count(x.astype(np.uint64)).astype(np.uint32) & 1, 10, 1, ws)  # parity: resilient
    _check(np.bitwise_count(((x & 31) & (x >> 5)).astype(np.uint64)).astype(np.uint32) & 1, 10, 1, ws)  # bent
    _check(np.arange(1 << 9), 9, 9, ws)  # identity
    x = np.arange(1 << 14)
    _check(np.bitwise_count(x.astype(np.uint64)).astype(np.uint32) & 1, 14, 1, ws)  # parity
    _check(np.bitwise_count(((x & 127) & (x >> 7)).astype(np.uint64)).astype(np.uint32) & 1, 14, 1, ws)  # bent
    _check(inputs.gf_inversion(13) & 0x7F, 13, 7, ws)
    A = np.arange(1 << 11)
    _check((A ^ (A >> 3)) & 0xFF, 11, 8, ws)  # linear: one nonzero W per mask


def test_criteria_inversion_and_nl_agree_with_fused_path():
    S = inputs.gf_inversion(12)
    summ, per = B.criteria(dev_table(S, 12), 12, 12, per_mask=False)
    assert per is None
    assert summ["nl"] == 1984 and summ["unbalanced"] == 0 and summ["abs_indicator"] == 128
    assert summ["nl"] == B.walsh_nl(dev_table(S, 12), 12, 12)[0]


@pytest.mark.parametrize("n,m", [(15, 3), (15, 4), (16, 2), (16, 3)])
def test_criteria_large_random(n, m):
    """n = 15 and 16 run the register-blocked kernel with one 512- or
    1,024-lane workgroup per mask (both transforms on one compute unit):
    bit-exact against the oracle."""
    _check(table(n, m, 12500 + n * m), n, m)


@pytest.mark.parametrize("n", [15, 16])
def test_criteria_large_structured(n):
    x = np.arange(1 << n)
    _check(np.bitwise_count(x.astype(np.uint64)).astype(np.uint32) & 1, n, 1)  # parity: (n-1)-resilient
    h = n // 2
    _check(np.bitwise_count(((x & ((1 << h) - 1)) & (x >> h)).astype(np.uint64)).astype(np.uint32) & 1, n, 1)
    A = x ^ (x >> 5) ^ ((x & 7) << 9)  # linear, invertible: one nonzero W per mask
    _check(A & 7, n, 3)


def test_criteria_15x15_sampled():
    """A 15 x 15 permutation, every mask through the kernel; per-mask values
    on sampled masks against the oracle's transform column and definition,
    the summary against the per-mask arrays and NL against the fused path."""
    n = 15
    S = inputs.permutation(n, inputs.rng(12800))
    Sd = dev_table(S, n)
    summ, per = B.criteria(Sd, n, n)
    per = {k: v.cpu().numpy() for k, v in per.items()}
    assert summ["nl"] == B.walsh_nl(Sd, n, n)[0]
    assert summ["unbalanced"] == 0 and np.all(per["w0"][1:] == 0)
    assert summ["abs_indicator"] == int(per["acmax"][1:].max())
    assert summ["ci_order"] == int(per["minwt"][1:].min()) - 1
    assert summ["pc_order"] == int(per["pcwt"][1:].min()) - 1
    wts = np.bitwise_count(np.arange(1 << n).astype(np.uint64))
    for b in [1, 0x7FFF]:
        col = oracle.walsh_column(S, n, n, b)
        assert per["minwt"][b] == int(wts[1:][col[1:] != 0].min())
        r = oracle.autocorrelation(S, n, n, b)
        assert per["acmax"][b] == int(np.abs(r[1:]).max())
        assert per["pcwt"][b] == int(wts[1:][r[1:] != 0].min())


def test_criteria_16x16_permutation():
    """The 16 x 16 workload box: NL equals the fused path's, a permutation is
    balanced in every component, and one sampled mask's autocorrelation
    maximum and propagation weight equal the oracle's (summed from the
    definition)."""
    S = inputs.workload_16x16()["perm"]
    Sd = dev_table(S, 16)
    summ, per = B.criteria(Sd, 16, 16)
    nl, _, _ = B.walsh_nl(Sd, 16, 16)
    assert summ["nl"] == nl and summ["unbalanced"] == 0 and summ["resiliency"] == summ["ci_order"]
    assert np.all(per["w0"].cpu().numpy()[1:] == 0)
    b = 0x1234
    r = oracle.autocorrelation(S, 16, 16, b)
    wts = np.bitwise_count(np.arange(1 << 16).astype(np.uint64))
    assert per["acmax"].cpu().numpy()[b] == int(np.abs(r[1:]).max())
    assert per["pcwt"].cpu().numpy()[b] == int(wts[1:][r[1:] != 0].min())
    acm = per["acmax"].cpu().numpy()
    assert summ["abs_indicator"] == int(acm[1:].max())


def _fwht(v):
    """Natural-order Walsh-Hadamard transform (int64), for the autocorrelation
    r = 2^-n H(W^2) of a transform column (Wiener-Khinchin)."""
    v = np.array(v, dtype=np.int64)
    h = 1
    while h < v.size:
        v = v.reshape(-1, 2, h)
        v = np.stack([v[:, 0] + v[:, 1], v[:, 0] - v[:, 1]], axis=1).reshape(-1)
        h *= 2
    return v


def test_criteria_largest_box_sampled():
    """n = 16, m = 24 (n + m = 40, 2^24 - 1 masks, 4,096 workgroups walking
    long Gray runs): sampled masks against the oracle's transform column (w0,
    CI weight) and its Wiener-Khinchin autocorrelation (absolute indicator,
    PC weight); the summary against the per-mask arrays."""
    n, m = 16, 24
    S = table(n, m, 12900)
    summ, per = B.criteria(dev_table(S, m), n, m)
    per = {k: v.cpu().numpy() for k, v in per.items()}
    assert summ["unbalanced"] == int(np.count_nonzero(per["w0"][1:]))
    assert summ["abs_indicator"] == int(per["acmax"][1:].max())
    assert summ["ci_order"] == int(per["minwt"][1:].min()) - 1
    assert summ["pc_order"] == int(per["pcwt"][1:].min()) - 1
    wts = np.bitwise_count(np.arange(1 << n).astype(np.uint64))
    g = inputs.rng(12901)
    for b in [1, (1 << m) - 1, 1 << 23, 0x5A5A5A] + [int(v) for v in g.integers(1, 1 << m, size=4)]:
        col = oracle.walsh_column(S, n, m, b).astype(np.int64)
        assert per["w0"][b] == col[0], b
        nz = wts[1:][col[1:] != 0]
        assert per["minwt"][b] == (int(nz.min()) if nz.size else n + 1), b
        r = _fwht(col * col) >> n  # H(W^2) = 2^n r
        assert r[0] == 1 << n
        assert per["acmax"][b] == int(np.abs(r[1:]).max()), b
        nzr = wts[1:][r[1:] != 0]
        assert per["pcwt"][b] == (int(nzr.min()) if nzr.size else n + 1), b


def test_criteria_ex_small_n_needs_no_workspace():
    import torch
    n, m = 10, 6
    S = table(n, m, 12600)
    Sd = dev_table(S, m)
    summ = torch.empty(8, dtype=torch.int32, device="cuda")
    st = int(torch.cuda.current_stream().cuda_stream)
    assert B.sbox_criteria_ex(Sd.data_ptr(), n, m, Sd.element_size(), summ.data_ptr(), 0, 0, 0, 0, 0, 0,
                              st) == B.SBOX_OK
    torch.cuda.synchronize()
    osumm, _ = oracle.criteria(S, n, m, nthreads=16)
    assert summ.cpu().tolist()[:6] == [osumm[k] for k in oracle.CRITERIA_FIELDS]
