"""GPU parity of the component criteria kernel against the oracle."""
import numpy as np
import pytest

import oracle
from paper_1912_03732_amd import binding as B
from paper_1912_03732_amd import inputs
from tests.gpu_util import dev_table, table

pytestmark = pytest.mark.gpu


def _check(S, n, m):
    summ, per = B.criteria(dev_table(S, m), n, m)
    osumm, oper = oracle.criteria(S, n, m, nthreads=16)
    assert summ == osumm
    for k in ("w0", "minwt", "acmax", "pcwt"):
        assert np.array_equal(per[k].cpu().numpy(), oper[k]), k


@pytest.mark.parametrize("n,m", [(1, 1), (2, 3), (3, 3), (4, 4), (5, 2), (6, 6), (7, 5), (8, 8), (9, 4),
                                 (10, 3), (11, 2), (12, 2), (13, 1), (14, 1)])
def test_criteria_random(n, m):
    _check(table(n, m, 12000 + n * m), n, m)


def test_criteria_structured_boxes():
    _check(inputs.aes_sbox(), 8, 8)
    _check(inputs.gf_inversion(6), 6, 6)
    x = np.arange(1 << 10)
    _check(np.bitwise_count(x.astype(np.uint64)).astype(np.uint32) & 1, 10, 1)  # parity: resilient
    _check(np.bitwise_count(((x & 31) & (x >> 5)).astype(np.uint64)).astype(np.uint32) & 1, 10, 1)  # bent
    _check(np.arange(1 << 9), 9, 9)  # identity


def test_criteria_inversion_and_nl_agree_with_fused_path():
    S = inputs.gf_inversion(12)
    summ, per = B.criteria(dev_table(S, 12), 12, 12, per_mask=False)
    assert per is None
    assert summ["nl"] == 1984 and summ["unbalanced"] == 0 and summ["abs_indicator"] == 128
    assert summ["nl"] == B.walsh_nl(dev_table(S, 12), 12, 12)[0]


@pytest.mark.parametrize("n,m", [(15, 3), (16, 2), (16, 3)])
def test_criteria_large_random(n, m):
    """n = 15, 16 go through the slab path (spectrum rows, squares, second
    transform, row reductions): bit-exact against the oracle."""
    _check(table(n, m, 12500 + n * m), n, m)


def test_criteria_large_structured():
    x = np.arange(1 << 16)
    _check(np.bitwise_count(x.astype(np.uint64)).astype(np.uint32) & 1, 16, 1)  # parity: 15-resilient
    _check(np.bitwise_count(((x & 255) & (x >> 8)).astype(np.uint64)).astype(np.uint32) & 1, 16, 1)  # bent


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
