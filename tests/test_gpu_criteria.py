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
