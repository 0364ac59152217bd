"""Pins for the oracle's component criteria (balancedness, correlation
immunity, autocorrelation), each checked against an identity or a closed
form that does not come from the oracle's own code path."""
import numpy as np
import pytest

import oracle
from paper_1912_03732_amd import inputs
from tests.test_oracle import popcount


@pytest.mark.parametrize("n,m", [(4, 4), (6, 3), (7, 7)])
def test_wiener_khinchin(n, m):
    """sum_d r_b(d) (-1)^(a.d) = W(a, b)^2: autocorrelation (summed from its
    definition) against the spectrum (FWHT), two independent routes."""
    S = inputs.random_function(n, m, inputs.rng(900 + n + m))
    d = np.arange(1 << n)
    chi = 1 - 2 * (popcount(d[:, None] & d[None, :]) & 1)
    for b in range(1, 1 << m):
        r = oracle.autocorrelation(S, n, m, b).astype(np.int64)
        W = oracle.walsh_column(S, n, m, b).astype(np.int64)
        assert np.array_equal(chi @ r, W * W)
        assert r[0] == 1 << n


def _bent_and_quadratic(n):
    """n even, m = 3: component 1 the bent x_lo . x_hi (r(d) = 0 for d != 0),
    component 2 the quadratic x0 x1 (every d with d0 = d1 = 0 is a linear
    structure), component 3 the balanced x0 ^ x2 x3: per-mask propagation
    weights 1, n + 1 and mixtures of them."""
    h = n // 2
    x = np.arange(1 << n)
    f1 = popcount((x & ((1 << h) - 1)) & (x >> h)) & 1
    f2 = (x & 1) & ((x >> 1) & 1)
    f3 = (x & 1) ^ (((x >> 2) & 1) & ((x >> 3) & 1))
    return f1 | (f2 << 1) | (f3 << 2)


@pytest.mark.parametrize("n,m,kind", [(7, 5, "random"), (6, 3, "structured"), (8, 3, "structured")])
def test_criteria_match_spectrum_and_definitions(n, m, kind):
    """Every per-mask output against the stored spectrum (w0, minwt) and the
    autocorrelation summed from its definition (acmax, pcwt)."""
    S = inputs.random_function(n, m, inputs.rng(901)) if kind == "random" else _bent_and_quadratic(n)
    summ, per = oracle.criteria(S, n, m)
    Wt = oracle.spectrum(S, n, m, oracle.B_MAJOR)
    wts = popcount(np.arange(1 << n))
    pcw = set()
    for b in range(1, 1 << m):
        assert per["w0"][b] == Wt[b, 0]
        nz = [int(wts[a]) for a in range(1, 1 << n) if Wt[b, a] != 0]
        assert per["minwt"][b] == (min(nz) if nz else n + 1)
        r = oracle.autocorrelation(S, n, m, b)
        assert per["acmax"][b] == int(np.abs(r[1:]).max())
        nzd = [int(wts[d]) for d in range(1, 1 << n) if r[d] != 0]
        assert per["pcwt"][b] == (min(nzd) if nzd else n + 1)
        pcw.add(int(per["pcwt"][b]))
    assert summ["nl"] == oracle.walsh_nl(S, n, m)[0]
    assert summ["unbalanced"] == int(np.count_nonzero(Wt[1:, 0]))
    assert summ["pc_order"] == min(pcw) - 1
    if kind == "structured":
        assert per["pcwt"][1] == n + 1 and per["pcwt"][2] == 1 and len(pcw) >= 2


@pytest.mark.parametrize("n", [4, 6, 8])
def test_bent_function(n):
    """m = 1, f = <x_lo, x_hi>: a bent function has r(d) = 0 for all d != 0,
    so its absolute indicator is 0 and its propagation order is n; |W| = 2^(n/2)
    everywhere, so it is unbalanced and 0-th order correlation immune."""
    h = n // 2
    x = np.arange(1 << n)
    S = popcount((x & ((1 << h) - 1)) & (x >> h)) & 1
    summ, per = oracle.criteria(S, n, 1)
    assert summ == {"nl": (1 << (n - 1)) - (1 << (h - 1)), "unbalanced": 1, "ci_order": 0, "resiliency": -1,
                    "abs_indicator": 0, "pc_order": n}


@pytest.mark.parametrize("n", [3, 5, 8])
def test_parity_function_is_maximally_resilient(n):
    """m = 1, f(x) = parity(x): W(a) != 0 only at a = all ones, so it is
    balanced and (n-1)-resilient; every d is a linear structure (|r(d)| = 2^n)."""
    S = popcount(np.arange(1 << n)) & 1
    summ, per = oracle.criteria(S, n, 1)
    assert summ["unbalanced"] == 0 and summ["ci_order"] == n - 1 and summ["resiliency"] == n - 1
    assert summ["abs_indicator"] == 1 << n and summ["pc_order"] == 0 and summ["nl"] == 0


def test_identity_permutation():
    """S(x) = x: component b is the linear function b.x, W(a, b) = 2^n [a = b],
    so the smallest nonzero weight is wt(b) and r_b(d) = 2^n (-1)^(b.d)."""
    n = 6
    S = np.arange(1 << n)
    summ, per = oracle.criteria(S, n, n)
    b = np.arange(1, 1 << n)
    assert np.array_equal(per["minwt"][1:], popcount(b))
    assert np.all(per["acmax"][1:] == 1 << n) and np.all(per["w0"][1:] == 0)
    assert summ["ci_order"] == 0 and summ["resiliency"] == 0 and summ["pc_order"] == 0


@pytest.mark.parametrize("n", [4, 6, 8])
def test_inversion_absolute_indicator_closed_form(n):
    """GF(2^n) inversion, n even: balanced, absolute indicator 2^(n/2+1)
    (the known value for the inverse function; 32 for the AES-size box)."""
    summ, _ = oracle.criteria(inputs.gf_inversion(n), n, n, nthreads=8)
    assert summ["unbalanced"] == 0 and summ["abs_indicator"] == 1 << (n // 2 + 1)
