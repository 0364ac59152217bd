"""Pins for the oracle's |W| histogram and its avalanche / bit-independence
routine, each checked against a library route, a closed form or an identity
that does not come from the routine's own code path."""
import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_1912_03732_amd import inputs
from tests.test_oracle import apply_linear, popcount, random_invertible


def library_spectrum(S, n, m):
    """W[b, a] through scipy's Sylvester Hadamard matrix times the +-1 columns."""
    H = scipy.linalg.hadamard(1 << n).astype(np.int64)
    b = np.arange(1 << m)
    pol = 1 - 2 * (popcount(np.asarray(S, dtype=np.int64)[:, None] & b[None, :]) & 1)   # [x, b]
    return (H @ pol).T                                                                   # [b, a]


def gf_inversion_box(n):
    return inputs.gf_inversion(n)


# ------------------------------------------------------------- histogram ---

@pytest.mark.parametrize("n,m", [(3, 3), (5, 4), (6, 6), (8, 8), (9, 3)])
def test_histogram_equals_library_route(n, m):
    S = inputs.random_function(n, m, inputs.rng(1700 + 13 * n + m))
    W = library_spectrum(S, n, m)[1:]
    ref = np.bincount((np.abs(W) // 2).ravel(), minlength=(1 << (n - 1)) + 1)
    assert np.array_equal(oracle.walsh_histogram(S, n, m), ref.astype(np.uint64))


@pytest.mark.parametrize("n,m", [(7, 7), (10, 6), (12, 3)])
def test_histogram_count_and_parseval(n, m):
    """sum_k hist[k] = 2^n (2^m - 1) and sum_k hist[k] (2k)^2 = (2^m - 1) 4^n."""
    S = inputs.random_function(n, m, inputs.rng(1710 + n))
    h = oracle.walsh_histogram(S, n, m, nthreads=4).astype(np.int64)
    k = np.arange(h.size, dtype=np.int64)
    assert h.sum() == (1 << n) * ((1 << m) - 1)
    assert int((h * (2 * k) ** 2).sum()) == ((1 << m) - 1) * (1 << (2 * n))
    # the largest occupied bin is 2^(n-1) - NL
    nl, _ = oracle.walsh_nl(S, n, m)
    assert int(np.nonzero(h)[0].max()) == (1 << (n - 1)) - nl


@pytest.mark.parametrize("n", [4, 7])
def test_histogram_affine_box(n):
    """S(x) = A x + c with A invertible: every component is affine, so each
    column has one |W| = 2^n and 2^n - 1 zeros."""
    g = inputs.rng(1720 + n)
    A = random_invertible(n, g)
    S = apply_linear(A, np.arange(1 << n)) ^ 5
    h = oracle.walsh_histogram(S, n, n).astype(np.int64)
    M1 = (1 << n) - 1
    assert h[1 << (n - 1)] == M1 and h[0] == M1 * M1 and h.sum() == M1 * (M1 + 1)


@pytest.mark.parametrize("n", [4, 6, 8])
def test_histogram_bent(n):
    """A bent Boolean function (m = 1) has |W| = 2^(n/2) at every a."""
    h2 = n // 2
    x = np.arange(1 << n)
    S = popcount((x & ((1 << h2) - 1)) & (x >> h2)) & 1
    h = oracle.walsh_histogram(S, n, 1).astype(np.int64)
    assert h[1 << (h2 - 1)] == 1 << n and h.sum() == 1 << n


@pytest.mark.parametrize("n", [6, 8])
def test_histogram_inversion_columns_alike(n):
    """For x -> x^-1 in GF(2^n) the component of mask b is that of mask 1
    composed with x -> b'x, so every column has the same |W| multiset: each
    count is a multiple of 2^n - 1, and the top bin gives the closed-form NL."""
    S = gf_inversion_box(n)
    h = oracle.walsh_histogram(S, n, n).astype(np.int64)
    assert np.all(h % ((1 << n) - 1) == 0)
    assert int(np.nonzero(h)[0].max()) == 1 << (n // 2)


# ------------------------------------------------------------- avalanche ---

@pytest.mark.parametrize("n,m", [(4, 4), (6, 3), (7, 7)])
def test_unit_autocorrelation_wiener_khinchin(n, m):
    """r_b(e_i) = 2^-n sum_a W(a, b)^2 (-1)^(a_i), with W from the library route."""
    S = inputs.random_function(n, m, inputs.rng(1730 + n + m))
    W = library_spectrum(S, n, m)
    _, r = oracle.avalanche(S, n, m)
    a = np.arange(1 << n)
    for i in range(n):
        sign = 1 - 2 * ((a >> i) & 1)
        ref = (W * W * sign[None, :]).sum(axis=1)
        assert np.all(ref % (1 << n) == 0)
        assert np.array_equal(r[i].astype(np.int64), ref >> n)


def test_unit_autocorrelation_brute_force_tiny():
    """A few entries written out in pure Python for a 4 x 3 box."""
    n, m = 4, 3
    S = [int(v) for v in inputs.random_function(n, m, inputs.rng(1740))]
    _, r = oracle.avalanche(np.array(S), n, m)
    for i in range(n):
        for b in range(1 << m):
            tot = 0
            for x in range(1 << n):
                y = S[x] ^ S[x ^ (1 << i)]
                tot += -1 if bin(b & y).count("1") % 2 else 1
            assert r[i, b] == tot


@pytest.mark.parametrize("n", [5, 8])
def test_unit_autocorrelation_linear_box(n):
    """S(x) = A x: the derivative in direction e_i is the constant A e_i, so
    r_b(e_i) = 2^n (-1)^(b . A e_i); every output bit that depends on input
    bit i flips always (|r| = 2^n)."""
    A = random_invertible(n, inputs.rng(1750 + n))
    S = apply_linear(A, np.arange(1 << n))
    summ, r = oracle.avalanche(S, n, n)
    b = np.arange(1 << n)
    for i in range(n):
        col = int(apply_linear(A, np.array([1 << i]))[0])
        assert np.array_equal(r[i], (1 << n) * (1 - 2 * (popcount(b & col) & 1)))
    assert summ["sac_max"] == 1 << n and summ["bic_nl"] == 0


@pytest.mark.parametrize("n", [6, 9])
def test_unit_autocorrelation_permutation_sums(n):
    """A permutation never has a zero derivative: sum_b r_b(e_i) = 2^m #{x:
    D_i(x) = 0} = 0; and r_0(e_i) = 2^n."""
    S = inputs.permutation(n, inputs.rng(1760 + n))
    _, r = oracle.avalanche(S, n, n)
    assert np.all(r[:, 0] == 1 << n)
    assert np.all(r.astype(np.int64).sum(axis=1) == 0)


@pytest.mark.parametrize("n", [5, 7])
def test_unit_autocorrelation_apn_inversion(n):
    """Inversion in GF(2^n), n odd, is APN: each derivative takes every value
    0 or 2 times, so sum_b r_b(e_i)^2 = 2^m * 4 * 2^(n-1) (Parseval over b)."""
    S = gf_inversion_box(n)
    _, r = oracle.avalanche(S, n, n)
    assert np.all((r.astype(np.int64) ** 2).sum(axis=1) == 1 << (2 * n + 1))


@pytest.mark.parametrize("n", [4, 6])
def test_avalanche_bent_function(n):
    """A bent function has r(d) = 0 for every d != 0: strict avalanche holds exactly."""
    h2 = n // 2
    x = np.arange(1 << n)
    S = popcount((x & ((1 << h2) - 1)) & (x >> h2)) & 1
    summ, r = oracle.avalanche(S, n, 1)
    assert summ == {"sac_max": 0, "bic_sac_max": -1, "bic_nl": -1}
    assert np.all(r[:, 1] == 0)


def test_avalanche_aes_bic_nl():
    """Every nonzero component of the AES box has NL 112 (Table 2's value),
    so the bit-independence nonlinearity over output-bit pairs is 112 too."""
    summ, _ = oracle.avalanche(inputs.aes_sbox(), 8, 8, full=False)
    assert summ["bic_nl"] == 112


@pytest.mark.parametrize("n,m", [(6, 5), (8, 8), (10, 7)])
def test_avalanche_summary_consistent(n, m):
    """The summary equals the maxima of the full r, and bic_nl the minimum of
    the per-mask nl over the weight-2 masks of the pinned fused routine."""
    S = inputs.random_function(n, m, inputs.rng(1770 + n + m))
    summ, r = oracle.avalanche(S, n, m, nthreads=4)
    summ2, _ = oracle.avalanche(S, n, m, full=False, nthreads=4)
    assert summ == summ2
    unit = [1 << j for j in range(m)]
    pairs = [(1 << j) | (1 << k) for j in range(m) for k in range(j + 1, m)]
    assert summ["sac_max"] == int(np.abs(r[:, unit]).max())
    assert summ["bic_sac_max"] == int(np.abs(r[:, pairs]).max())
    _, maxabs = oracle.walsh_nl(S, n, m)
    assert summ["bic_nl"] == min(((1 << n) - int(maxabs[b])) // 2 for b in pairs)


def test_unit_autocorrelation_masks_match_full():
    n, m = 7, 6
    S = inputs.random_function(n, m, inputs.rng(1780))
    _, r = oracle.avalanche(S, n, m)
    masks = [0, 1, 5, 17, 63, 40]
    assert np.array_equal(oracle.unit_autocorrelation_masks(S, n, m, masks), r[:, masks])
