"""Seeded synthetic inputs: S-box tables, batches and request traces.

This module only *makes inputs*.  It holds none of the Walsh / nonlinearity
arithmetic, so the CPU oracle (under ``oracle/``) and the HIP path can both
be fed from it without sharing any of the method.

Workload recipes (the paper's own S-boxes are not published: its AES box is
replaced by GF(2^8) inversion, which is affine-equivalent to AES and so has
the same nonlinearity, 112 (Section 6, Table 2); its two Sage-generated boxes
are replaced by seeded random permutations and random functions of the same
sizes and larger):

* ``permutation(n)``: a uniformly random bijection of {0..2^n-1}, drawn with
  an explicit Fisher-Yates shuffle.
* ``gf_inversion(n, poly)``: x -> x^(2^n - 2) in GF(2)[t]/(poly) (0 -> 0).
* ``random_function(n, m)``: 2^n iid uniform values below 2^m.
* ``mixed_batch``: box sizes n = m drawn from a weighted list, then one
  permutation per box from the same stream.
* ``poisson_trace``: exponential inter-arrival gaps at a given rate, with a
  size drawn per request.

Every generator takes a ``numpy.random.Generator`` (PCG64) so that a seed
fixes the bytes.  Tables use the narrowest unsigned dtype that holds m bits.
"""
from __future__ import annotations

import hashlib

import numpy as np

# Seed base: the arXiv number of the paper.  Workload i uses SEED_BASE + i.
SEED_BASE = 191203732

# Reduction polynomials for GF(2^n) (bit i = coefficient of t^i).  Each is
# irreducible; the test-suite checks x * inv(x) == 1 for every nonzero x.
GF_POLY = {
    3: 0xB, 4: 0x13, 5: 0x25, 6: 0x43, 7: 0x83, 8: 0x11B, 9: 0x211, 10: 0x409,
    11: 0x805, 12: 0x1053, 13: 0x201B, 14: 0x4443, 15: 0x8003, 16: 0x1002D,
}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def table_dtype(m: int):
    if m <= 8:
        return np.uint8
    if m <= 16:
        return np.uint16
    return np.uint32


def permutation(n: int, g: np.random.Generator) -> np.ndarray:
    """Fisher-Yates: for i = N-1 down to 1, swap slot i with a uniform j in [0, i]."""
    N = 1 << n
    t = np.arange(N, dtype=np.int64)
    js = g.integers(0, np.arange(N, 0, -1, dtype=np.int64))  # js[k] uniform in [0, N-1-k]
    for k in range(N - 1):
        i = N - 1 - k
        j = int(js[k])
        t[i], t[j] = t[j], t[i]
    return t.astype(table_dtype(n))


def _gf_mul(a: np.ndarray, b: np.ndarray, n: int, poly: int) -> np.ndarray:
    """Carry-less product of a and b reduced modulo poly, elementwise."""
    a = a.astype(np.int64).copy()
    b = b.astype(np.int64).copy()
    acc = np.zeros_like(a)
    top = 1 << n
    for _ in range(n):
        acc ^= np.where(b & 1, a, 0)
        b >>= 1
        a <<= 1
        a = np.where(a & top, a ^ poly, a)
    return acc


def gf_mul(a, b, n: int, poly: int | None = None) -> np.ndarray:
    return _gf_mul(np.asarray(a), np.asarray(b), n, GF_POLY[n] if poly is None else poly)


def gf_inversion(n: int, poly: int | None = None) -> np.ndarray:
    """S(x) = x^(2^n - 2) in GF(2^n), which is x^-1 for x != 0 and 0 for x = 0."""
    poly = GF_POLY[n] if poly is None else poly
    x = np.arange(1 << n, dtype=np.int64)
    e = (1 << n) - 2
    result = np.ones_like(x)
    base = x.copy()
    while e:
        if e & 1:
            result = _gf_mul(result, base, n, poly)
        base = _gf_mul(base, base, n, poly)
        e >>= 1
    result[0] = 0
    return result.astype(table_dtype(n))


def random_function(n: int, m: int, g: np.random.Generator) -> np.ndarray:
    return g.integers(0, 1 << m, size=1 << n, dtype=np.uint64).astype(table_dtype(m))


def mixed_batch(count: int, sizes, weights, g: np.random.Generator):
    """List of (n, table) with n = m drawn per box, then a permutation per box."""
    ns = g.choice(np.asarray(sizes), size=count, p=np.asarray(weights, dtype=np.float64))
    return [(int(n), permutation(int(n), g)) for n in ns]


def poisson_trace(rate: float, count: int, sizes, weights, g: np.random.Generator):
    """Arrival times (s, from 0) and sizes for an open-loop Poisson request stream."""
    gaps = g.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    ns = g.choice(np.asarray(sizes), size=count, p=np.asarray(weights, dtype=np.float64))
    return t, ns.astype(np.int64)


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


# ---------------------------------------------------------------------------
# The five workloads the test-suite and the benchmark use.
# ---------------------------------------------------------------------------

def workload_8x8(seed: int = SEED_BASE + 1):
    """Single 8x8 box: a random permutation and GF(2^8) inversion (poly 0x11B)."""
    g = rng(seed)
    return {"perm": permutation(8, g), "inv": gf_inversion(8, 0x11B), "n": 8, "m": 8}


def workload_16x16(seed: int = SEED_BASE + 2):
    """Single 16x16 box: a random permutation and GF(2^16) inversion (poly 0x1002D)."""
    g = rng(seed)
    return {"perm": permutation(16, g), "inv": gf_inversion(16, 0x1002D), "n": 16, "m": 16}


def workload_nonsquare(seed: int = SEED_BASE + 3):
    """20x16 and 16x20 uniform random functions, plus the 12x12 slice of the first:
    x -> S20x16[x] & 0xFFF for x < 4096."""
    g = rng(seed)
    s20x16 = random_function(20, 16, g)
    s16x20 = random_function(16, 20, g)
    slice12 = (s20x16[:4096].astype(np.uint32) & 0xFFF).astype(np.uint16)
    return {"s20x16": s20x16, "s16x20": s16x20, "slice12": slice12}


def workload_batched(count: int = 4096, seed: int = SEED_BASE + 4):
    """Mixed batch: n = m in {6, 8, 10, 12} with weights 0.4/0.3/0.2/0.1."""
    g = rng(seed)
    return mixed_batch(count, [6, 8, 10, 12], [0.4, 0.3, 0.2, 0.1], g)


def workload_serving(rate: float, count: int = 20000, pool: int = 64, seed: int = SEED_BASE + 5):
    """Poisson request stream, sizes 8/12/16 at 0.70/0.25/0.05; tables drawn from
    per-size pools of distinct permutations (pool boxes per size)."""
    g = rng(seed)
    t, ns = poisson_trace(rate, count, [8, 12, 16], [0.70, 0.25, 0.05], g)
    pools = {n: [permutation(n, g) for _ in range(pool)] for n in (8, 12, 16)}
    pick = g.integers(0, pool, size=count)
    return t, ns, pick, pools


def aes_sbox() -> np.ndarray:
    """The AES S-box (FIPS-197, Section 5.1.1): GF(2^8) inversion modulo 0x11B
    followed by the affine map b'_i = b_i ^ b_(i+4) ^ b_(i+5) ^ b_(i+6) ^ b_(i+7) ^ c_i
    (indices mod 8) with c = 0x63."""
    inv = gf_inversion(8, 0x11B).astype(np.int64)
    out = np.zeros_like(inv)
    for i in range(8):
        bit = ((inv >> i) ^ (inv >> ((i + 4) % 8)) ^ (inv >> ((i + 5) % 8))
               ^ (inv >> ((i + 6) % 8)) ^ (inv >> ((i + 7) % 8)) ^ (0x63 >> i)) & 1
        out |= bit << i
    return out.astype(np.uint8)
