"""Seeded input generators: determinism, bijectivity, field arithmetic."""
import json
import os

import numpy as np
import pytest

from paper_1912_03732_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_permutation_is_bijection_and_deterministic():
    for n in (1, 2, 5, 8, 12):
        p1 = inputs.permutation(n, inputs.rng(7))
        p2 = inputs.permutation(n, inputs.rng(7))
        assert np.array_equal(p1, p2)
        assert sorted(p1.tolist()) == list(range(1 << n))
        assert p1.dtype == inputs.table_dtype(n)
    assert not np.array_equal(inputs.permutation(8, inputs.rng(1)), inputs.permutation(8, inputs.rng(2)))


@pytest.mark.parametrize("n", sorted(inputs.GF_POLY))
def test_gf_inversion_is_field_inverse(n):
    inv = inputs.gf_inversion(n).astype(np.int64)
    x = np.arange(1, 1 << n)
    prod = inputs.gf_mul(x, inv[1:], n)
    # x * x^-1 == 1 for every nonzero x also proves the polynomial is irreducible
    assert np.all(prod == 1)
    assert inv[0] == 0
    assert sorted(inv.tolist()) == list(range(1 << n))


def test_aes_table_matches_fips197_entries():
    with open(os.path.join(GOLDEN, "fips197_sbox.json")) as f:
        gold = json.load(f)
    s = inputs.aes_sbox()
    for x, y in gold["entries"].items():
        assert int(s[int(x)]) == y


def test_random_function_range_and_dtype():
    f = inputs.random_function(10, 20, inputs.rng(3))
    assert f.size == 1024 and f.dtype == np.uint32 and int(f.max()) < (1 << 20)
    g = inputs.random_function(10, 5, inputs.rng(3))
    assert g.dtype == np.uint8 and int(g.max()) < 32


def test_workloads_are_reproducible():
    a = inputs.workload_8x8()
    b = inputs.workload_8x8()
    assert inputs.sha256(a["perm"]) == inputs.sha256(b["perm"])
    batch1 = inputs.workload_batched(count=64)
    batch2 = inputs.workload_batched(count=64)
    assert [n for n, _ in batch1] == [n for n, _ in batch2]
    assert all(np.array_equal(s1, s2) for (_, s1), (_, s2) in zip(batch1, batch2))
    assert set(n for n, _ in batch1) <= {6, 8, 10, 12}


def test_poisson_trace_shape():
    t, ns = inputs.poisson_trace(1000.0, 500, [8, 12, 16], [0.7, 0.25, 0.05], inputs.rng(5))
    assert t.shape == (500,) and t[0] == 0.0 and np.all(np.diff(t) >= 0)
    assert set(ns.tolist()) <= {8, 12, 16}
    # mean gap close to 1/rate
    assert 0.5e-3 < float(np.mean(np.diff(t))) < 2e-3
