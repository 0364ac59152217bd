"""Shared helpers of the GPU tests (device tables, oracle comparisons)."""
import numpy as np

import oracle
from paper_1912_03732_amd import binding as B
from paper_1912_03732_amd import inputs


def dev_table(S, m):
    return B.table_to_device(S, m)


def gpu_nl(S, n, m, **kw):
    nl, mx, spec = B.walsh_nl(dev_table(S, m), n, m, **kw)
    return nl, (mx.cpu().numpy() if mx is not None else None), (spec.cpu().numpy() if spec is not None else None)


def check_against_oracle(S, n, m, nthreads=16, **kw):
    nl, mx, _ = gpu_nl(S, n, m, **kw)
    onl, omx = oracle.walsh_nl(S, n, m, nthreads=nthreads)
    assert np.array_equal(mx, omx), first_diff(mx, omx)
    assert nl == onl
    return nl, mx


def first_diff(a, b):
    idx = np.nonzero(a != b)[0]
    if idx.size == 0:
        return "equal"
    i = int(idx[0])
    return "first mismatch at b=%d: gpu %d oracle %d (%d mismatches)" % (i, int(a[i]), int(b[i]), idx.size)


def table(n, m, seed, kind="random"):
    g = inputs.rng(seed)
    if kind == "perm" and n == m:
        return inputs.permutation(n, g)
    return inputs.random_function(n, m, g)
