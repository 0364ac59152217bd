"""CPU oracle for the S-box Walsh spectrum / nonlinearity path.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers.  The product path (the
HIP library and its Python binding) never imports this package, and the two
share no code.  The arithmetic lives in ``walsh_oracle.c`` (plain C, built
with gcc); this module only builds it, loads it and marshals numpy arrays.

Every routine follows the paper's definitions: the Walsh matrix of Eq. 1
(exponent read as <a,x> xor <b,S(x)>), the component functions of Eq. 2,
the nonlinearity of Eq. 3 over the nonzero output masks, the column-wise
fast transform of Algorithm 1, the fused per-column maximum of
Algorithm 3 and the minimum of Algorithm 6.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "walsh_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

B_MAJOR = 1
A_MAJOR = 2

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP over masks).  Returns the .so path."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall", "-Wextra",
               "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        lib.oracle_walsh_nl.argtypes = [u32p, ctypes.c_int, ctypes.c_int, i32p, i32p, ctypes.c_int]
        lib.oracle_walsh_maxabs_masks.argtypes = [u32p, ctypes.c_int, ctypes.c_int, u32p,
                                                  ctypes.c_int64, i32p, ctypes.c_int]
        lib.oracle_spectrum_threads.argtypes = [u32p, ctypes.c_int, ctypes.c_int, ctypes.c_int, i32p,
                                                ctypes.c_int]
        lib.oracle_nl_from_spectrum_threads.argtypes = [i32p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                                        i32p, i32p, ctypes.c_int]
        lib.oracle_walsh_column.argtypes = [u32p, ctypes.c_int, ctypes.c_int, ctypes.c_uint32, i32p]
        lib.oracle_walsh_entry.argtypes = [u32p, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32]
        lib.oracle_walsh_entry.restype = ctypes.c_int32
        lib.oracle_criteria.argtypes = [u32p, ctypes.c_int, ctypes.c_int, i32p, i32p, i32p, i32p, i32p,
                                        ctypes.c_int]
        lib.oracle_criteria.restype = ctypes.c_int
        lib.oracle_autocorrelation.argtypes = [u32p, ctypes.c_int, ctypes.c_int, ctypes.c_uint32, i32p]
        lib.oracle_autocorrelation.restype = ctypes.c_int
        lib.oracle_walsh_histogram.argtypes = [u32p, ctypes.c_int, ctypes.c_int,
                                               ctypes.POINTER(ctypes.c_uint64), ctypes.c_int]
        lib.oracle_walsh_histogram.restype = ctypes.c_int
        lib.oracle_avalanche.argtypes = [u32p, ctypes.c_int, ctypes.c_int, i32p, i32p, ctypes.c_int]
        lib.oracle_avalanche.restype = ctypes.c_int
        lib.oracle_unit_autocorrelation_masks.argtypes = [u32p, ctypes.c_int, ctypes.c_int, u32p, ctypes.c_int64,
                                                          i32p, ctypes.c_int]
        lib.oracle_unit_autocorrelation_masks.restype = ctypes.c_int
        for f in (lib.oracle_walsh_nl, lib.oracle_walsh_maxabs_masks, lib.oracle_spectrum_threads,
                  lib.oracle_nl_from_spectrum_threads, lib.oracle_walsh_column):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _table(S, n: int) -> np.ndarray:
    t = np.ascontiguousarray(np.asarray(S).astype(np.uint32, copy=False).reshape(-1))
    if t.size != (1 << n):
        raise ValueError("S must have 2^n = %d entries, got %d" % (1 << n, t.size))
    return t


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def walsh_nl(S, n: int, m: int, nthreads: int = 1):
    """Fused per-mask transform + maximum.  Returns (nl, maxabs[2^m] int32)."""
    lib = _load()
    t = _table(S, n)
    maxabs = np.empty(1 << m, dtype=np.int32)
    nl = np.zeros(1, dtype=np.int32)
    rc = lib.oracle_walsh_nl(_p(t, ctypes.c_uint32), n, m, _p(maxabs, ctypes.c_int32),
                             _p(nl, ctypes.c_int32), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_walsh_nl rejected its arguments")
    return int(nl[0]), maxabs


def maxabs_for_masks(S, n: int, m: int, masks, nthreads: int = 1) -> np.ndarray:
    """max_a |W(a, b)| for each listed nonzero mask b."""
    lib = _load()
    t = _table(S, n)
    bs = np.ascontiguousarray(np.asarray(masks, dtype=np.uint32).reshape(-1))
    out = np.empty(bs.size, dtype=np.int32)
    rc = lib.oracle_walsh_maxabs_masks(_p(t, ctypes.c_uint32), n, m, _p(bs, ctypes.c_uint32),
                                       bs.size, _p(out, ctypes.c_int32), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_walsh_maxabs_masks rejected its arguments")
    return out


def spectrum(S, n: int, m: int, layout: int = B_MAJOR, nthreads: int = 1) -> np.ndarray:
    """Full spectrum, shape (2^m, 2^n) for B_MAJOR or (2^n, 2^m) for A_MAJOR
    (masks split among nthreads threads in contiguous blocks)."""
    lib = _load()
    t = _table(S, n)
    W = np.empty(1 << (n + m), dtype=np.int32)
    rc = lib.oracle_spectrum_threads(_p(t, ctypes.c_uint32), n, m, int(layout), _p(W, ctypes.c_int32),
                                     int(nthreads))
    if rc != 0:
        raise ValueError("oracle_spectrum_threads rejected its arguments")
    return W.reshape((1 << m, 1 << n) if layout == B_MAJOR else (1 << n, 1 << m))


def nl_from_spectrum(W, n: int, m: int, layout: int = B_MAJOR, nthreads: int = 1):
    """Unfused re-scan of a stored spectrum.  Returns (nl, maxabs[2^m])."""
    lib = _load()
    w = np.ascontiguousarray(np.asarray(W, dtype=np.int32).reshape(-1))
    maxabs = np.empty(1 << m, dtype=np.int32)
    nl = np.zeros(1, dtype=np.int32)
    rc = lib.oracle_nl_from_spectrum_threads(_p(w, ctypes.c_int32), n, m, int(layout),
                                             _p(maxabs, ctypes.c_int32), _p(nl, ctypes.c_int32), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_nl_from_spectrum_threads rejected its arguments")
    return int(nl[0]), maxabs


def walsh_column(S, n: int, m: int, b: int) -> np.ndarray:
    """W(a, b) for all a."""
    lib = _load()
    t = _table(S, n)
    col = np.empty(1 << n, dtype=np.int32)
    rc = lib.oracle_walsh_column(_p(t, ctypes.c_uint32), n, m, int(b), _p(col, ctypes.c_int32))
    if rc != 0:
        raise ValueError("oracle_walsh_column rejected its arguments")
    return col


def walsh_entry(S, n: int, a: int, b: int) -> int:
    """W(a, b) summed straight from the definition."""
    lib = _load()
    t = _table(S, n)
    return int(lib.oracle_walsh_entry(_p(t, ctypes.c_uint32), n, int(a), int(b)))


CRITERIA_FIELDS = ("nl", "unbalanced", "ci_order", "resiliency", "abs_indicator", "pc_order")


def criteria(S, n: int, m: int, nthreads: int = 1):
    """Component criteria (balancedness, correlation immunity, autocorrelation).

    Returns (summary dict, per-mask dict of arrays w0, minwt, acmax, pcwt)."""
    lib = _load()
    t = _table(S, n)
    M = 1 << m
    arrs = {k: np.empty(M, dtype=np.int32) for k in ("w0", "minwt", "acmax", "pcwt")}
    summ = np.zeros(8, dtype=np.int32)
    rc = lib.oracle_criteria(_p(t, ctypes.c_uint32), n, m, _p(arrs["w0"], ctypes.c_int32),
                             _p(arrs["minwt"], ctypes.c_int32), _p(arrs["acmax"], ctypes.c_int32),
                             _p(arrs["pcwt"], ctypes.c_int32), _p(summ, ctypes.c_int32), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_criteria rejected its arguments")
    return {k: int(summ[i]) for i, k in enumerate(CRITERIA_FIELDS)}, arrs


def autocorrelation(S, n: int, m: int, b: int) -> np.ndarray:
    """r_b(d) for all d, summed from the definition."""
    lib = _load()
    t = _table(S, n)
    r = np.empty(1 << n, dtype=np.int32)
    rc = lib.oracle_autocorrelation(_p(t, ctypes.c_uint32), n, m, int(b), _p(r, ctypes.c_int32))
    if rc != 0:
        raise ValueError("oracle_autocorrelation rejected its arguments")
    return r


def walsh_histogram(S, n: int, m: int, nthreads: int = 1) -> np.ndarray:
    """hist[k] = #{(a, b): b != 0, |W(a, b)| = 2k}, k = 0 .. 2^(n-1) (uint64)."""
    lib = _load()
    t = _table(S, n)
    h = np.zeros((1 << (n - 1)) + 1, dtype=np.uint64)
    rc = lib.oracle_walsh_histogram(_p(t, ctypes.c_uint32), n, m, _p(h, ctypes.c_uint64), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_walsh_histogram rejected its arguments")
    return h


AVALANCHE_FIELDS = ("sac_max", "bic_sac_max", "bic_nl")


def avalanche(S, n: int, m: int, full: bool = True, nthreads: int = 1):
    """Unit-difference autocorrelations and the avalanche / bit-independence summary.

    Returns (summary dict, r) with r of shape (n, 2^m) (None when full is False:
    then only the entries the summary needs are summed)."""
    lib = _load()
    t = _table(S, n)
    r = np.empty((n, 1 << m), dtype=np.int32) if full else None
    summ = np.zeros(3, dtype=np.int32)
    rc = lib.oracle_avalanche(_p(t, ctypes.c_uint32), n, m, _p(r, ctypes.c_int32) if full else None,
                              _p(summ, ctypes.c_int32), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_avalanche rejected its arguments")
    return {k: int(summ[i]) for i, k in enumerate(AVALANCHE_FIELDS)}, r


def unit_autocorrelation_masks(S, n: int, m: int, masks, nthreads: int = 1) -> np.ndarray:
    """r[i, j] = r_{masks[j]}(e_i) from the definition, for a sample of masks (n <= 20)."""
    lib = _load()
    t = _table(S, n)
    bs = np.ascontiguousarray(np.asarray(masks, dtype=np.uint32))
    r = np.empty((n, bs.size), dtype=np.int32)
    rc = lib.oracle_unit_autocorrelation_masks(_p(t, ctypes.c_uint32), n, m, _p(bs, ctypes.c_uint32), bs.size,
                                               _p(r, ctypes.c_int32), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_unit_autocorrelation_masks rejected its arguments")
    return r
