"""The C-ABI library: it loads, exports every symbol include/sbox_walsh.h
declares, and rejects invalid arguments on the host before touching the GPU
(no compute call is made here)."""
import ctypes
import os
import re

import pytest

from paper_1912_03732_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sbox_walsh.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(sbox_[a-z_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.fail("libsboxwalsh.so not built: run __graft_entry__.build()")
    return B.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(B.EXPORTS)


def test_version(lib):
    assert re.match(r"^\d+\.\d+\.\d+$", B.sbox_version())


@pytest.mark.parametrize("n,m,layout,ok", [
    (1, 1, 0, True), (16, 16, 0, True), (24, 16, 0, True), (16, 24, 0, True),
    (0, 4, 0, False), (4, 0, 0, False), (25, 1, 0, False), (20, 21, 0, False),
    (16, 16, 1, True), (16, 18, 2, True), (20, 16, 1, False), (4, 4, 3, False), (4, 4, -1, False),
    (8, 8, 0x11, True), (8, 8, 0x12, True), (8, 8, 0x10, False), (8, 8, 0x13, False)])
def test_workspace_query(lib, n, m, layout, ok):
    v = B.sbox_walsh_nl_workspace_bytes(n, m, layout)
    assert (v > 0) == ok
    if ok and n <= 16:
        # queue counters + m bit-sliced slices of 2^(n-5) words
        assert v >= 256 + m * (1 << max(0, n - 5)) * 4


def test_large_n_workspace_grows_with_n(lib):
    assert B.sbox_walsh_nl_workspace_bytes(20, 16, 0) > B.sbox_walsh_nl_workspace_bytes(17, 16, 0) > 0


@pytest.mark.parametrize("n", [12, 13, 14, 15, 16])
def test_a_major_workspace_holds_the_inverse_route(lib, n):
    """An a-major spectrum (or LAT) with n = m >= 14 also holds the inverse
    table (uint16), its bit-sliced words and a flag beside the slab; the
    b-major layout, non-square boxes and n = m < 14 do not."""
    a = B.sbox_walsh_nl_workspace_bytes(n, n, B.SPECTRUM_A_MAJOR)
    assert a == B.sbox_walsh_nl_workspace_bytes(n, n, B.LAT_A_MAJOR)
    b = B.sbox_walsh_nl_workspace_bytes(n, n, B.SPECTRUM_B_MAJOR)
    slab = min(1 << n, max(64, (1 << 27) >> n)) * (1 << n) * 2   # int16 rows of 2^27 entries at most
    route = 256 + (2 << n) + n * (1 << (n - 3))                   # flag, inverse table, its words
    assert a - b == slab + (route if n >= 14 else 0)
    # non-square boxes take the slab only
    if n <= 15:
        a1 = B.sbox_walsh_nl_workspace_bytes(n, n + 1, B.SPECTRUM_A_MAJOR)
        b1 = B.sbox_walsh_nl_workspace_bytes(n, n + 1, B.SPECTRUM_B_MAJOR)
        assert a1 - b1 == min(1 << (n + 1), max(64, (1 << 27) >> n)) * (1 << n) * 2


@pytest.mark.parametrize("args,status", [
    (dict(n=0, m=4), B.SBOX_ERR_UNSUPPORTED),
    (dict(n=4, m=25), B.SBOX_ERR_UNSUPPORTED),
    (dict(S=0), B.SBOX_ERR_INVALID_ARG),
    (dict(nl=0), B.SBOX_ERR_INVALID_ARG),
    (dict(eb=3), B.SBOX_ERR_INVALID_ARG),
    (dict(layout=5), B.SBOX_ERR_INVALID_ARG),
    (dict(layout=1, spec=0), B.SBOX_ERR_INVALID_ARG),
    (dict(ws=0), B.SBOX_ERR_WORKSPACE),
    (dict(ws_bytes=16), B.SBOX_ERR_WORKSPACE),
    (dict(ws=4096 + 8), B.SBOX_ERR_INVALID_ARG),
    (dict(n=12, tuning=B.sbox_tuning(5, 0, 0, 0)), B.SBOX_ERR_INVALID_ARG),
    (dict(n=16, tuning=B.sbox_tuning(7, 0, 0, 0)), B.SBOX_ERR_INVALID_ARG),
    (dict(tuning=B.sbox_tuning(0, -1, 0, 0)), B.SBOX_ERR_INVALID_ARG),
    (dict(tuning=B.sbox_tuning(0, 0, 0, 5)), B.SBOX_ERR_INVALID_ARG),
    (dict(tuning=B.sbox_tuning(0, 0, 0, 4)), B.SBOX_ERR_INVALID_ARG),
    (dict(n=16, m=16, tuning=B.sbox_tuning(0, 0, 0, 4)), B.SBOX_ERR_INVALID_ARG),
    (dict(n=12, m=12, layout=1, spec=4096, tuning=B.sbox_tuning(0, 0, 0, 4)), B.SBOX_ERR_INVALID_ARG),
    (dict(n=13, tuning=B.sbox_tuning(0, 0, 0, 3)), B.SBOX_ERR_INVALID_ARG),
    (dict(n=12, m=12, layout=1, spec=4096, tuning=B.sbox_tuning(0, 0, 0, 3)), B.SBOX_ERR_INVALID_ARG),
    (dict(n=16, m=8, tuning=B.sbox_tuning(6, 0, 0, 3)), B.SBOX_ERR_INVALID_ARG),
    (dict(n=16, m=16, layout=1, spec=4096, tuning=B.sbox_tuning(0, 0, 0, 3)), B.SBOX_ERR_INVALID_ARG),
    (dict(n=13, tuning=B.sbox_tuning(0, 0, 0, 2)), B.SBOX_ERR_INVALID_ARG),
    (dict(n=12, m=12, layout=1, spec=4096, tuning=B.sbox_tuning(0, 0, 0, 2)), B.SBOX_ERR_INVALID_ARG),
    (dict(n=16, m=16, layout=1, spec=4096, tuning=B.sbox_tuning(0, 0, 0, 2)), B.SBOX_ERR_INVALID_ARG),
])
def test_invalid_arguments_rejected_before_launch(lib, args, status):
    # Fake (never dereferenced) pointers: validation rejects before any HIP call.
    a = dict(S=4096, n=8, m=8, eb=1, mx=0, nl=8192, spec=0, layout=0, ws=4096, ws_bytes=1 << 20,
             tuning=None)
    a.update(args)
    st = B.sbox_walsh_nl_ex(a["S"], a["n"], a["m"], a["eb"], a["mx"], a["nl"], a["spec"], a["layout"],
                            a["ws"], a["ws_bytes"], a["tuning"], 0)
    assert st == status
    assert B.sbox_last_error() != ""


def test_batched_rejects_large_n_and_bad_jobs(lib):
    jobs = (B.sbox_job * 2)()
    jobs[0].S, jobs[0].n, jobs[0].m, jobs[0].s_elem_bytes, jobs[0].nl = 4096, 17, 4, 1, 8192
    assert B.sbox_walsh_nl_batched(jobs, 1, 4096, 1 << 20, 0) == B.SBOX_ERR_UNSUPPORTED
    jobs[0].n, jobs[0].s_elem_bytes = 8, 3
    assert B.sbox_walsh_nl_batched(jobs, 1, 4096, 1 << 20, 0) == B.SBOX_ERR_INVALID_ARG
    jobs[0].s_elem_bytes, jobs[0].nl = 1, None
    assert B.sbox_walsh_nl_batched(jobs, 1, 4096, 1 << 20, 0) == B.SBOX_ERR_INVALID_ARG
    assert B.sbox_walsh_nl_batched(jobs, -1, 4096, 1 << 20, 0) == B.SBOX_ERR_INVALID_ARG
    assert B.sbox_plan_launch(None, 0) == B.SBOX_ERR_INVALID_ARG
    st, h = B.sbox_plan_create(jobs, 1, None)
    assert st == B.SBOX_ERR_INVALID_ARG and not h
    B.sbox_plan_destroy(None)  # no-op


def test_gray_code_block_mapping():
    """The a-major slab path relies on this: Gray indices in block i visit
    exactly the masks of block gray(i), so mask block j is covered by index
    block gray^-1(j)."""
    def gray(k):
        return k ^ (k >> 1)

    def inverse_gray(j):
        r = 0
        while j:
            r ^= j
            j >>= 1
        return r
    R = 64
    for j in range(32):
        assert sorted(gray(k) for k in range(j * R, (j + 1) * R)) == list(range(gray(j) * R, (gray(j) + 1) * R))
        i = inverse_gray(j)
        assert gray(i) == j
        assert sorted(gray(k) for k in range(i * R, (i + 1) * R)) == list(range(j * R, (j + 1) * R))


@pytest.mark.parametrize("args,status", [
    (dict(n=17), B.SBOX_ERR_UNSUPPORTED),
    (dict(m=25), B.SBOX_ERR_UNSUPPORTED),
    (dict(S=0), B.SBOX_ERR_INVALID_ARG),
    (dict(hist=0), B.SBOX_ERR_INVALID_ARG),
    (dict(eb=3), B.SBOX_ERR_INVALID_ARG),
    (dict(ws=0), B.SBOX_ERR_WORKSPACE),
    (dict(ws_bytes=64), B.SBOX_ERR_WORKSPACE),
    (dict(ws=4096 + 8), B.SBOX_ERR_INVALID_ARG),
])
def test_histogram_rejects_invalid_arguments(lib, args, status):
    a = dict(S=4096, n=8, m=8, eb=1, hist=8192, ws=4096, ws_bytes=1 << 20)
    a.update(args)
    assert B.sbox_walsh_histogram(a["S"], a["n"], a["m"], a["eb"], a["hist"], 0, 0, a["ws"], a["ws_bytes"],
                                  0) == status
    assert B.sbox_last_error() != ""


def test_histogram_workspace_query(lib):
    assert B.sbox_walsh_histogram_workspace_bytes(16, 16) > B.sbox_walsh_nl_workspace_bytes(16, 16, 0)
    assert B.sbox_walsh_histogram_workspace_bytes(17, 4) == 0
    assert B.sbox_walsh_histogram_workspace_bytes(8, 25) == 0


@pytest.mark.parametrize("args,status", [
    (dict(n=25), B.SBOX_ERR_UNSUPPORTED),
    (dict(m=21), B.SBOX_ERR_UNSUPPORTED),
    (dict(n=22, m=19), B.SBOX_ERR_UNSUPPORTED),
    (dict(S=0), B.SBOX_ERR_INVALID_ARG),
    (dict(summary=0), B.SBOX_ERR_INVALID_ARG),
    (dict(eb=5), B.SBOX_ERR_INVALID_ARG),
    (dict(ws=0), B.SBOX_ERR_WORKSPACE),
    (dict(ws_bytes=1024), B.SBOX_ERR_WORKSPACE),
    (dict(ws=4096 + 4), B.SBOX_ERR_INVALID_ARG),
])
def test_avalanche_rejects_invalid_arguments(lib, args, status):
    a = dict(S=4096, n=8, m=8, eb=1, r=0, summary=8192, ws=4096, ws_bytes=1 << 20)
    a.update(args)
    assert B.sbox_avalanche(a["S"], a["n"], a["m"], a["eb"], a["r"], a["summary"], 0, a["ws"], a["ws_bytes"],
                            0) == status
    assert B.sbox_last_error() != ""


def test_avalanche_workspace_query(lib):
    assert B.sbox_avalanche_workspace_bytes(16, 16) == 16 * 65536 * 4
    assert B.sbox_avalanche_workspace_bytes(24, 16) == 24 * 65536 * 4
    assert B.sbox_avalanche_workspace_bytes(8, 21) == 0
    assert B.sbox_avalanche_workspace_bytes(0, 4) == 0


@pytest.mark.parametrize("args,status", [
    (dict(n=17), B.SBOX_ERR_UNSUPPORTED),
    (dict(n=16, m=25), B.SBOX_ERR_UNSUPPORTED),
    (dict(S=0), B.SBOX_ERR_INVALID_ARG),
    (dict(summary=0), B.SBOX_ERR_INVALID_ARG),
    (dict(eb=3), B.SBOX_ERR_INVALID_ARG),
    (dict(ws=0), B.SBOX_ERR_WORKSPACE),
    (dict(ws_bytes=4096), B.SBOX_ERR_WORKSPACE),
    (dict(ws=4096 + 16), B.SBOX_ERR_INVALID_ARG),
])
def test_criteria_ex_rejects_invalid_arguments(lib, args, status):
    a = dict(S=4096, n=16, m=4, eb=2, summary=8192, ws=4096, ws_bytes=1 << 30)
    a.update(args)
    assert B.sbox_criteria_ex(a["S"], a["n"], a["m"], a["eb"], a["summary"], 0, 0, 0, 0, a["ws"], a["ws_bytes"],
                              0) == status
    assert B.sbox_last_error() != ""


def test_criteria_without_workspace_stops_at_14(lib):
    assert B.sbox_criteria(4096, 15, 4, 2, 8192, 0, 0, 0, 0, 0) == B.SBOX_ERR_UNSUPPORTED
    # n = 15, 16: the same words and slots (the transforms stay on chip)
    assert B.sbox_criteria_workspace_bytes(16, 16) == 16 * 2048 * 4 + 4096 * 32
    # 5 <= n <= 14: the bit-sliced words (m x 2^(n-5) x 4 bytes, 256-aligned) of the register-blocked
    # kernel and 4096 slots of 8 ints for its per-workgroup aggregates
    assert B.sbox_criteria_workspace_bytes(14, 8) == 8 * 512 * 4 + 4096 * 32
    assert B.sbox_criteria_workspace_bytes(5, 3) == 256 + 4096 * 32
    assert B.sbox_criteria_workspace_bytes(4, 4) == 256
    assert B.sbox_criteria_workspace_bytes(17, 4) == 0


def test_criteria_ex_small_n_workspace_checked_when_given(lib):
    """For 5 <= n <= 14 a workspace is optional, but one that is passed must
    be aligned and large enough."""
    need = B.sbox_criteria_workspace_bytes(12, 8)
    assert B.sbox_criteria_ex(4096, 12, 8, 1, 8192, 0, 0, 0, 0, 4096, need - 1, 0) == B.SBOX_ERR_WORKSPACE
    assert B.sbox_criteria_ex(4096, 12, 8, 1, 8192, 0, 0, 0, 0, 4096 + 16, need, 0) == B.SBOX_ERR_INVALID_ARG


def test_short_form_and_reservation_validate_on_the_host(lib):
    """The short form and the scratch reservation check their arguments
    before any HIP call (the GPU tests cover the missing-reservation path)."""
    assert B.sbox_walsh_nl(0, 8, 8, 0, 8192, 0) == B.SBOX_ERR_INVALID_ARG
    assert B.sbox_walsh_nl(4096, 8, 8, 0, 0, 0) == B.SBOX_ERR_INVALID_ARG
    assert B.sbox_walsh_nl(4096, 0, 8, 0, 8192, 0) == B.SBOX_ERR_UNSUPPORTED
    assert B.sbox_walsh_nl(4096, 20, 21, 0, 8192, 0) == B.SBOX_ERR_UNSUPPORTED
    assert B.sbox_scratch_reserve(0, 4, 0) == B.SBOX_ERR_UNSUPPORTED
    assert B.sbox_scratch_reserve(25, 1, 0) == B.SBOX_ERR_UNSUPPORTED
    assert "unsupported" in B.sbox_last_error()
