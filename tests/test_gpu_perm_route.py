"""GPU parity of the a-major spectrum of n = m boxes (n >= 14), whose call
decides on the device whether the box is a permutation: if it is, the rows
of the b-major matrix of the inverse map are the a-major matrix (Eq. 1 with
y = S(x) substituted), else the transposed slabs write it.  Both routes run
here, on permutations and on boxes one entry away from one, against the
oracle's a-major spectrum (Alg. 1), alone and replayed from one captured
HIP graph with the table switched between the two kinds."""
import numpy as np
import pytest

import oracle
from paper_1912_03732_amd import binding as B
from paper_1912_03732_amd import inputs
from tests.gpu_util import dev_table, first_diff

pytestmark = pytest.mark.gpu

NT = 16


def _not_onto(S, seed):
    """S with one entry replaced by another's value: no longer a permutation."""
    g = inputs.rng(seed)
    i, j = (int(v) for v in g.choice(S.size, size=2, replace=False))
    T = S.copy()
    T[i] = T[j]
    return T


def _full_check(S, n, kind, maxabs):
    import torch
    nl, mx, spec = B.walsh_nl(dev_table(S, n), n, n, spectrum=kind, maxabs=maxabs)
    ref = oracle.spectrum(S, n, n, oracle.A_MAJOR, nthreads=NT)
    if kind == "lat-a":
        ref //= 2
    got = spec.cpu().numpy()
    del spec
    torch.cuda.empty_cache()
    for a in range(0, 1 << n, 1024):  # row blocks: a readable first difference
        blk, rblk = got[a:a + 1024], ref[a:a + 1024]
        assert np.array_equal(blk, rblk), (kind, a, first_diff(blk.ravel(), rblk.ravel()))
    onl, omx = oracle.walsh_nl(S, n, n, nthreads=NT)
    assert nl == onl
    if maxabs:
        mx = mx.cpu().numpy()
        assert np.array_equal(mx, omx), first_diff(mx, omx)


@pytest.mark.parametrize("kind,maxabs", [("a", True), ("lat-a", False)])
def test_permutation_14_full(kind, maxabs):
    """A 14x14 permutation: every entry; with the per-mask maxima (fused pass
    over S) or without them (NL from the rows of S^-1)."""
    S = inputs.permutation(14, inputs.rng(15100))
    _full_check(S, 14, kind, maxabs)


@pytest.mark.parametrize("kind,maxabs", [("a", True), ("lat-a", False)])
def test_not_a_permutation_14_full(kind, maxabs):
    """The same permutation with one repeated value: the slab route."""
    S = _not_onto(inputs.permutation(14, inputs.rng(15100)), 15101)
    _full_check(S, 14, kind, maxabs)


def test_affine_permutation_14():
    """x -> x ^ c, a permutation with |W| = 2^14 on the diagonal (W(a, a) =
    2^14 (-1)^(a . c)) and 0 elsewhere: NL = 0."""
    n = 14
    S = (np.arange(1 << n) ^ 0x2B5D).astype(np.uint16)
    _full_check(S, n, "a", True)


@pytest.mark.parametrize("kind", ["perm", "not", "affine", "affine-lat"])
def test_15_and_16_sampled(kind):
    """n = m = 15 and 16: sampled columns and rows against the oracle, and
    for a permutation Parseval over b on the first 4096 rows a (row a of S's
    matrix is the spectrum of the component a . S^-1).  The affine map
    x -> x ^ c reaches |W| = 2^n, at n = 16 one past the int16 range, also
    as the LAT (W/2)."""
    import torch
    perm = kind != "not"
    lat = kind.endswith("-lat")
    for n in (15, 16):
        S = inputs.permutation(n, inputs.rng(15200 + n))
        if kind == "not":
            S = _not_onto(S, 15210 + n)
        if kind.startswith("affine"):
            S = (np.arange(1 << n) ^ (0x5A3C & ((1 << n) - 1))).astype(np.uint16)
        nl, mx, spec = B.walsh_nl(dev_table(S, n), n, n, spectrum="lat-a" if lat else "a")
        div = 2 if lat else 1
        g = inputs.rng(15220 + n)
        for b in [0, 1, (1 << n) - 1] + [int(v) for v in g.integers(1, 1 << n, size=4)]:
            col = spec[:, b].cpu().numpy()
            ref = oracle.walsh_column(S, n, n, b) // div
            assert np.array_equal(col, ref), (n, kind, b, first_diff(col, ref))
        for a in [0, 1, (1 << n) - 1, int(g.integers(2, 1 << n))]:
            row = spec[a, ::257].cpu().numpy()
            ref = np.array([oracle.walsh_entry(S, n, a, b) for b in range(0, 1 << n, 257)]) // div
            assert np.array_equal(row, ref), (n, kind, a, first_diff(row, ref))
        if perm:
            sq = spec[:4096].to(torch.float64).square().sum(dim=1)
            assert bool((sq == float(1 << (2 * n)) / (div * div)).all())
        onl, omx = oracle.walsh_nl(S, n, n, nthreads=NT)
        assert nl == onl
        assert np.array_equal(mx.cpu().numpy(), omx)
        del spec
        torch.cuda.empty_cache()


def test_graph_replay_switches_route():
    """One captured call on a 14x14 table buffer, replayed with a permutation,
    then a box that is not one, then the permutation again (eager work and
    poisoned outputs between): each replay takes its route on the device."""
    import torch
    n = 14
    P = inputs.permutation(n, inputs.rng(15300))
    Q = _not_onto(P, 15301)
    refs = {}
    for key, S in (("perm", P), ("not", Q)):
        refs[key] = (oracle.spectrum(S, n, n, oracle.A_MAJOR, nthreads=NT), oracle.walsh_nl(S, n, n, nthreads=NT))
    t = dev_table(P, n)
    ws = B.Workspace(B.sbox_walsh_nl_workspace_bytes(n, n, B.SPECTRUM_A_MAJOR))
    spec = torch.empty(1 << (2 * n), dtype=torch.int32, device="cuda")
    mx = torch.empty(1 << n, dtype=torch.int32, device="cuda")
    nl = torch.empty(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        st = B.sbox_walsh_nl_ex(t.data_ptr(), n, n, t.element_size(), mx.data_ptr(), nl.data_ptr(),
                                spec.data_ptr(), B.SPECTRUM_A_MAJOR, ws.ptr, ws.nbytes, None, int(s.cuda_stream))
    assert st == B.SBOX_OK, B.last_error()
    for rep, key in enumerate(("perm", "not", "perm")):
        t.copy_(dev_table(P if key == "perm" else Q, n))
        spec.fill_(-7)
        mx.fill_(-7)
        nl.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        rspec, (rnl, rmx) = refs[key]
        got = spec.view(1 << n, 1 << n).cpu().numpy()
        assert np.array_equal(got, rspec), (rep, key, first_diff(got.ravel(), rspec.ravel()))
        assert int(nl.item()) == rnl, (rep, key)
        assert np.array_equal(mx.cpu().numpy(), rmx), (rep, key)
    del spec
    torch.cuda.empty_cache()

