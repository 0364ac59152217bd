"""GPU parity of the benchmarked workloads at their full sizes, in the launch
configurations the benchmark times:

* the 4096-box mixed batch (n = m in {6, 8, 10, 12}) as one plan replayed
  from a captured HIP graph: every box's per-mask maxima and NL against the
  oracle;
* a batch with classes of >= 32 boxes at n = 9..12, so that the long work
  items of the batched launch run on every engine, including the n = 12
  matrix-core kernel;
* the 20x16 and 16x20 random functions on every mask: per-mask maxima
  against block digests of the oracle's full pass (written by
  tests/golden/make_nonsquare_digests.py, which calls only the oracle), NL
  against the oracle's, and the first differing mask named from a fresh
  oracle pass over the differing block;
* the 16 GiB b-major spectrum of the 16x16 permutation: sampled rows against
  the oracle's columns and, over all 2^32 entries, the identities every
  spectrum of a permutation satisfies (Parseval per row, even entries,
  W(0, b) = 0 for b != 0, row b = 0).
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_1912_03732_amd import binding as B
from paper_1912_03732_amd import inputs
from tests.gpu_util import dev_table, first_diff

pytestmark = pytest.mark.gpu

NT = min(16, os.cpu_count() or 1)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "nonsquare_maxabs_digests.json")


def _graph_replayed_plan(tabs, ns, ms, tuning=None):
    """Plan launched once, then captured into a HIP graph and replayed with
    its outputs poisoned in between (as the benchmark runs it)."""
    import torch
    plan = B.Plan(tabs, ns, ms, tuning=tuning)
    plan.launch()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch()
    plan.nl.fill_(-7)
    for t in plan.maxabs:
        t.fill_(-7)
    torch.cuda.synchronize()
    for _ in range(2):
        g.replay()
    torch.cuda.synchronize()
    return plan, g


def test_batched_workload_4096_graph_replay_vs_oracle():
    batch = inputs.workload_batched()
    assert len(batch) == 4096
    tabs = [dev_table(S, n) for n, S in batch]
    ns = [n for n, _ in batch]
    plan, g = _graph_replayed_plan(tabs, ns, ns)
    nl = plan.nl.cpu().numpy()
    mxs = [t.cpu().numpy() for t in plan.maxabs]
    counts = {}
    for i, (n, S) in enumerate(batch):
        onl, omx = oracle.walsh_nl(S, n, n, nthreads=NT if n >= 10 else 1)
        assert nl[i] == onl, (i, n, int(nl[i]), onl)
        assert np.array_equal(mxs[i], omx), (i, n, first_diff(mxs[i], omx))
        counts[n] = counts.get(n, 0) + 1
    # every size class is large enough for the long-item rule of the batched launch
    assert all(c >= 32 for c in counts.values()), counts
    plan.close()


@pytest.mark.parametrize("variant", [0, 1, 4])
def test_batched_long_items_every_engine(variant):
    """Classes of >= 32 boxes at n = 9, 10, 11, 12 (ragged m, so items cover
    partial boxes too), with the default engines (matrix cores at n = 12),
    the VALU kernels everywhere, or the int8 first pass at n = 12."""
    g = inputs.rng(10701 + variant)
    boxes = []
    for n, count in ((12, 72), (11, 33), (10, 40), (9, 32), (6, 5)):
        for k in range(count):
            m = n if k % 3 == 0 else int(g.integers(1, 17))
            S = inputs.permutation(n, g) if m == n else inputs.random_function(n, m, g)
            boxes.append((n, m, S))
    order = g.permutation(len(boxes))
    boxes = [boxes[i] for i in order]
    tabs = [dev_table(S, m) for n, m, S in boxes]
    tuning = B.sbox_tuning(0, 0, 0, variant) if variant else None
    plan, _ = _graph_replayed_plan(tabs, [b[0] for b in boxes], [b[1] for b in boxes], tuning=tuning)
    nl = plan.nl.cpu().numpy()
    for i, (n, m, S) in enumerate(boxes):
        onl, omx = oracle.walsh_nl(S, n, m, nthreads=NT)
        mx = plan.maxabs[i].cpu().numpy()
        assert nl[i] == onl, (variant, i, n, m)
        assert np.array_equal(mx, omx), (variant, i, n, m, first_diff(mx, omx))
    plan.close()


def _digests(maxabs, block):
    a = np.ascontiguousarray(maxabs.astype("<i4"))
    return [hashlib.sha256(a[i:i + block].tobytes()).hexdigest()[:32] for i in range(0, a.size, block)]


@pytest.mark.parametrize("key", ["s20x16", "s16x20"])
def test_nonsquare_workload_every_mask(key):
    with open(GOLDEN) as f:
        rec = json.load(f)
    box = rec["boxes"][key]
    n, m, block = box["n"], box["m"], rec["block_masks"]
    S = inputs.workload_nonsquare()[key]
    assert inputs.sha256(S) == box["table_sha256"], "input generator changed: regenerate the digests"
    nl, mx, _ = B.walsh_nl(dev_table(S, m), n, m)
    mx = mx.cpu().numpy()
    got = _digests(mx, block)
    bad = [i for i, (a, b) in enumerate(zip(got, box["block_sha256_32"])) if a != b]
    if bad:
        i = bad[0]
        masks = np.arange(i * block, min((i + 1) * block, 1 << m), dtype=np.uint32)
        ref = oracle.maxabs_for_masks(S, n, m, masks[masks > 0], nthreads=NT)
        if i == 0:
            ref = np.concatenate([[1 << n], ref])
        pytest.fail("%s: %d of %d blocks differ; block %d: %s"
                    % (key, len(bad), len(got), i, first_diff(mx[masks], ref)))
    assert len(got) == len(box["block_sha256_32"])
    assert nl == box["nl"]
    assert int(mx[1:].max()) == box["maxabs_max"] and int(mx[1:].min()) == box["maxabs_min"]


def test_b_major_spectrum_16x16_full_size():
    """The whole 16 GiB b-major spectrum of the 16x16 permutation in the
    launch the benchmark's spectrum workload uses."""
    import torch
    n = m = 16
    S = inputs.workload_16x16()["perm"]
    t = dev_table(S, m)
    spec = torch.empty(1 << (n + m), dtype=torch.int32, device="cuda")
    mx = torch.empty(1 << m, dtype=torch.int32, device="cuda")
    nl = torch.empty(1, dtype=torch.int32, device="cuda")
    ws = B.Workspace(B.sbox_walsh_nl_workspace_bytes(n, m, B.SPECTRUM_B_MAJOR))
    st = B.sbox_walsh_nl_ex(t.data_ptr(), n, m, 2, mx.data_ptr(), nl.data_ptr(), spec.data_ptr(),
                            B.SPECTRUM_B_MAJOR, ws.ptr, ws.nbytes, None, int(torch.cuda.current_stream().cuda_stream))
    assert st == B.SBOX_OK, B.last_error()
    torch.cuda.synchronize()
    W = spec.view(1 << m, 1 << n)
    g = inputs.rng(10801)
    rows = sorted(set([1, 2, 3, 0x8000, 0xFFFF, 0xFFFE, 0x5555, 0xAAAA]
                      + [int(v) for v in g.integers(1, 1 << m, size=40)]))
    got = W[torch.tensor(rows, device="cuda")].cpu().numpy()
    for k, b in enumerate(rows):
        ref = oracle.walsh_column(S, n, m, b)
        assert np.array_equal(got[k], ref), (b, first_diff(got[k], ref))
    # identities over every entry, 4096 rows at a time
    full = 1 << n
    assert int(W[0, 0].item()) == full and int(W[0, 1:].abs().sum().item()) == 0
    for r0 in range(0, 1 << m, 4096):
        blk = W[r0:r0 + 4096]
        assert not bool((blk & 1).any()), r0
        sq = blk.to(torch.float64).square().sum(dim=1)  # exact: sums below 2^53
        lo = 1 if r0 == 0 else 0
        assert bool((sq[lo:] == float(full) * full).all()), r0
        assert bool((blk[lo:, 0] == 0).all()), r0
    ref_nl, ref_mx = oracle.walsh_nl(S, n, m, nthreads=NT)
    assert int(nl.item()) == ref_nl
    assert np.array_equal(mx.cpu().numpy(), ref_mx)
    del W, spec
    torch.cuda.empty_cache()
