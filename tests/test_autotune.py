"""Autotuner: candidate generation and the JSON cache (CPU); a real sweep
whose winner must be bit-exact against the oracle (GPU)."""
import json

import numpy as np
import pytest

from paper_1912_03732_amd import autotune


def test_valid_splits_match_the_compiled_kernels():
    assert autotune.valid_splits(5) == [5]
    assert autotune.valid_splits(9) == [6, 7, 8]
    assert autotune.valid_splits(12) == [6, 7, 8]
    assert autotune.valid_splits(13) == [7, 8]
    assert autotune.valid_splits(14) == [7, 8]
    assert autotune.valid_splits(15) == [8]
    assert autotune.valid_splits(16) == [8]


def test_candidates_cover_chunks_and_grids():
    c = autotune.candidates(12, 12, cus=256)
    assert (6, 1, 0, 1) in c and (8, 64, 512, 1) in c and (0, 8, 256, 2) in c
    assert all(p in (6, 7, 8) for p, _, _, v in c if v == 1)
    c10 = autotune.candidates(10, 10, cus=256)
    assert (6, 1, 0, 0) in c10 and {v for _, _, _, v in c10} == {0}
    c16 = autotune.candidates(16, 16)
    assert {p for p, _, _, v in c16 if v == 1} == {8} and {g for _, _, g, _ in c16} == {0}
    assert {v for _, _, _, v in c16} == {1, 2, 3}
    assert {p for p, _, _, v in c16 if v == 3} == {4, 8}  # the fp4 engine's exchange rounds
    assert {v for _, _, _, v in c} == {1, 2, 3, 4}  # at n = 12 also the fp4 and int8 first passes
    assert {p for p, _, _, v in c if v >= 2} == {0}
    assert {p for p, _, _, _ in autotune.candidates(7, 7)} == {0}


def test_cache_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv(autotune.CACHE_ENV, str(path))
    k = autotune.key("gfx950", "1.0.0", 16, 16)
    assert autotune.get(k) is None
    autotune.store(k, {"split_p": 8, "chunk": 16, "grid": 0, "ms": 1.2})
    assert json.loads(path.read_text())[k]["chunk"] == 16
    assert autotune.get(k)["split_p"] == 8
    autotune.store(autotune.key("gfx950", "1.0.0", 12, 12), {"split_p": 6, "chunk": 2, "grid": 512, "ms": 0.1})
    assert len(json.loads(path.read_text())) == 2


@pytest.mark.gpu
def test_tuned_config_is_bit_exact(tmp_path, monkeypatch):
    import oracle
    from paper_1912_03732_amd import binding as B
    from paper_1912_03732_amd import inputs
    monkeypatch.setenv(autotune.CACHE_ENV, str(tmp_path / "t.json"))
    r = autotune.tune(11, 10, reps=2)
    assert r["best"] is not None and all(x["exact"] for x in r["results"] if x["ms"] is not None)
    best = r["best"]
    S = inputs.random_function(11, 10, inputs.rng(4242))
    tun = B.sbox_tuning(best["split_p"], best["chunk"], best["grid"], 0)
    nl, mx, _ = B.walsh_nl(B.table_to_device(S, 10), 11, 10, tuning=tun)
    onl, omx = oracle.walsh_nl(S, 11, 10)
    assert nl == onl and np.array_equal(mx.cpu().numpy(), omx)
    # walsh_nl picks the cached tuning up by itself
    assert autotune.lookup(11, 10) is not None
