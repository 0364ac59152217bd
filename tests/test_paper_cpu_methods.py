"""The rerun of the paper's CPU methods (Table 4: the primary a-major
matrix with a separate scan, (a) the transposed matrix, (b) the same over
threads, (c) the fused maximum; Fig. ch1's thread sweep) that the
benchmark's CPU-baseline leg reports: every method reaches the same NL, the
closed form where there is one."""
import bench
from paper_1912_03732_amd import inputs
import oracle


def test_table4_methods_agree_on_small_boxes():
    out = bench.paper_table4(sizes=((6, 6), (8, 8)), sweep_size=(8, 8), sweep=range(1, 4), threads=3)
    for key in ("6x6", "8x8"):
        row = out[key]
        nls = {name: r["nl"] for name, r in row.items()}
        assert len(set(nls.values())) == 1, nls
        n = int(key.split("x")[0])
        S = inputs.permutation(n, inputs.rng(inputs.SEED_BASE + 10 + n))
        assert nls["c_fused"] == oracle.walsh_nl(S, n, n)[0]
        assert row["primary"]["threads"] == 1 and row["b_threads"]["threads"] == 3
        assert all(r["fwht_ms"] >= 0 and r["nl_ms"] >= 0 for r in row.values())
    assert sorted(out["thread_sweep_b_8x8_fwht_ms"]) == ["1", "2", "3"]
