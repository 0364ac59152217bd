"""CPU checks of the benchmark's bookkeeping: the HBM traffic figure is
reported only while the kernel source it was measured on is unchanged, and
the matrix-core instruction counts and peaks the roofline uses agree with
the instruction shapes and the 16-cycle rates of gfx950."""
import json
import os
import shutil

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join("paper_1912_03732_amd", "csrc", "walsh_kernels.hpp")


@pytest.fixture
def tree(tmp_path, monkeypatch):
    """A copy of the kernel header and the profiles folder under a temporary root."""
    os.makedirs(tmp_path / "paper_1912_03732_amd" / "csrc")
    shutil.copy(os.path.join(ROOT, HDR), tmp_path / HDR)
    os.makedirs(tmp_path / "profiles")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    return tmp_path


def _edit(path, old, new):
    text = path.read_text()
    assert text.count(old) >= 1, old
    path.write_text(text.replace(old, new, 1))


def test_traffic_reported_only_for_the_measured_source(tree):
    digest = bench.kernel_source_digest(3)
    assert len(digest) == 16 and int(digest, 16) >= 0
    rec = {"kernel_source_sha256_16": digest, "traffic_bytes_per_dispatch": 12345}
    (tree / "profiles" / "t.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("t.json", 3) == 12345
    rec["kernel_source_sha256_16"] = "0" * 16
    (tree / "profiles" / "t.json").write_text(json.dumps(rec))
    assert bench.measured_traffic("t.json", 3) is None
    assert bench.measured_traffic("missing.json", 3) is None


def test_digest_follows_the_kernel_section_and_the_shared_prefix(tree):
    hdr = tree / HDR
    d3, d2 = bench.kernel_source_digest(3), bench.kernel_source_digest(2)
    # an edit inside the fp4 16x16 kernel's section changes only its digest
    start, func = bench.KERNEL_SECTIONS[3]
    text = hdr.read_text()
    i = text.index(func, text.index(start))
    hdr.write_text(text[:i] + "/* edit */ " + text[i:])
    assert bench.kernel_source_digest(3) != d3
    assert bench.kernel_source_digest(2) == d2
    # an edit in the definitions shared by every kernel changes both
    shutil.copy(os.path.join(ROOT, HDR), hdr)
    _edit(hdr, "constexpr int kWG = 256;", "constexpr int kWG = 256; /* edit */")
    assert bench.kernel_source_digest(3) != d3 and bench.kernel_source_digest(2) != d2
    # an edit in another kernel (the criteria) changes neither
    shutil.copy(os.path.join(ROOT, HDR), hdr)
    _edit(hdr, "void k_crit_wide(const CritRegParams p) {", "void k_crit_wide(const CritRegParams p) { /* edit */")
    assert bench.kernel_source_digest(3) == d3 and bench.kernel_source_digest(2) == d2


def test_committed_traffic_files_are_consistent():
    for variant, info in bench.KERNELS.items():
        path = os.path.join(ROOT, "profiles", info["traffic"])
        if not os.path.exists(path):
            continue
        with open(path) as f:
            rec = json.load(f)
        kib = rec["fetch_size_kib_per_dispatch"] * rec["fetch_scale"] + rec["write_size_kib_per_dispatch"] * rec["write_scale"]
        assert abs(rec["traffic_bytes_per_dispatch"] - kib * 1024) <= 0.001 * kib * 1024 + 64, variant
        # the scales are what a plain 1 GiB device copy read on the two counters
        cr = rec["copy_reference"]
        assert abs(rec["fetch_scale"] - (cr["bytes"] / 1024) / cr["fetch_size_kib"]) < 0.01
        assert abs(rec["write_scale"] - (cr["bytes"] / 1024) / cr["write_size_kib"]) < 0.01


def test_matrix_core_counts_and_peaks():
    """Per mask the fp4 16x16 engine issues, over its 4 waves, 64 + 128 + 128
    instructions a wave: 256 v_mfma_scale_f32_16x16x128_f8f6f4 (2*16*16*128
    flops) and 512 v_mfma_f32_16x16x32_f16 (2*16*16*32 flops).  At the
    published dense peaks each takes 16 cycles on one of the 1,024 SIMDs at
    2.4 GHz, the rate measured for both on gfx950."""
    mf = dict((fl, (cnt, pk)) for cnt, fl, pk in bench.KERNELS[3]["mfma"])
    assert mf[2 * 16 * 16 * 128][0] == 4 * 64
    assert mf[2 * 16 * 16 * 32][0] == 4 * 128
    simd_hz = 256 * 4 * 2.4e9
    for fl, (cnt, pk) in mf.items():
        cycles = fl / (pk * 1e12 / simd_hz)
        assert abs(cycles - 16) < 0.25, (fl, cycles)
    assert bench.PEAK_FP16_MFMA_TFLOPS == 2500 and bench.PEAK_FP4_MFMA_TFLOPS == 10100
    assert bench.PEAK_HBM_GBS == 8000
