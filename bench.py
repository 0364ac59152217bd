"""Benchmark: fused Walsh spectrum + nonlinearity of a 16x16 S-box on one MI355X.

One step = one pass of the whole path over the 16x16 random-permutation
S-box (65,535 nonzero output masks x a 65,536-point transform each, fused
max |W| per mask and NL, no spectrum stored): bit-slicing of the table,
initialisation, and the fused transform kernel.  The table, outputs and
workspace are resident in HBM before timing starts.

Prints one JSON line (rank 0, N = 1) with the throughput in Walsh
coefficients per second, the roofline of the dominant kernel and the CPU
oracle's rate on a bounded sample of the same workload.  Unless --quick is
given, the line also carries the batched workload (4096 uneven boxes in one
planned launch against a loop of single-box calls) and the other workloads
(each with its own roofline fraction) under "batched" and "extra".
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 3.93e13 32-bit VALU lane-ops/s;
# packed 16-bit ops (v_pk_add_u16 ...) do two element-ops per lane-op.
PEAK_INT32_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
PEAK_PK16_TOPS = 2 * PEAK_INT32_TOPS
# Published dense fp16 matrix-core peak of the MI355X (no sparsity).
PEAK_FP16_MFMA_TFLOPS = 2500.0
# One v_mfma_f32_16x16x32_f16 is 16 x 16 x 32 multiply-adds (16,384 flops);
# at the published peak a SIMD retires one every 16 cycles.  Applied as half
# of H_32 to 16 rows it does the work of 16 x 16 x 5 = 1,280 butterfly
# add/subs, so the matrix cores run at most 1.966e14 butterfly ops/s.
MFMA_F16_FLOPS = 16 * 16 * 32 * 2
PEAK_MFMA_BUTTERFLY_TOPS = 256 * 4 * 2.4e9 / 16 * 1280 / 1e12
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=100, help="untimed steps first")
    ap.add_argument("--warmup-ms", type=float, default=60.0,
                    help="keep warming up until this much time has passed (the clocks ramp up over ~20 ms)")
    ap.add_argument("--cpu-sample-masks", type=int, default=32768,
                    help="masks of the 16x16 box the CPU oracle is timed on")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--paper-cpu-16", action="store_true",
                    help="also rerun the paper's CPU methods at 16x16 (16 GiB matrices; minutes)")
    ap.add_argument("--quick", action="store_true", help="the headline workload only (no batch, no extras)")
    ap.add_argument("--batched", action="store_true", help="time the mixed 4096-box batch (default unless --quick)")
    ap.add_argument("--serving", action="store_true",
                    help="the full Poisson serving sweep (1k-50k req/s); without it three rates run unless --quick")
    ap.add_argument("--serving-count", type=int, default=2000, help="requests per rate in the sweep")
    ap.add_argument("--extra", action="store_true",  # default unless --quick
                    help="also time the other workloads (8x8, 20x16, 16x20, 12x12 slice, 16x16 spectrum)")
    ap.add_argument("--variant", type=int, default=0, choices=(0, 1, 2, 3, 4),
                    help="butterfly engine for the 16x16 kernel: 0 library default, 1 VALU, 2 matrix cores "
                         "after popcount stages, 3 fp4 + fp16 matrix-core passes; with --batched-only or "
                         "--extra-only it applies to the batch's plan and the 12x12 fused call, where 4 "
                         "(int8 + fp16 passes, n = 12 only) is accepted too")
    ap.add_argument("--rounds", type=int, default=0, choices=(0, 4, 8),
                    help="with --variant 3: LDS exchange rounds per mask (0: library default)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (reference for HBM byte counters) and exit")
    ap.add_argument("--batched-only", action="store_true",
                    help="time only the 4096-box batch (for a profiler run), print it as one JSON object and exit")
    ap.add_argument("--no-plain-loop", action="store_true",
                    help="with --batched-only: time the graph replays only, not the loop of single-box calls")
    ap.add_argument("--extra-only", default="",
                    help="comma-separated name prefixes: time only those extra workloads (e.g. criteria_16x16, "
                         "for a profiler run), print them as one JSON object and exit")
    args = ap.parse_args()
    if not args.quick:
        args.batched = args.extra = True
    return args


# The fused 16x16 kernel each butterfly engine launches, the file holding its
# rocprofv3 FETCH_SIZE / WRITE_SIZE figures, the arithmetic type and the
# roofline it is reported against.  Packed int16 butterflies run on the VALU
# (peak: packed 16-bit lane-ops).  The matrix-core engines are exact (every
# operand an integer of at most 2^11, or a table bit, fp32 accumulation);
# their peak is the published dense fp16 matrix-core rate (variant 3 runs
# a third of its MFMAs on fp4 operands, whose own peak is four times
# higher, so the fp16 figure is the stricter one).  "mfma" lists, per mask,
# (instructions, flops each, published peak of their type in TFLOP/s).
PEAK_FP4_MFMA_TFLOPS = 10100.0
KERNELS = {1: {"kernel": "k_walsh<16,8,0>", "traffic": "k_walsh_16x16_traffic.json", "dtype": "i16",
               "bound": "alu", "peak": PEAK_PK16_TOPS, "unit": "TOP/s", "mfma": []},
           2: {"kernel": "k_walsh_mfma16<4>", "traffic": "k_walsh_mfma16_16x16_traffic.json", "dtype": "f16",
               "bound": "mfma", "peak": PEAK_FP16_MFMA_TFLOPS, "unit": "TFLOP/s",
               "mfma": [(512, MFMA_F16_FLOPS, PEAK_FP16_MFMA_TFLOPS)]},
           3: {"kernel": "k_walsh_mx16", "traffic": "k_walsh_mx16_16x16_traffic.json", "dtype": "fp4+f16",
               "bound": "mfma", "peak": PEAK_FP16_MFMA_TFLOPS, "unit": "TFLOP/s",
               "mfma": [(256, 16 * 16 * 128 * 2, PEAK_FP4_MFMA_TFLOPS),
                        (512, MFMA_F16_FLOPS, PEAK_FP16_MFMA_TFLOPS)]}}
# The paper's own figures (Table 4, Fig. ch2; one Core i7 of 12 threads, 16 GB
# DDR4, Windows 10, MSVC 2017, Table 3), quoted as context only.
PAPER_CONTEXT = {
    "hardware": "Intel Core i7 8400K, 12 threads (as printed), 16 GB DDR4, Windows 10 x64, MSVC 2017 (Table 3)",
    "walsh_speedup_16x16": 39.784, "nl_speedup_16x16": 563.05,
    "fwht_16x16_ms": {"primary": 2496726, "a_transposed": 326331, "b_10_threads": 62756, "c_fused_nl": 83013},
    "nl_16x16_ms": {"primary": 46741627, "a_transposed": 539120, "b_10_threads": 539120, "c_fused_nl": 83015},
}
DEFAULT_VARIANT = 3
# Where each kernel's source starts and which function ends it: the counters
# stay valid while the shared definitions before the first kernel and this
# section are unchanged.
KERNEL_SECTIONS = {1: ("// Main fused kernel", "void k_walsh(const KParams kp)"),
                   2: ("// n = 16, max mode, matrix-core variant.", "void k_walsh_mfma16(const KParams kp)"),
                   3: ("// n = 16, max mode, three matrix-core passes", "void k_walsh_mx16(const KParams kp)")}


def kernel_source_digest(variant):
    """SHA-256 (16 hex digits) of the shared prefix of walsh_kernels.hpp and
    of the section holding the kernel of this engine."""
    import hashlib
    with open(os.path.join(ROOT, "paper_1912_03732_amd", "csrc", "walsh_kernels.hpp")) as f:
        text = f.read()
    start, func = KERNEL_SECTIONS[variant]
    prefix = text[:text.index("// Main fused kernel")]
    i = text.index(start)
    j = text.index("\n}\n", text.index(func, i)) + 3
    return hashlib.sha256((prefix + text[i:j]).encode()).hexdigest()[:16]


def measured_traffic(fname, variant):
    """HBM bytes per dispatch of the fused 16x16 kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs, or None if the kernel's source has
    changed since they were taken."""
    try:
        with open(os.path.join(ROOT, "profiles", fname)) as f:
            rec = json.load(f)
        digest = kernel_source_digest(variant)
    except (OSError, ValueError):
        return None
    return rec["traffic_bytes_per_dispatch"] if rec.get("kernel_source_sha256_16") == digest else None


def host_cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(S, n, m, sample_masks, runs=3):
    """The oracle on the host: all usable cores (threads over masks, the
    paper's partition of the masks among threads), the median of `runs`
    runs, then one core on a sixteenth of the sample."""
    import numpy as np
    import oracle
    cores = host_cores()
    masks = np.arange(1, min(sample_masks, (1 << m) - 1) + 1, dtype=np.uint32)
    oracle.maxabs_for_masks(S, n, m, masks[:64], nthreads=cores)  # load + warm
    times = []
    for _ in range(runs):
        t0 = time.perf_counter()
        oracle.maxabs_for_masks(S, n, m, masks, nthreads=cores)
        times.append(time.perf_counter() - t0)
    dt = sorted(times)[len(times) // 2]
    one = masks[:max(1, masks.size // 16)]
    t0 = time.perf_counter()
    oracle.maxabs_for_masks(S, n, m, one, nthreads=1)
    dt1 = time.perf_counter() - t0
    return {"value": masks.size * (1 << n) / dt, "unit": "coeff/s", "cores": cores, "kind": "oracle",
            "sample": "masks b=1..%d of the same %dx%d box, median of %d runs (%s s wall on %d threads)"
                      % (masks.size, n, m, runs, ", ".join("%.2f" % t for t in times), cores),
            "single_core": {"value": one.size * (1 << n) / dt1, "unit": "coeff/s",
                            "sample": "masks b=1..%d on 1 thread (%.1f s wall)" % (one.size, dt1)},
            "cpu_model": host_cpu_model()}


def paper_table4(sizes=((10, 10), (12, 12)), sweep_size=(12, 12), sweep=range(7, 13), threads=10):
    """The paper's CPU methods (Table 4, Fig. ch1) rerun on this host with the
    oracle's routines, as a historical baseline:
      primary: the a-major matrix of Algorithm 1 on one thread, then the
               unfused NL scan of Algorithm 2;
      (a)      the transposed (b-major) matrix of Section 5.1, one thread;
      (b)      (a) with the masks split among `threads` threads (Alg. 4);
      (c)      (b) with the maximum folded into the transform (Alg. 5), no matrix.
    'fwht_ms' is the matrix (or fused pass) time, 'nl_ms' the scan after it;
    the sweep repeats (b) over the paper's 7..12 threads.  Seeded permutations."""
    import numpy as np
    import oracle
    from paper_1912_03732_amd import inputs

    def timed(fn):
        t0 = time.perf_counter()
        r = fn()
        return (time.perf_counter() - t0) * 1e3, r

    out = {}
    for n, m in sizes:
        S = inputs.permutation(n, inputs.rng(inputs.SEED_BASE + 10 + n))
        row = {}
        for name, layout, nt in (("primary", oracle.A_MAJOR, 1), ("a_transposed", oracle.B_MAJOR, 1),
                                 ("b_threads", oracle.B_MAJOR, threads)):
            t_w, W = timed(lambda: oracle.spectrum(S, n, m, layout, nthreads=nt))
            t_n, (nl, _) = timed(lambda: oracle.nl_from_spectrum(W, n, m, layout, nthreads=nt))
            row[name] = {"fwht_ms": t_w, "nl_ms": t_n, "nl": nl, "threads": nt}
            del W
        t_c, (nl, _) = timed(lambda: oracle.walsh_nl(S, n, m, nthreads=threads))
        row["c_fused"] = {"fwht_ms": t_c, "nl_ms": t_c, "nl": nl, "threads": threads}
        out["%dx%d" % (n, m)] = row
    n, m = sweep_size
    S = inputs.permutation(n, inputs.rng(inputs.SEED_BASE + 10 + n))
    sw = {}
    for nt in sweep:
        t_w, W = timed(lambda: oracle.spectrum(S, n, m, oracle.B_MAJOR, nthreads=nt))
        sw[str(nt)] = t_w
        del W
    out["thread_sweep_b_%dx%d_fwht_ms" % (n, m)] = sw
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the Walsh/NL path is built and timed on a single "
              "MI355X (sharding the masks over several GPUs is described, not implemented)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_1912_03732_amd import binding as B
    from paper_1912_03732_amd import inputs

    if args.copy_calibration:
        copy_calibration(torch)
        return
    side_tuning = B.sbox_tuning(0, 0, 0, args.variant) if args.variant else None
    if args.batched_only:
        dev = torch.device("cuda:0")
        torch.cuda.set_device(dev)
        print(json.dumps({"batched": bench_batched(torch, B, inputs, dev, plain_loop=not args.no_plain_loop,
                                                   tuning=side_tuning)}), flush=True)
        return
    if args.extra_only:
        dev = torch.device("cuda:0")
        torch.cuda.set_device(dev)
        only = tuple(p for p in args.extra_only.split(",") if p)
        print(json.dumps({"extra": bench_extra(torch, B, inputs, dev, only, tuning12=side_tuning)}), flush=True)
        return
    if args.variant == 4:
        raise SystemExit("--variant 4 (int8 first pass) covers n = 12 only: use it with --batched-only or "
                         "--extra-only 12x12_perm_fused")
    n = m = 16
    w = inputs.workload_16x16()
    S_host = w["perm"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    S = B.table_to_device(S_host, m, device=dev)
    nl = torch.empty(1, dtype=torch.int32, device=dev)
    mx = torch.empty(1 << m, dtype=torch.int32, device=dev)
    ws = B.Workspace(B.sbox_walsh_nl_workspace_bytes(n, m, 0), dev)
    stream = torch.cuda.current_stream(dev)
    sptr = int(stream.cuda_stream)

    tuning = B.sbox_tuning(args.rounds, 0, 0, args.variant) if args.variant else None
    variant = args.variant or DEFAULT_VARIANT
    kinfo = KERNELS[variant]

    def step():
        st = B.sbox_walsh_nl_ex(S.data_ptr(), n, m, 2, mx.data_ptr(), nl.data_ptr(), 0, 0,
                                ws.ptr, ws.nbytes, tuning, sptr)
        if st != 0:
            raise RuntimeError(B.last_error())

    # untimed warm-up: the requested steps, continued until at least
    # --warmup-ms of work has run (the clocks ramp up over the first ~20 ms)
    t_w = time.perf_counter()
    done = 0
    while done < args.warmup or (time.perf_counter() - t_w) * 1e3 < args.warmup_ms:
        for _ in range(10):
            step()
        done += 10
        torch.cuda.synchronize(dev)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        step()
        b.record(stream)
    torch.cuda.synchronize(dev)
    t1 = time.perf_counter()
    nl_val = int(nl.item())
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    ev_ms = sorted(a.elapsed_time(b) for a, b in ev)
    ev_mean = sum(ev_ms) / len(ev_ms)
    coeffs = (1 << n) * ((1 << m) - 1)
    ops = n * coeffs  # Table 1: n add/sub per coefficient
    value = coeffs / (ms_per_step * 1e-3)
    achieved_tops = ops / (ev_mean * 1e-3) / 1e12
    masks = (1 << m) - 1
    roof = {"bound": kinfo["bound"], "achieved": achieved_tops, "peak": kinfo["peak"], "unit": kinfo["unit"],
            "frac": achieved_tops / kinfo["peak"], "traffic": measured_traffic(kinfo["traffic"], variant),
            "kernel": kinfo["kernel"], "event_ms_per_step": ev_mean,
            "achieved_is": "algorithmic add/sub of the transform (n per coefficient) per second",
            "int32_valu_peak": PEAK_INT32_TOPS, "int32_valu_frac": achieved_tops / PEAK_INT32_TOPS,
            "pk16_valu_peak": PEAK_PK16_TOPS, "pk16_valu_frac": achieved_tops / PEAK_PK16_TOPS}
    if kinfo["mfma"]:
        # the matrix cores' own utilisation: issued flops of each type against its peak
        sec = ev_mean * 1e-3
        issued = sum(cnt * fl * masks for cnt, fl, _ in kinfo["mfma"]) / sec / 1e12
        busy = sum(cnt * fl * masks / (pk * 1e12) for cnt, fl, pk in kinfo["mfma"]) / sec
        roof.update({"mfma_issued_tflops": issued, "mfma_issued_frac": busy,
                     "mfma_per_mask": [[cnt, fl] for cnt, fl, _ in kinfo["mfma"]],
                     "mfma_butterfly_peak": PEAK_MFMA_BUTTERFLY_TOPS,
                     "mfma_butterfly_frac": achieved_tops / PEAK_MFMA_BUTTERFLY_TOPS})

    out = {
        "metric": "Walsh coefficients/s, fused NL of a 16x16 S-box (65,535 masks x 65,536-point FWHT)",
        "value": value,
        "unit": "coeff/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": done,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": kinfo["dtype"],
        "data": "synthetic",
        "config": {"workload": "single 16x16 S-box, seeded Fisher-Yates permutation (seed %d), fused "
                               "max|W| per mask + NL, no spectrum" % (inputs.SEED_BASE + 2),
                   "n": n, "m": m, "masks": masks, "nl": nl_val},
        "roofline": roof,
        "paper_context": dict(PAPER_CONTEXT, speedup_vs_paper_best_fused_nl=PAPER_CONTEXT["nl_16x16_ms"]["c_fused_nl"]
                              / ms_per_step),
    }
    if args.batched:
        out["batched"] = bench_batched(torch, B, inputs, dev)
    if args.extra:
        out["extra"] = bench_extra(torch, B, inputs, dev)
    if args.serving or not args.quick:
        from paper_1912_03732_amd import serving
        rates = (1000, 2000, 5000, 10000, 20000, 50000) if args.serving else (2000, 10000, 30000)
        out["serving"] = serving.sweep(rates=rates, count=args.serving_count)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(S_host, n, m, args.cpu_sample_masks)
        big = ((10, 10), (12, 12), (16, 16)) if args.paper_cpu_16 else ((10, 10), (12, 12))
        out["cpu_baseline"]["paper_table4"] = paper_table4(
            sizes=big, sweep_size=(16, 16) if args.paper_cpu_16 else (12, 12))
    print(json.dumps(out), flush=True)


def copy_calibration(torch, nbytes=1 << 30, reps=3):
    """A plain device-to-device copy of known size: the reference that scales
    the FETCH_SIZE / WRITE_SIZE counters into bytes."""
    src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)


def _time_call(torch, fn, reps, warm_ms=30.0):
    """Mean ms per call over `reps` calls, after at least `warm_ms` of
    untimed calls (the clocks ramp up over tens of milliseconds)."""
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < warm_ms:
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(s)
    for _ in range(reps):
        fn()
    b.record(s)
    b.synchronize()
    return a.elapsed_time(b) / reps


def bench_extra(torch, B, inputs, dev, only=(), tuning12=None):
    """The other workloads, timed with HIP events (ms per call); `only`
    (name prefixes) restricts them; `tuning12` applies to the 12x12 fused call."""
    out = {}

    def want(name):
        return not only or any(name.startswith(p) for p in only)

    def single(S_host, n, m, layout=0, reps=5, tuning=None):
        S = B.table_to_device(S_host, m, device=dev)
        nl = torch.empty(1, dtype=torch.int32, device=dev)
        mx = torch.empty(1 << m, dtype=torch.int32, device=dev)
        spec = torch.empty(1 << (n + m), dtype=torch.int32, device=dev) if layout else None
        ws = B.Workspace(B.sbox_walsh_nl_workspace_bytes(n, m, layout), dev)
        sptr = int(torch.cuda.current_stream(dev).cuda_stream)

        def call():
            st = B.sbox_walsh_nl_ex(S.data_ptr(), n, m, S.element_size(), mx.data_ptr(), nl.data_ptr(),
                                    spec.data_ptr() if spec is not None else 0, layout, ws.ptr, ws.nbytes,
                                    tuning, sptr)
            if st != 0:
                raise RuntimeError(B.last_error())
        ms = _time_call(torch, call, reps)
        coeffs = (1 << n) * ((1 << m) - 1)
        row = {"ms": ms, "coeff_per_s": coeffs / (ms * 1e-3), "int_ops_per_s": n * coeffs / (ms * 1e-3),
               "nl": int(nl.item())}
        if layout:
            # a stored spectrum makes the call HBM-bound: 4 bytes per coefficient
            gbs = 4 * (1 << (n + m)) / (ms * 1e-3) / 1e9
            row["spectrum_GB_per_s"] = gbs
            row["roofline"] = {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                               "frac": gbs / PEAK_HBM_GBS}
        else:
            # n = 12, 16: the matrix-core engines (published dense fp16 peak);
            # other n: packed 16-bit VALU butterflies (the last stages of
            # n > 16 run in int32; the packed peak is the stricter one)
            tops = n * coeffs / (ms * 1e-3) / 1e12
            if n in (12, 16):
                row["roofline"] = {"bound": "mfma", "achieved": tops, "peak": PEAK_FP16_MFMA_TFLOPS,
                                   "unit": "TFLOP/s", "frac": tops / PEAK_FP16_MFMA_TFLOPS,
                                   "mfma_butterfly_frac": tops / PEAK_MFMA_BUTTERFLY_TOPS}
            else:
                row["roofline"] = {"bound": "alu", "achieved": tops, "peak": PEAK_PK16_TOPS, "unit": "TOP/s",
                                   "frac": tops / PEAK_PK16_TOPS}
        return row

    w8 = inputs.workload_8x8()
    ns = inputs.workload_nonsquare()
    singles = [("8x8_perm_fused", lambda: single(w8["perm"], 8, 8, reps=50)),
               ("8x8_perm_spectrum_b", lambda: single(w8["perm"], 8, 8, 1, reps=50)),
               ("8x8_perm_spectrum_a", lambda: single(w8["perm"], 8, 8, 2, reps=50)),
               ("12x12_perm_fused", lambda: single(inputs.permutation(12, inputs.rng(inputs.SEED_BASE + 6)), 12, 12,
                                                   reps=50, tuning=tuning12)),
               # n = 12 engine comparison at scale (2^20 masks): the fp4 (default) or, with
               # --variant 4, the int8 first pass
               ("12x20_fused", lambda: single(inputs.random_function(12, 20, inputs.rng(inputs.SEED_BASE + 11)), 12,
                                              20, reps=10, tuning=tuning12)),
               ("16x20_fused", lambda: single(ns["s16x20"], 16, 20, reps=2)),
               ("20x16_fused", lambda: single(ns["s20x16"], 20, 16, reps=1)),
               ("12x12_slice_spectrum_a", lambda: single(ns["slice12"], 12, 12, 2, reps=10)),
               ("12x12_slice_spectrum_b", lambda: single(ns["slice12"], 12, 12, 1, reps=10)),
               ("16x16_perm_spectrum_b", lambda: single(inputs.workload_16x16()["perm"], 16, 16, 1, reps=2)),
               ("16x16_perm_spectrum_a", lambda: single(inputs.workload_16x16()["perm"], 16, 16, 2, reps=2))]
    for name, run in singles:
        if want(name):
            out[name] = run()
    # component criteria (balancedness, correlation immunity, autocorrelation): two
    # int32 transforms per mask, register-blocked
    for n in (8, 12, 14, 16):
        if not want("criteria_%dx%d" % (n, n)):
            continue
        S = B.table_to_device(inputs.permutation(n, inputs.rng(inputs.SEED_BASE + 6)), n, device=dev)
        summ = torch.empty(8, dtype=torch.int32, device=dev)
        sptr = int(torch.cuda.current_stream(dev).cuda_stream)
        cws = B.Workspace(B.sbox_criteria_workspace_bytes(n, n), dev)

        def crit():
            st = B.sbox_criteria_ex(S.data_ptr(), n, n, S.element_size(), summ.data_ptr(), 0, 0, 0, 0, cws.ptr,
                                    cws.nbytes, sptr)
            if st != 0:
                raise RuntimeError(B.last_error())
        ms = _time_call(torch, crit, 1 if n == 16 else (3 if n == 14 else 10))
        coeffs = (1 << n) * ((1 << n) - 1)
        tops = 2 * n * coeffs / (ms * 1e-3) / 1e12
        out["criteria_%dx%d" % (n, n)] = {"ms": ms, "coeff_per_s": coeffs / (ms * 1e-3),
                                          "int_ops_per_s": 2 * n * coeffs / (ms * 1e-3),
                                          "summary": summ.cpu().tolist()[:6],
                                          # two int32 transforms (n 2^n add/sub each) per mask
                                          "roofline": {"bound": "alu", "achieved": tops, "peak": PEAK_INT32_TOPS,
                                                       "unit": "TOP/s", "frac": tops / PEAK_INT32_TOPS}}
    # |W| histogram over all nonzero masks (fused into the transform)
    for name, S_host, n in (("8x8_perm", w8["perm"], 8), ("16x16_perm", inputs.workload_16x16()["perm"], 16)):
        if not want("histogram_" + name):
            continue
        S = B.table_to_device(S_host, n, device=dev)
        hist = torch.empty((1 << (n - 1)) + 1, dtype=torch.int64, device=dev)
        nl = torch.empty(1, dtype=torch.int32, device=dev)
        ws = B.Workspace(B.sbox_walsh_histogram_workspace_bytes(n, n), dev)
        sptr = int(torch.cuda.current_stream(dev).cuda_stream)

        def hcall():
            st = B.sbox_walsh_histogram(S.data_ptr(), n, n, S.element_size(), hist.data_ptr(), 0, nl.data_ptr(),
                                        ws.ptr, ws.nbytes, sptr)
            if st != 0:
                raise RuntimeError(B.last_error())
        ms = _time_call(torch, hcall, 3 if n == 16 else 20)
        coeffs = (1 << n) * ((1 << n) - 1)
        h = hist.cpu()
        tops = n * coeffs / (ms * 1e-3) / 1e12
        out["histogram_%s" % name] = {"ms": ms, "coeff_per_s": coeffs / (ms * 1e-3), "nl": int(nl.item()),
                                      "max_bin": int(torch.nonzero(h).max()),
                                      # the packed-int16 store-mode transform plus one LDS count per value
                                      "roofline": {"bound": "alu", "achieved": tops, "peak": PEAK_PK16_TOPS,
                                                   "unit": "TOP/s", "frac": tops / PEAK_PK16_TOPS}}
    # unit-difference autocorrelations (strict avalanche / bit independence)
    for name, S_host, n in (("8x8_perm", w8["perm"], 8), ("16x16_perm", inputs.workload_16x16()["perm"], 16)):
        if not want("avalanche_" + name):
            continue
        S = B.table_to_device(S_host, n, device=dev)
        r = torch.empty(n << n, dtype=torch.int32, device=dev)
        summ = torch.empty(3, dtype=torch.int32, device=dev)
        sptr = int(torch.cuda.current_stream(dev).cuda_stream)

        def acall():
            st = B.sbox_avalanche(S.data_ptr(), n, n, S.element_size(), r.data_ptr(), summ.data_ptr(), 0, 0, 0,
                                  sptr)
            if st != 0:
                raise RuntimeError(B.last_error())
        ms = _time_call(torch, acall, 20)
        out["avalanche_%s" % name] = {"ms": ms, "summary": summ.cpu().tolist()}
    return out


def bench_batched(torch, B, inputs, dev, reps=5, plain_loop=True, tuning=None):
    """4096 mixed boxes (n = m in {6,8,10,12}): one planned batched launch vs a
    loop of single-box calls on one stream."""
    batch = inputs.workload_batched()
    tabs = [B.table_to_device(S, n, device=dev) for n, S in batch]
    ns = [n for n, _ in batch]
    plan = B.Plan(tabs, ns, ns, tuning=tuning)
    stream = torch.cuda.current_stream(dev)
    plan.launch()
    torch.cuda.synchronize(dev)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch()
    g.replay()
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()  # untimed replays for at least 30 ms: the clocks ramp up first
    while time.perf_counter() - t0 < 0.03:
        g.replay()
        torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize(dev)
    t_batch = (time.perf_counter() - t0) / reps
    coeffs = sum((1 << n) * ((1 << n) - 1) for n in ns)
    if not plain_loop:
        plan.close()
        return {"boxes": len(batch), "sboxes_per_s": len(batch) / t_batch, "ms": t_batch * 1e3,
                "coeff_per_s": coeffs / t_batch}
    # plain loop: one sbox_walsh_nl_ex per box
    nl = torch.empty(1, dtype=torch.int32, device=dev)
    outs = [torch.empty(1 << n, dtype=torch.int32, device=dev) for n in ns]
    ws = B.Workspace(max(B.sbox_walsh_nl_workspace_bytes(n, n, 0) for n in ns), dev)
    sptr = int(stream.cuda_stream)

    def loop():
        for t, n, o in zip(tabs, ns, outs):
            B.sbox_walsh_nl_ex(t.data_ptr(), n, n, t.element_size(), o.data_ptr(), nl.data_ptr(), 0, 0,
                               ws.ptr, ws.nbytes, None, sptr)
    loop()
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    loop()
    torch.cuda.synchronize(dev)
    t_loop = time.perf_counter() - t0
    plan.close()
    return {"boxes": len(batch), "sboxes_per_s": len(batch) / t_batch, "ms": t_batch * 1e3,
            "coeff_per_s": coeffs / t_batch, "plain_loop_ms": t_loop * 1e3,
            "plain_loop_sboxes_per_s": len(batch) / t_loop, "speedup_vs_plain_loop": t_loop / t_batch}


if __name__ == "__main__":
    main()
