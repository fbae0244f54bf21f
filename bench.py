"""Benchmark: branch-free multicomponent GEMM on one MI355X.

Headline workload: square QD GEMM, m = n = k = 2048, entries generated as in
the seeded uniform recipe (leading component U[-1, 1), lower components
scaled by 2^-53 u and made non-overlapping).  One step = one C = A B.
Throughput is reported in multicomponent operations per second
(2 m n k: one BF multiply and one BF add per multiply-add) and as a fraction
of the FP64 vector issue peak (each BF op is a fixed count of FP64 VALU
instructions: QD multiply-add = 209).

Printed JSON line (one): metric/value/unit, ms_per_step, roofline of the
GEMM kernel (HIP-event timing on the launch stream), the CPU oracle timed on
a bounded row sample of the same product, and secondary rows (TD / DD / FF
GEMM at 2048) for context.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP64 VALU instructions per multiply-add (BF mul + BF add), from Tables 1-2
# and the double-word algorithms: DD 9 + 20, TD 39 + 57, QD 106 + 103.
INSTR_PER_MAC = {"dd": 29, "td": 96, "qd": 209, "ff": 29}
PEAK_ISSUE_TOPS = 256 * 64 * 2.4e9 / 1e12       # FP64 (and non-packed FP32) lane-ops/s: 39.3 T
METRIC = "TD/QD GEMM mp-op/s & % FP64 peak; Ozaki-MFMA vs branch-free DD at equal error"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--prec", default="qd")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary precisions")
    return ap.parse_args()


def time_gemm(mpx, torch, p, n, steps, warmup, seed_base):
    from paper_2603_14926_amd import synth
    dt = np.float32 if p == "ff" else np.float64
    K = mpx.ncomp(p)
    A = torch.from_numpy(synth.mp_array(K, (n, n), synth.seed_for(1, seed_base), "U", dtype=dt)).cuda()
    B = torch.from_numpy(synth.mp_array(K, (n, n), synth.seed_for(1, seed_base + 1), "U", dtype=dt)).cuda()
    Cm = torch.empty_like(A)
    mpx.gemm_autotune(p, A, B, Cm, reps=1)
    for _ in range(warmup):
        mpx.gemm(p, A, B, out=Cm)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        mpx.gemm(p, A, B, out=Cm)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_kernel = e0.elapsed_time(e1) / steps
    return ms_kernel, wall / steps * 1e3, (A, B, Cm)


def cpu_baseline(p, n, target_s=12.0):
    """The CPU oracle (sequential triple loop per entry) on a row sample of
    the same n x n x n product, OpenMP over rows, timed on the host."""
    import oracle
    from paper_2603_14926_amd import synth
    K = {"dd": 2, "td": 3, "qd": 4}[p]
    A = synth.mp_array(K, (n, n), synth.seed_for(1, 0), "U")
    B = synth.mp_array(K, (n, n), synth.seed_for(1, 1), "U")
    threads = min(os.cpu_count() or 1, 16)
    oracle.set_threads(threads)
    rows = max(threads, 2)
    t0 = time.perf_counter()
    oracle.gemm(K, A[:, :rows, :], B)
    dt = time.perf_counter() - t0
    # grow the sample to roughly target_s of work
    scale = max(1, int(target_s / max(dt, 1e-3)))
    rows2 = min(n, rows * scale)
    rows2 = max(threads, (rows2 // threads) * threads)
    t0 = time.perf_counter()
    oracle.gemm(K, A[:, :rows2, :], B)
    dt = time.perf_counter() - t0
    macs = rows2 * n * n
    return {
        "value": 2.0 * macs / dt,
        "unit": "mp-op/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{p.upper()} GEMM rows 0..{rows2 - 1} of the {n}x{n}x{n} product "
                  f"({rows2}x{n}x{n} multiply-adds, {dt:.1f} s)",
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the kernels are "
              f"single-GPU and no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2603_14926_amd import mpx
    mpx.lib()
    p, n = args.prec, args.n
    ms, wall_ms, _ = time_gemm(mpx, torch, p, n, args.steps, args.warmup, 0)
    macs = float(n) ** 3
    value = 2.0 * macs / (ms * 1e-3)
    achieved = macs * INSTR_PER_MAC[p] / (ms * 1e-3) / 1e12
    flops_per_mac = {"dd": 30, "td": 99, "qd": 215, "ff": 30}[p]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "mp-op/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "wall_ms_per_step": wall_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if p == "ff" else "f64",
        "data": "synthetic (seeded SplitMix64, uniform leading component)",
        "config": {"workload": f"{p}_gemm_{n}", "precision": p.upper(), "m": n, "n": n, "k": n,
                   "variant": "autotuned"},
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_ISSUE_TOPS,
            "unit": "TOP/s (FP64 VALU lane-instructions)",
            "frac": achieved / PEAK_ISSUE_TOPS,
            "frac_fp64_flop_peak": macs * flops_per_mac / (ms * 1e-3) / 78.6e12,
            "traffic": None,
        },
    }
    if not args.no_extra:
        rows = {}
        for q in ("td", "dd", "ff"):
            if q == p:
                continue
            qms, _, _ = time_gemm(mpx, torch, q, n, max(3, args.steps // 2), 1, 10)
            rows[q] = {"ms": qms, "mp_op_s": 2.0 * macs / (qms * 1e-3),
                       "frac_issue_peak": macs * INSTR_PER_MAC[q] / (qms * 1e-3) / 1e12 / PEAK_ISSUE_TOPS}
        out["other_precisions_gemm_2048"] = rows
    if not args.no_cpu and p != "ff":
        out["cpu_baseline"] = cpu_baseline(p, n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
