"""Benchmark of the branch-free multicomponent kernels on one MI355X.

Headline (the `value` of the JSON line): square QD GEMM, m = n = k = 2048,
seeded uniform inputs (leading component U[-1, 1), lower components the
previous one times 2^-53 u, made non-overlapping).  One step = one C = A B.
Throughput in multicomponent operations per second (2 m n k: one BF multiply
and one BF add per multiply-add), and as a fraction of the FP64 VALU issue
peak (a QD multiply-add is 209 FP64 VALU instructions; peak = 256 CUs x 64
lanes x 2.4 GHz = 39.3 T lane-instructions/s).  The kernel time comes from
HIP events recorded on the stream the kernel is launched on.

The same line carries, under "rows", the other rows of the hot path, each
measured on its own synthetic workload:
  gemm          DD / TD / QD at 512, 1024, 2048 and FF at 2048;
  gemv          n = 8192 (QD, TD, DD);
  vector        AXPY and dot at n = 4096 (latency) and n = 2^24 (HBM);
  cgemm_3m      complex GEMM by the 3M method at n = 2048 and 2049;
  polyeval      Horner versus Estrin, batch 1024, degrees 16 .. 4095;
  durand_kerner 4096 complex QD polynomials, degrees 16..512, 200 sweeps
                in one graph-replayed persistent launch: roots/s, residual,
                error on 16 known-root polynomials;
  autograd      QD and DD GEMM 2048 forward + backward, Horner backward
                (degree 1024, batch 1024);
  ozaki         Ozaki-split DD GEMM on FP64 MFMA vs the branch-free DD GEMM
                at n = 4096 and 8192, phi = 1, 4, 8; slices chosen as the
                fewest meeting the DD bound n 2^-104 sum|ab| ("at_bound")
                and the BF DD GEMM's own measured error ("at_bf_error").
and "cpu_baseline": the CPU oracle on a bounded row sample of the headline
product.  --quick skips the rows.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP64 (FP32 for FF) VALU instructions per multiply-add: BF mul + BF add
# (Tables 1-2 and the double-word algorithms): DD 9 + 20, TD 39 + 57, QD 106 + 103.
INSTR_PER_MAC = {"dd": 29, "td": 96, "qd": 209, "ff": 29}
FLOP_PER_MAC = {"dd": 30, "td": 99, "qd": 215, "ff": 30}   # FMA counted as 2
PEAK_F64_ISSUE = 256 * 64 * 2.4e9            # 39.3e12 FP64 lane-instructions/s
PEAK_F32_ISSUE = 2 * PEAK_F64_ISSUE          # binary32 VALU issues at twice the FP64 rate
PEAK_F64_FLOP = 78.6e12
PEAK_MFMA_F64 = 78.6e12
PEAK_HBM = 8.0e12
METRIC = "TD/QD GEMM mp-op/s & % FP64 peak; Ozaki-MFMA vs branch-free DD at equal error"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=2048, help="headline GEMM size (and --only gemm's)")
    ap.add_argument("--prec", default="qd")
    ap.add_argument("--quick", action="store_true", help="headline only (no rows, no CPU baseline)")
    ap.add_argument("--no-8192", action="store_true", help="skip the n = 8192 Ozaki comparison")
    ap.add_argument("--only", default=None,
                    choices=["gemm", "gemv", "vector", "cgemm", "polyeval", "nobf", "strassen", "batched",
                             "durand_kerner", "autograd", "ozaki", "vector_sweep"],
                    help="measure one row only (skips the headline and the CPU baseline); "
                         "vector_sweep (n = 2^16 .. 2^26) runs only when named here")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--peak-probe", action="store_true",
                    help="measure the FP64 / FP32 VALU issue rates the rooflines use, print them, exit")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 512 MiB read + 512 MiB write kernel (counter calibration)")
    return ap.parse_args()


class Timer:
    """Median time per call (ms): untimed calls (at least `warmup`, and more
    until about `warm_s` seconds have passed: the engine clock ramps up over
    tens of milliseconds of sustained work, and a DD GEMM of a millisecond
    runs up to 25 % slower in its first calls after an idle spell), then
    `samples` samples, each the HIP-event time of `reps` back-to-back calls
    on the current stream divided by `reps` (reps > 1 only for calls of a
    few microseconds, where one event pair per call would dominate)."""

    def __init__(self, torch):
        self.torch = torch

    def __call__(self, fn, reps=1, samples=10, warmup=3, warm_s=0.1):
        torch = self.torch
        t0, i = time.perf_counter(), 0
        while i < warmup or time.perf_counter() - t0 < warm_s:
            fn()
            i += 1
            if i % 8 == 0:
                torch.cuda.synchronize()  # keep the host from running ahead of the GPU
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(samples)]
        for e0, e1 in ev:
            e0.record(s)
            for _ in range(reps):
                fn()
            e1.record(s)
        torch.cuda.synchronize()
        return float(np.median([e0.elapsed_time(e1) / reps for e0, e1 in ev]))


def measured_traffic(workload: str, tiling: str):
    """HBM bytes per launch of the headline GEMM kernel in the given tiling
    from the committed rocprofv3 counter summary (FETCH_SIZE, WRITE_SIZE,
    each scaled by the same counter on a copy kernel of known size; the
    counter runs autotune, so every tiling of the size is counted), or None
    when the summary is missing, is for another workload, lacks the tiling,
    or was taken on different kernel sources (SHA-256 prefix of the sources
    recorded with the counters)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{workload}_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    h = hashlib.sha256()
    for f in rec.get("sources", []):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != rec.get("source_sha256_16"):
        return None
    return rec.get("traffic_bytes_by_tiling", {}).get(tiling)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def gpu_mp(torch, K, shape, seed, dist="U", phi=4.0, dtype=np.float64):
    from paper_2603_14926_amd import synth
    return torch.from_numpy(synth.mp_array(K, shape, seed, dist, phi=phi, dtype=dtype)).cuda()


# ------------------------------------------------------------------ GEMM ----

def gemm_row(mpx, torch, T, p, n):
    dt = np.float32 if p == "ff" else np.float64
    K = mpx.ncomp(p)
    from paper_2603_14926_amd import synth
    A = gpu_mp(torch, K, (n, n), synth.seed_for(1, 0), dtype=dt)
    B = gpu_mp(torch, K, (n, n), synth.seed_for(1, 1), dtype=dt)
    Cm = torch.empty_like(A)
    # three calls per sample: single calls of the short products (FF, DD,
    # n <= 1024) ranked tilings a few percent apart in either order
    v, _ = mpx.gemm_autotune(p, A, B, Cm, reps=3)
    ms = T(lambda: mpx.gemm(p, A, B, out=Cm))
    macs = float(n) ** 3
    peak = PEAK_F32_ISSUE if p == "ff" else PEAK_F64_ISSUE
    return {"ms": ms, "mp_op_s": 2 * macs / (ms * 1e-3),
            "frac_issue_peak": macs * INSTR_PER_MAC[p] / (ms * 1e-3) / peak,
            "variant": mpx.gemm_variants(p)[v]}


def _oracle_gemm_rate(oracle, K, A, B, n, threads, target_s):
    """mp-op/s of the oracle's GEMM on `threads` threads over a row sample of
    A B sized for about target_s seconds; returns (rate, rows, seconds)."""
    oracle.set_threads(threads)
    rows = max(threads, 2)
    t0 = time.perf_counter()
    oracle.gemm(K, A[:, :rows, :], B)
    dt = time.perf_counter() - t0
    rows2 = min(n, rows * max(1, int(target_s / max(dt, 1e-3))))
    rows2 = max(threads, (rows2 // threads) * threads)
    t0 = time.perf_counter()
    oracle.gemm(K, A[:, :rows2, :], B)
    dt = time.perf_counter() - t0
    return 2.0 * rows2 * n * n / dt, rows2, dt


def cpu_baseline(p, n, target_s=12.0, target_1t_s=8.0):
    """The CPU oracle (sequential triple loop per entry) on a row sample of
    the same n x n x n product, OpenMP over rows, timed on the host with all
    cores (up to 16) and on one thread."""
    import oracle
    from paper_2603_14926_amd import synth
    K = {"dd": 2, "td": 3, "qd": 4}[p]
    A = synth.mp_array(K, (n, n), synth.seed_for(1, 0), "U")
    B = synth.mp_array(K, (n, n), synth.seed_for(1, 1), "U")
    threads = min(os.cpu_count() or 1, 16)
    v, rows, dt = _oracle_gemm_rate(oracle, K, A, B, n, threads, target_s)
    v1, rows1, dt1 = _oracle_gemm_rate(oracle, K, A, B, n, 1, target_1t_s)
    oracle.set_threads(threads)
    return {"value": v, "unit": "mp-op/s", "cores": threads, "kind": "oracle",
            "sample": f"{p.upper()} GEMM rows 0..{rows - 1} of the {n}x{n}x{n} product "
                      f"({rows}x{n}x{n} multiply-adds in {dt:.1f} s)",
            "single_thread": {"value": v1, "unit": "mp-op/s", "cores": 1,
                              "sample": f"{p.upper()} GEMM rows 0..{rows1 - 1} of the same product "
                                        f"({rows1}x{n}x{n} multiply-adds in {dt1:.1f} s)"}}


# -------------------------------------------------------- GEMV and vector ----

def gemv_rows(mpx, torch, T):
    from paper_2603_14926_amd import synth
    out = {}
    n = 8192
    A4 = gpu_mp(torch, 4, (n, n), synth.seed_for(1, 20))
    x4 = gpu_mp(torch, 4, n, synth.seed_for(1, 21))
    for p in ("qd", "td", "dd"):
        K = mpx.ncomp(p)
        A, x = A4[:K], x4[:K]      # the leading K components are a K-component input
        y = torch.empty((K, n), dtype=torch.float64, device="cuda")
        ws = mpx.workspace(mpx.OP_GEMV, p, n, n, 0)
        ms = T(lambda: mpx.gemv(p, A, x, out=y, ws=ws))
        macs = float(n) * n
        bytes_ = K * 8.0 * (n * n + 2 * n)
        out[p] = {"ms": ms, "mp_op_s": 2 * macs / (ms * 1e-3),
                  "GB_s": bytes_ / (ms * 1e-3) / 1e9, "frac_hbm_peak": bytes_ / (ms * 1e-3) / PEAK_HBM,
                  "frac_issue_peak": macs * INSTR_PER_MAC[p] / (ms * 1e-3) / PEAK_F64_ISSUE}
    del A4, x4
    return out


def vector_rows(mpx, torch, T):
    from paper_2603_14926_amd import synth
    out = {}
    for p in ("qd", "td", "dd"):
        K = mpx.ncomp(p)
        row = {}
        for n in (4096, 1 << 24):
            x = gpu_mp(torch, K, n, synth.seed_for(0, 1))
            y = gpu_mp(torch, K, n, synth.seed_for(0, 2))
            alpha = [0.75] + [0.0] * (K - 1)
            r = torch.empty(K, dtype=torch.float64, device="cuda")
            ws = mpx.workspace(mpx.OP_DOT, p, n)
            reps = 100 if n == 4096 else 1
            t_axpy = T(lambda: mpx.axpy(p, alpha, x, y), reps=reps)
            t_dot = T(lambda: mpx.dot(p, x, y, out=r, ws=ws), reps=reps)
            b_axpy, b_dot = 3 * K * 8.0 * n, 2 * K * 8.0 * n
            row[str(n)] = {
                "axpy_us": t_axpy * 1e3, "axpy_GB_s": b_axpy / (t_axpy * 1e-3) / 1e9,
                "axpy_frac_hbm": b_axpy / (t_axpy * 1e-3) / PEAK_HBM,
                "dot_us": t_dot * 1e3, "dot_GB_s": b_dot / (t_dot * 1e-3) / 1e9,
                "dot_frac_hbm": b_dot / (t_dot * 1e-3) / PEAK_HBM,
            }
            if n == 4096:
                # launch-bound size: the same calls captured 100 at a time in
                # one HIP graph and replayed (per-call time and calls/s)
                calls = 100
                for name, fn in (("axpy", lambda: mpx.axpy(p, alpha, x, y)),
                                 ("dot", lambda: mpx.dot(p, x, y, out=r, ws=ws))):
                    g = torch.cuda.CUDAGraph()
                    fn()
                    torch.cuda.synchronize()
                    with torch.cuda.graph(g):
                        for _ in range(calls):
                            fn()
                    tg = T(lambda: g.replay()) / calls
                    row[str(n)][f"{name}_graph_us"] = tg * 1e3
                    row[str(n)][f"{name}_graph_calls_per_s"] = 1.0 / (tg * 1e-3)
                    del g
        out[p] = row
    return out


def vector_sweep_rows(mpx, torch, T):
    """Bandwidth sweep (an extension of the n = 4096 / 2^24 rows): elementwise
    add, AXPY and dot for n = 2^16 .. 2^26, DD / TD / QD, GB/s against the
    8 TB/s HBM peak.  One QD pair of 2^26 elements (a seeded block of 1000003
    values repeated) serves every row: smaller n and K use its leading
    components and elements (plane stride 2^26)."""
    from paper_2603_14926_amd import synth
    nmax, period = 1 << 26, 1_000_003

    def tiled(seed):
        # the seeded block repeated along the planes (generating 2^26 QD values
        # on the host takes minutes; streaming bandwidth does not see values)
        base = gpu_mp(torch, 4, period, seed)
        t = torch.empty((4, nmax), dtype=torch.float64, device="cuda")
        q, rem = divmod(nmax, period)
        t[:, :q * period].view(4, q, period).copy_(base[:, None, :].expand(4, q, period))
        t[:, q * period:].copy_(base[:, :rem])
        return t

    x4, y4 = tiled(synth.seed_for(0, 11)), tiled(synth.seed_for(0, 12))
    z4 = torch.empty_like(x4)
    out = {}
    for p in ("qd", "td", "dd"):
        K = mpx.ncomp(p)
        alpha = [0.75] + [0.0] * (K - 1)
        r = torch.empty(K, dtype=torch.float64, device="cuda")
        for lg in range(16, 27, 2):
            n = 1 << lg
            x, y, z = x4[:K, :n], y4[:K, :n], z4[:K, :n]
            ws = mpx.workspace(mpx.OP_DOT, p, n)
            reps = 100 if n <= (1 << 20) else 1
            best = lambda fn: T(fn, reps=reps)
            t_add = best(lambda: mpx.add(p, x, y, out=z))
            t_axpy = best(lambda: mpx.axpy(p, alpha, x, z))
            t_dot = best(lambda: mpx.dot(p, x, y, out=r, ws=ws))
            b3, b2 = 3 * K * 8.0 * n, 2 * K * 8.0 * n
            out[f"{p}_2^{lg}"] = {
                "add_us": t_add * 1e3, "add_GB_s": b3 / (t_add * 1e-3) / 1e9,
                "axpy_us": t_axpy * 1e3, "axpy_GB_s": b3 / (t_axpy * 1e-3) / 1e9,
                "dot_us": t_dot * 1e3, "dot_GB_s": b2 / (t_dot * 1e-3) / 1e9,
                "frac_hbm": {"add": b3 / (t_add * 1e-3) / PEAK_HBM, "axpy": b3 / (t_axpy * 1e-3) / PEAK_HBM,
                             "dot": b2 / (t_dot * 1e-3) / PEAK_HBM},
            }
    del x4, y4, z4
    return out


# ------------------------------------------------- Horner versus Estrin ----

def polyeval_rows(mpx, torch, T):
    """Real-argument polynomial evaluation (Section 4.1): Horner (one thread
    per polynomial, a dependent chain of deg steps) versus Estrin (one wave per
    polynomial, log-depth; four waves for lists of 2^12 and more), batch 1024,
    random coefficients, x in [-1, 1)."""
    from paper_2603_14926_amd import synth
    out = {}
    batch = 1024
    for p in ("qd", "td", "dd"):
        K = mpx.ncomp(p)
        for deg in (16, 64, 256, 1024, 2047, 4095):
            coef = gpu_mp(torch, K, (batch, deg + 1), synth.seed_for(6, deg))
            x = gpu_mp(torch, K, batch, synth.seed_for(6, 1))
            y = torch.empty((K, batch), dtype=torch.float64, device="cuda")
            th = T(lambda: mpx.polyval(p, coef, x, out=y))
            te = T(lambda: mpx.polyval(p, coef, x, out=y, method="estrin"))
            out[f"{p}_deg{deg}"] = {"horner_us": th * 1e3, "estrin_us": te * 1e3, "estrin_speedup": th / te}
        # the same at complex points (real coefficients; Estrin up to degree 4095)
        for deg in (16, 64, 256, 1023, 2047):
            coef = gpu_mp(torch, K, (batch, deg + 1), synth.seed_for(6, deg))
            xr = gpu_mp(torch, K, batch, synth.seed_for(6, 1))
            xi = gpu_mp(torch, K, batch, synth.seed_for(6, 2))
            y = (torch.empty((K, batch), dtype=torch.float64, device="cuda"),
                 torch.empty((K, batch), dtype=torch.float64, device="cuda"))
            th = T(lambda: mpx.polyval_cplx(p, coef, xr, xi, out=y))
            te = T(lambda: mpx.polyval_cplx(p, coef, xr, xi, out=y, method="estrin"))
            out[f"{p}_complex_deg{deg}"] = {"horner_us": th * 1e3, "estrin_us": te * 1e3,
                                            "estrin_speedup": th / te}
    return out


# ------------------------------------------------------- BF vs NoBF ----

# FP64 operations per conventional multiply-add on the typical path (the
# conventional addition plus multiplication, renormalisation included).
NOBF_OPS_PER_MAC = {"dd_nobf": 11 + 9, "dd_nobf_acc": 20 + 9, "td_nobf": 60 + 129, "qd_nobf": 85 + 145}


def nobf_rows(mpx, torch, T):
    """Branch-free versus conventional arithmetic (the comparison of Tables 3-4
    and Figure 3): GEMM n = 1024, 2048 (each arithmetic autotuned), batched
    Horner at real and complex points, and batched Durand-Kerner on the
    Chebyshev polynomial (each arithmetic autotuned); speedup = conventional
    time / BF time."""
    from paper_2603_14926_amd import synth
    out = {}
    pairs = [("qd", "qd_nobf"), ("td", "td_nobf"), ("dd", "dd_nobf"), ("dd", "dd_nobf_acc")]
    for n in (1024, 2048):
        for bf, nb in pairs:
            K = mpx.ncomp(bf)
            A = gpu_mp(torch, K, (n, n), synth.seed_for(1, 0))
            B = gpu_mp(torch, K, (n, n), synth.seed_for(1, 1))
            Cm = torch.empty_like(A)
            r = {}
            for q in (bf, nb):
                v, _ = mpx.gemm_autotune(q, A, B, Cm, reps=1)
                r[q] = (T(lambda: mpx.gemm(q, A, B, out=Cm)), mpx.gemm_variants(q)[v])
            tb, tn = r[bf][0], r[nb][0]
            out[f"gemm_{nb}_{n}"] = {"bf_ms": tb, "nobf_ms": tn, "speedup_bf": tn / tb,
                                    "bf_variant": r[bf][1], "nobf_variant": r[nb][1],
                                    "nobf_ops_per_mac": NOBF_OPS_PER_MAC[nb]}
            del A, B, Cm
    # Horner at the autograd shape (1024 polynomials of degree 1024, one
    # thread each): a dependent chain, so the time is the chain's latency, the
    # GPU analogue of the paper's one-evaluation-per-core timings.
    batch, deg = 1024, 1024
    for bf, nb in pairs:
        K = mpx.ncomp(bf)
        coef = gpu_mp(torch, K, (batch, deg + 1), synth.seed_for(6, deg))
        x = gpu_mp(torch, K, batch, synth.seed_for(6, 1))
        y = torch.empty((K, batch), dtype=torch.float64, device="cuda")
        tb = T(lambda: mpx.polyval(bf, coef, x, out=y))
        tn = T(lambda: mpx.polyval(nb, coef, x, out=y))
        out[f"horner_{nb}_b{batch}_deg{deg}"] = {"bf_ms": tb, "nobf_ms": tn, "speedup_bf": tn / tb}
        xi = gpu_mp(torch, K, batch, synth.seed_for(6, 2))
        yc = (y, torch.empty_like(y))
        tb = T(lambda: mpx.polyval_cplx(bf, coef, x, xi, out=yc))
        tn = T(lambda: mpx.polyval_cplx(nb, coef, x, xi, out=yc))
        out[f"horner_complex_{nb}_b{batch}_deg{deg}"] = {"bf_ms": tb, "nobf_ms": tn, "speedup_bf": tn / tb}
        del coef, x, y, xi, yc
    # Durand-Kerner on the Chebyshev integration polynomial n = 64 (Table 6's
    # problem), 4096 copies in one persistent launch, Aberth start, 200 sweeps
    # (every copy is one 64-lane item, so the launch shape matters: autotuned).
    from fractions import Fraction  # noqa: F401  (coefficients are exact rationals)
    n, copies, iters = 64, 4096, 200
    a = synth.chebyshev_coefficients(n)
    deg = np.full(copies, n, np.int32)
    for bf, nb in pairs:
        K = mpx.ncomp(bf)
        one = np.stack([synth.round_greedy(c, K) for c in a], axis=1)
        cre = torch.from_numpy(np.tile(one, (1, copies))).cuda()
        cim = torch.zeros_like(cre)
        zr = torch.zeros((K, n * copies), dtype=torch.float64, device="cuda")
        zi = torch.zeros_like(zr)
        r, var = {}, {}
        for q in (bf, nb):   # each arithmetic at its own autotuned launch shape
            plan = mpx.RootsPlan(q, deg, iters=iters, init=True, graph=True)
            var[q], _ = plan.autotune(cre, cim, zr, zi, iters_probe=8)
            r[q] = T(lambda: plan.run(cre, cim, zr, zi))
        out[f"dk_chebyshev64_{nb}_x{copies}_{iters}it"] = {"bf_ms": r[bf], "nobf_ms": r[nb],
                                                          "speedup_bf": r[nb] / r[bf],
                                                          "bf_variant": int(var[bf]),
                                                          "nobf_variant": int(var[nb])}
        del cre, cim, zr, zi
    return out


# --------------------------------------------------------- batched GEMM ----

def batched_gemm_rows(mpx, torch, T):
    """The batching pattern for small products: 4096 QD GEMMs with m, n, k
    uniform in [16, 128] in one persistent launch (autotuned tiling), against
    one mpx_gemm launch per problem on the same packed buffers."""
    from paper_2603_14926_amd import synth
    rng = np.random.default_rng(synth.seed_for(1, 50))
    count, K = 4096, 4
    ms, ns, ks = (rng.integers(16, 129, count) for _ in range(3))
    plan = mpx.GemmBatchPlan("qd", ms, ns, ks)
    a_off, b_off, c_off, (ta, tb, tc) = plan.offsets()
    A = gpu_mp(torch, K, ta, synth.seed_for(1, 51))
    B = gpu_mp(torch, K, tb, synth.seed_for(1, 52))
    Cm = torch.empty((K, tc), dtype=torch.float64, device="cuda")
    v, _ = plan.autotune(A, B, Cm, reps=1)
    t = T(lambda: plan.run(A, B, Cm))
    macs = float(np.sum(ms * ns * ks))
    views = [(A[:, a_off[i]:a_off[i] + ms[i] * ks[i]].view(K, int(ms[i]), int(ks[i])),
              B[:, b_off[i]:b_off[i] + ks[i] * ns[i]].view(K, int(ks[i]), int(ns[i])),
              Cm[:, c_off[i]:c_off[i] + ms[i] * ns[i]].view(K, int(ms[i]), int(ns[i])))
             for i in range(count)]
    tl = T(lambda: [mpx.gemm("qd", a, b, out=c) for a, b, c in views], reps=1, warmup=1)
    return {"problems": count, "sizes": "m, n, k uniform in [16, 128]", "ms": t,
            "mp_op_s": 2 * macs / (t * 1e-3),
            "frac_issue_peak": macs * INSTR_PER_MAC["qd"] / (t * 1e-3) / PEAK_F64_ISSUE,
            "variant": int(v), "per_problem_launches_ms": tl, "speedup_vs_launches": tl / t}


# -------------------------------------------------------------- Strassen ----

def strassen_rows(mpx, torch, T):
    """Strassen's recursion (the scheme Section 3.1 benchmarks) against the
    classical product at the same size; cutoff 2048: one level at n = 2048,
    two at 4096, leaves of 1024^3 on the tuned GEMM.  Also BF against
    conventional arithmetic under Strassen at n = 2048 (Table 4's pairing)."""
    from paper_2603_14926_amd import synth
    out = {}
    runs = [("qd", 2048), ("qd", 4096), ("td", 2048), ("td", 4096), ("dd", 2048), ("dd", 4096),
            ("qd_nobf", 2048), ("td_nobf", 2048)]
    times = {}
    for p, n in runs:
        cutoff, leaf = 2048, 1024
        K = mpx.ncomp(p)
        A = gpu_mp(torch, K, (n, n), synth.seed_for(1, 0))
        B = gpu_mp(torch, K, (n, n), synth.seed_for(1, 1))
        Cm = torch.empty_like(A)
        ws = mpx.workspace(mpx.OP_STRASSEN, p, n, n, n, cutoff)
        mpx.gemm_autotune(p, A[:, :leaf, :leaf], B[:, :leaf, :leaf], Cm[:, :leaf, :leaf], reps=1)
        ts = T(lambda: mpx.gemm_strassen(p, A, B, cutoff, out=Cm, ws=ws))
        mpx.gemm_autotune(p, A, B, Cm, reps=1)
        tc = T(lambda: mpx.gemm(p, A, B, out=Cm))
        times[(p, n)] = ts
        levels = 0
        d = n
        while d >= cutoff:
            d = (d + 1) // 2
            levels += 1
        out[f"{p}_{n}"] = {"strassen_ms": ts, "classic_ms": tc, "speedup": tc / ts, "levels": levels,
                           "cutoff": cutoff, "classical_mp_op_s": 2.0 * n ** 3 / (ts * 1e-3)}
        del A, B, Cm, ws
    for q in ("qd", "td"):
        out[f"{q}_2048"]["speedup_bf_over_nobf"] = times[(q + "_nobf", 2048)] / times[(q, 2048)]
    return out


# ------------------------------------------------------------ complex 3M ----

def cgemm_rows(mpx, torch, T):
    """Complex GEMM by the 3M method (Section 3.2) at n = 2048 and the
    paper's n = 2049; reports time and the complex / real time ratio."""
    from paper_2603_14926_amd import synth
    out = {}
    for p in ("qd", "td", "dd"):
        K = mpx.ncomp(p)
        for n in (2048, 2049):
            mk = lambda s: gpu_mp(torch, K, (n, n), synth.seed_for(5, s), "W", phi=1.0)
            Are, Aim, Bre, Bim = mk(0), mk(1), mk(2), mk(3)
            Cre, Cim = torch.empty_like(Are), torch.empty_like(Are)
            ws = mpx.workspace(mpx.OP_CGEMM, p, n, n, n)
            t_c = T(lambda: mpx.cgemm_3m(p, Are, Aim, Bre, Bim, out=(Cre, Cim), ws=ws))
            t_r = T(lambda: mpx.gemm(p, Are, Bre, out=Cre))
            macs = 3.0 * n ** 3
            out[f"{p}_{n}"] = {"ms": t_c, "real_gemm_ms": t_r, "complex_over_real": t_c / t_r,
                               "frac_issue_peak": macs * INSTR_PER_MAC[p] / (t_c * 1e-3) / PEAK_F64_ISSUE}
            del Are, Aim, Bre, Bim, Cre, Cim, ws
    return out


# --------------------------------------------------------- Durand-Kerner ----

def dk_residual(deg, cre, cim, zr, zi, polys):
    """max_i |q(z_i)| / sum_k |c_k| |z_i|^k over the roots of the given
    polynomials (binary64 from the leading components; z scaled by
    max(1, |z|) so degree-512 values do not overflow)."""
    from paper_2603_14926_amd import synth
    coff, roff = synth.offsets(deg)
    worst_small, worst = 0.0, 0.0
    for b in polys:
        n = int(deg[b])
        a = cre[0, coff[b]:coff[b + 1]] + 1j * cim[0, coff[b]:coff[b + 1]]
        c = a / a[-1]
        z = zr[0, roff[b]:roff[b + 1]] + 1j * zi[0, roff[b]:roff[b + 1]]
        if not np.all(np.isfinite(z)):
            return float("nan"), float("nan")
        s = np.maximum(1.0, np.abs(z))
        w = z / s
        num = np.ones_like(z)
        den = np.ones(z.shape)
        inv = 1.0 / s
        scale = np.ones(z.shape)
        for k in range(n - 1, -1, -1):
            scale = scale * inv
            num = num * w + c[k] * scale
            den = den * np.abs(w) + abs(c[k]) * scale
        r = float(np.max(np.abs(num) / den))
        worst = max(worst, r)
        if n <= 24:
            worst_small = max(worst_small, r)
    return worst, worst_small


def dk_row(mpx, torch, T):
    from paper_2603_14926_amd import synth
    K = 4
    deg, cre, cim, known = synth.dk_batch(K, 4096, 16, 512, seed=synth.seed_for(2, 0), n_known=16)
    total_roots = int(deg.sum())
    gcr, gci = torch.from_numpy(cre).cuda(), torch.from_numpy(cim).cuda()
    zr = torch.zeros((K, total_roots), dtype=torch.float64, device="cuda")
    zi = torch.zeros_like(zr)
    # start values (Aberth) from a 0-sweep init plan, then the timed 200-sweep plan
    mpx.RootsPlan("qd", deg, iters=0, init=True, graph=False).run(gcr, gci, zr, zi)
    z0r, z0i = zr.clone(), zi.clone()
    plan = mpx.RootsPlan("qd", deg, iters=200, init=False, graph=True)
    variant, probe_ms = plan.autotune(gcr, gci, z0r, z0i, iters_probe=8)
    stream = torch.cuda.Stream()
    st = torch.zeros(deg.size, dtype=torch.int32, device="cuda")
    times = []
    for rep in range(10):   # the autotuner's probe runs are the warm-up
        zr.copy_(z0r); zi.copy_(z0i)
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            plan.run(gcr, gci, zr, zi, status=st)
            e1.record(stream)
        stream.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    r, i = zr.cpu().numpy(), zi.cpu().numpy()
    sample = list(range(16)) + list(range(16, deg.size, 16))
    worst, worst_small = dk_residual(deg, cre, cim, r, i, sample)
    _, roff = synth.offsets(deg)
    kerr = 0.0
    for b in range(16):
        z = r[0, roff[b]:roff[b + 1]] + 1j * i[0, roff[b]:roff[b + 1]]
        kerr = max(kerr, max(float(np.min(np.abs(z - w))) for w in known[b]))
    n2 = float((deg.astype(np.float64) ** 2).sum())
    instr = 1672.0 * n2 * 200          # ~1672 FP64 VALU instr per root pair per sweep (QD)
    return {"polys": int(deg.size), "roots": total_roots, "sweeps": 200, "ms": ms,
            "roots_per_s": total_roots / (ms * 1e-3),
            "frac_issue_peak_est": instr / (ms * 1e-3) / PEAK_F64_ISSUE,
            "variant": int(variant), "nonfinite_polys": int(st.sum().item()),
            "max_residual": worst, "max_residual_deg_le_24": worst_small,
            "residual_sample": f"{len(sample)} polynomials (16 known-root + every 16th)",
            "known_root_max_error": kerr}


# -------------------------------------------------------------- autograd ----

def autograd_row(mpx, torch, T):
    from paper_2603_14926_amd import autograd as ag, synth
    out = {}
    n = 2048
    for p in ("qd", "dd"):
        K = mpx.ncomp(p)
        A = gpu_mp(torch, K, (n, n), synth.seed_for(3, 0)).requires_grad_(True)
        B = gpu_mp(torch, K, (n, n), synth.seed_for(3, 1)).requires_grad_(True)
        G = gpu_mp(torch, K, (n, n), synth.seed_for(3, 2))

        def step():
            A.grad = None; B.grad = None
            ag.gemm(A, B, p).backward(G)
        ms = T(step)
        macs = 3.0 * n ** 3
        out[f"{p}_gemm_fwd_bwd_{n}"] = {"ms": ms, "mp_op_s": 2 * macs / (ms * 1e-3),
                                        "frac_issue_peak": macs * INSTR_PER_MAC[p] / (ms * 1e-3) / PEAK_F64_ISSUE}
    K, batch, deg = 4, 1024, 1024
    coef = gpu_mp(torch, K, (batch, deg + 1), synth.seed_for(3, 10)).requires_grad_(True)
    x = gpu_mp(torch, K, batch, synth.seed_for(3, 11)).requires_grad_(True)
    g = gpu_mp(torch, K, batch, synth.seed_for(3, 12))
    ms_f = T(lambda: ag.polyval(coef, x, "qd"))

    def hstep():
        coef.grad = None; x.grad = None
        ag.polyval(coef, x, "qd").backward(g)
    ms_fb = T(hstep)
    out["qd_horner_1024x1024"] = {"fwd_ms": ms_f, "fwd_bwd_ms": ms_fb}
    return out


# ----------------------------------------------------------------- Ozaki ----

def exact_dot(a, b):
    """sum_k (sum_c a[c, k]) (sum_c b[c, k]) exactly, as a Fraction: every
    binary64 is an integer times a power of two, so each multicomponent value
    becomes one integer over the smallest power of two among its components
    and the products are summed as integers."""
    from fractions import Fraction

    def scaled(p):
        m, e = np.frexp(np.asarray(p, np.float64))
        mi = (m * 9007199254740992.0).astype(np.int64)       # m 2^53: exact
        ee = e.astype(np.int64) - 53
        low = int(ee[mi != 0].min()) if np.any(mi != 0) else 0
        vals = [0] * p.shape[1]
        for c in range(p.shape[0]):
            for k, (x, sh) in enumerate(zip(mi[c].tolist(), (ee[c] - low).tolist())):
                if x:
                    vals[k] += x << sh
        return vals, low

    va, ea = scaled(a)
    vb, eb = scaled(b)
    return Fraction(sum(x * y for x, y in zip(va, vb))) * Fraction(2) ** (ea + eb)


def sampled_entries(n, count, rng):
    """(rows, cols) of `count` entries of an n x n product: the first pair
    up each row and column index at the edges of the 16- and 32-wide MFMA
    tiles and of the matrix (first / last, centre) with another such edge,
    the rest uniformly random."""
    edges = sorted({0, 1, 15, 16, 31, 32, 63, 64, 127, 128, n // 2 - 1, n // 2,
                    n - 33, n - 32, n - 17, n - 16, n - 2, n - 1})
    rows = np.array(edges + rng.integers(0, n, count - len(edges)).tolist())
    cols = np.array(edges[::-1] + rng.integers(0, n, count - len(edges)).tolist())
    return rows, cols


class ExactSample:
    """Exact values sum_k a_ik b_kj (rationals) of sampled entries of C = A B,
    computed once, and the errors of any computed C at those entries:
      sum_norm  max |C_ij - exact| / sum_k |a_ik[0] b_kj[0]|
                (the normalisation of the reduction bound n 2^-104 sum|ab|)
      rel       max |C_ij - exact| / |exact|   (componentwise relative)."""

    def __init__(self, A, B, rows, cols):
        self.rows, self.cols = rows, cols
        self.ex, self.sc = [], []
        for i, j in zip(rows, cols):
            a = np.ascontiguousarray(A[:, i, :]); b = np.ascontiguousarray(B[:, :, j])
            self.ex.append(exact_dot(a, b))
            self.sc.append(float(np.sum(np.abs(a[0]) * np.abs(b[0]))))

    def errors(self, torch, Cm):
        from fractions import Fraction
        ri = torch.as_tensor(self.rows, device=Cm.device)
        ci = torch.as_tensor(self.cols, device=Cm.device)
        Cs = Cm[:, ri, ci].cpu().numpy()
        e_sum = e_rel = 0.0
        for t, (ex, sc) in enumerate(zip(self.ex, self.sc)):
            d = abs(sum((Fraction(float(v)) for v in Cs[:, t]), Fraction(0)) - ex)
            e_sum = max(e_sum, float(d) / sc)
            e_rel = max(e_rel, float(d / abs(ex)) if ex != 0 else (0.0 if d == 0 else float("inf")))
        return {"sum_norm": e_sum, "rel": e_rel}


# Ozaki candidates in order of cost (slice-pair products s(s+1)/2): beta = 22
# (22 bits per slice, exact level sums with kblk = 256 up to 6 slices), then
# beta = 20 for more slices.
# (slices, beta, kblk), each meeting kblk 2^(2 beta) (1 + max(0, s-2)/4) <= 2^53
# so the slice products are exact; ordered by cost (slice pairs, then folds).
OZAKI_CANDIDATES = [(4, 22, 256), (5, 22, 256), (6, 22, 256), (6, 23, 64), (7, 22, 128),
                    (8, 22, 128), (9, 22, 128), (10, 22, 128), (12, 22, 128)]
OZAKI_SAMPLES = 64


def ozaki_row(mpx, torch, T, sizes):
    """Ozaki DD GEMM against the branch-free DD GEMM at n in `sizes`,
    phi = 1, 4, 8.  Errors on OZAKI_SAMPLES sampled entries (tile and matrix
    edges plus random ones) against exact rationals.  at_bound: the cheapest
    candidate whose sum-normalised error meets the DD reduction bound
    n 2^-104; at_bf_error: the cheapest whose componentwise relative error
    is no larger than the branch-free DD GEMM's on the same entries."""
    from paper_2603_14926_amd import synth
    out = {}
    rng = np.random.default_rng(11)
    for n in sizes:
        for phi in (1.0, 4.0, 8.0):
            log(f"ozaki n={n} phi={phi}")
            A_np = synth.mp_array(2, (n, n), synth.seed_for(4, int(phi)), "W", phi=phi)
            B_np = synth.mp_array(2, (n, n), synth.seed_for(4, 10 + int(phi)), "W", phi=phi)
            A, B = torch.from_numpy(A_np).cuda(), torch.from_numpy(B_np).cuda()
            rows, cols = sampled_entries(n, OZAKI_SAMPLES, rng)
            ref = ExactSample(A_np, B_np, rows, cols)
            del A_np, B_np
            Cbf = torch.empty_like(A)
            mpx.gemm_autotune("dd", A, B, Cbf, reps=1)
            t_bf = T(lambda: mpx.gemm("dd", A, B, out=Cbf))
            err_bf = ref.errors(torch, Cbf)
            del Cbf
            bound = n * 2.0 ** -104
            chosen, sweep = None, {}
            Coz = torch.empty_like(A)
            for (s, beta, kblk) in OZAKI_CANDIDATES:
                ws = mpx.workspace(mpx.OP_OZAKI, "dd", n, n, n, s)
                mpx.gemm_ozaki_dd(A, B, s, beta=beta, kblk=kblk, out=Coz, ws=ws)
                err = ref.errors(torch, Coz)
                sweep[(s, beta, kblk)] = err
                del ws
                if err["sum_norm"] <= bound and chosen is None:
                    chosen = (s, beta, kblk)
                if err["rel"] <= err_bf["rel"]:
                    break
            s_eq = next((c for c, e in sweep.items() if e["rel"] <= err_bf["rel"]), None)
            res = {"bf_dd_ms": t_bf, "bf_dd_err": err_bf, "bound_sum_norm": bound,
                   "error_by_slices": {f"s{s}_beta{b}_kblk{kb}": v for (s, b, kb), v in sweep.items()},
                   "sampled_entries": int(rows.size),
                   "equal_error_rule": "componentwise relative error (rel) <= the BF DD GEMM's"}
            for tag, cfg in (("at_bound", chosen), ("at_bf_error", s_eq)):
                if cfg is None:
                    continue
                s, beta, kblk = cfg
                ws = mpx.workspace(mpx.OP_OZAKI, "dd", n, n, n, s)
                t = T(lambda: mpx.gemm_ozaki_dd(A, B, s, beta=beta, kblk=kblk, out=Coz, ws=ws))
                prods = s * (s + 1) / 2
                res[tag] = {"slices": s, "beta": beta, "kblk": kblk, "ms": t, "err": sweep[cfg],
                            "frac_mfma_peak": prods * 2.0 * n ** 3 / (t * 1e-3) / PEAK_MFMA_F64,
                            "speedup_vs_bf_dd": t_bf / t}
                del ws
            out[f"n{n}_phi{int(phi)}"] = res
            del A, B, Coz
            torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the kernels are "
              f"single-GPU and no multi-GPU path is built.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2603_14926_amd import mpx, synth
    mpx.lib()
    T = Timer(torch)
    if args.peak_probe:
        # launches of ~60 ms (2^16 iterations), the engine clock brought to its
        # steady state by 10 untimed launches, median of 5
        r = {k: mpx.probe_valu(k, iters=1 << 16, reps=5, warmup=10) for k in mpx.PROBES}
        # FP64 additions at low occupancy: fraction of the issue peak for
        # 1, 2, 4 waves per SIMD and 1..16 independent chains per lane
        low = {f"{w}_waves_per_simd": {f"{c}_chains": mpx.probe_chains(c, w, iters=(1 << 16) // c)
                                       / PEAK_F64_ISSUE for c in (1, 2, 4, 8, 16)}
               for w in (1, 2, 4)}
        print(json.dumps({"peak_probe_lane_ops_per_s": r,
                          "assumed": {"f64": PEAK_F64_ISSUE, "f32": PEAK_F32_ISSUE},
                          "f64_add_fraction_low_occupancy": low}), flush=True)
        return
    if args.only:
        fn = {"gemm": lambda: {q: gemm_row(mpx, torch, T, q, args.n) for q in ("qd", "td", "dd", "ff")},
              "gemv": lambda: gemv_rows(mpx, torch, T),
              "vector": lambda: vector_rows(mpx, torch, T),
              "vector_sweep": lambda: vector_sweep_rows(mpx, torch, T),
              "cgemm": lambda: cgemm_rows(mpx, torch, T),
              "polyeval": lambda: polyeval_rows(mpx, torch, T),
              "nobf": lambda: nobf_rows(mpx, torch, T),
              "strassen": lambda: strassen_rows(mpx, torch, T),
              "batched": lambda: batched_gemm_rows(mpx, torch, T),
              "durand_kerner": lambda: dk_row(mpx, torch, T),
              "autograd": lambda: autograd_row(mpx, torch, T),
              "ozaki": lambda: ozaki_row(mpx, torch, T, (4096,) if args.no_8192 else (4096, 8192))}[args.only]
        print(json.dumps({"only": args.only, "row": fn()}), flush=True)
        return
    if args.calib_copy:
        src = torch.ones(64 << 20, dtype=torch.float64, device="cuda")   # 512 MiB
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    p, n = args.prec, args.n
    K = mpx.ncomp(p)
    dt = np.float32 if p == "ff" else np.float64
    log(f"headline {p} gemm n={n}")
    A = gpu_mp(torch, K, (n, n), synth.seed_for(1, 0), dtype=dt)
    B = gpu_mp(torch, K, (n, n), synth.seed_for(1, 1), dtype=dt)
    Cm = torch.empty_like(A)
    variant, _ = mpx.gemm_autotune(p, A, B, Cm, reps=1)
    for _ in range(args.warmup):
        mpx.gemm(p, A, B, out=Cm)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        mpx.gemm(p, A, B, out=Cm)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps * 1e3
    ms = e0.elapsed_time(e1) / args.steps
    macs = float(n) ** 3
    peak = PEAK_F32_ISSUE if p == "ff" else PEAK_F64_ISSUE
    achieved = macs * INSTR_PER_MAC[p] / (ms * 1e-3)
    out = {
        "metric": METRIC,
        "value": 2.0 * macs / (ms * 1e-3),
        "unit": "mp-op/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "wall_ms_per_step": wall,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if p == "ff" else "f64",
        "data": "synthetic (seeded SplitMix64; uniform leading component, non-overlapping lower components)",
        "config": {"workload": f"{p}_gemm_{n}x{n}x{n}", "precision": p.upper(), "m": n, "n": n, "k": n,
                   "kernel_variant": mpx.gemm_variants(p)[variant]},
        "roofline": {
            "bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12,
            "unit": "T FP64 VALU lane-instructions/s" if p != "ff" else "T FP32 VALU lane-instructions/s",
            "frac": achieved / peak,
            "frac_fp64_flop_peak": macs * FLOP_PER_MAC[p] / (ms * 1e-3) / PEAK_F64_FLOP,
            "traffic": measured_traffic(f"{p}_gemm_{n}", mpx.gemm_variants(p)[variant]),
            "traffic_unit": "bytes per launch (HBM fetch + write, rocprofv3 counters scaled by a copy kernel)",
            "algorithmic_bytes": 3.0 * K * (4 if p == "ff" else 8) * n * n,
        },
    }
    del A, B, Cm
    if not args.quick:
        def gemm_rows():
            g = {}
            for q in ("qd", "td", "dd"):
                for nn in (512, 1024, 2048):
                    g[f"{q}_{nn}"] = gemm_row(mpx, torch, T, q, nn)
            g["ff_2048"] = gemm_row(mpx, torch, T, "ff", 2048)
            return g
        plan = [("gemm", gemm_rows),
                ("gemv_8192", lambda: gemv_rows(mpx, torch, T)),
                ("vector", lambda: vector_rows(mpx, torch, T)),
                ("cgemm_3m", lambda: cgemm_rows(mpx, torch, T)),
                ("polyeval", lambda: polyeval_rows(mpx, torch, T)),
                ("bf_vs_nobf", lambda: nobf_rows(mpx, torch, T)),
                ("strassen", lambda: strassen_rows(mpx, torch, T)),
                ("batched_gemm", lambda: batched_gemm_rows(mpx, torch, T)),
                ("durand_kerner", lambda: dk_row(mpx, torch, T)),
                ("autograd", lambda: autograd_row(mpx, torch, T)),
                ("ozaki", lambda: ozaki_row(mpx, torch, T, (4096,) if args.no_8192 else (4096, 8192)))]
        rows = {}
        for i, (name, fn) in enumerate(plan):
            log(f"row {name}")
            try:
                rows[name] = fn()
            except Exception as e:
                # the headline is already measured: record the failure, run no
                # further GPU work after it, and still print the line
                rows[name] = {"error": f"{type(e).__name__}: {e}"}
                rows["skipped_after_error"] = [nm for nm, _ in plan[i + 1:]]
                log(f"row {name} failed ({type(e).__name__}: {e}); remaining rows skipped")
                break
        out["rows"] = rows
    if not args.no_cpu and not args.quick and p != "ff":
        log("cpu baseline")
        try:
            out["cpu_baseline"] = cpu_baseline(p, n)
        except Exception as e:  # the line is printed regardless
            out["cpu_baseline"] = {"error": f"{type(e).__name__}: {e}"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
