"""CPU checks of bench.py's contract: one GPU only (more exits with a
message), the HBM-traffic figure is taken only from counters recorded on the
current kernel sources, and the CPU baseline leg reports the oracle with the
fields the JSON line carries."""
import importlib.util
import json
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout.strip() == ""            # no JSON line for an unmeasured N


def _sources_hash(root, files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def test_traffic_only_from_counters_on_current_sources(tmp_path):
    bench = _bench()
    rec = json.load(open(os.path.join(ROOT, "profiles", "qd_gemm_2048_counters.json")))
    assert "paper_2603_14926_amd/csrc/mpx_gemm.hip" in rec["sources"]
    # the tree itself: the recorded figure exactly when the sources match
    fresh = _sources_hash(ROOT, rec["sources"]) == rec["source_sha256_16"]
    by = rec["traffic_bytes_by_tiling"]
    assert by[rec["tiling"]] == rec["traffic_bytes"]
    for name, t in by.items():
        assert bench.measured_traffic("qd_gemm_2048", name) == (t if fresh else None)
    assert bench.measured_traffic("qd_gemm_2048", "no_such_tiling") is None
    assert bench.measured_traffic("no_such_workload", rec["tiling"]) is None
    # a copy whose record matches its sources, then one byte changed: no traffic
    os.makedirs(tmp_path / "profiles")
    for f in rec["sources"]:
        dst = tmp_path / f
        os.makedirs(dst.parent, exist_ok=True)
        shutil.copy(os.path.join(ROOT, f), dst)
    rec2 = dict(rec, source_sha256_16=_sources_hash(str(tmp_path), rec["sources"]))
    with open(tmp_path / "profiles" / "qd_gemm_2048_counters.json", "w") as fh:
        json.dump(rec2, fh)
    bench.ROOT = str(tmp_path)
    assert bench.measured_traffic("qd_gemm_2048", rec["tiling"]) == rec["traffic_bytes"]
    with open(tmp_path / rec["sources"][0], "ab") as fh:
        fh.write(b"\n")
    assert bench.measured_traffic("qd_gemm_2048", rec["tiling"]) is None


def test_cpu_baseline_fields():
    bench = _bench()
    r = bench.cpu_baseline("qd", 64, target_s=0.05, target_1t_s=0.05)
    assert r["kind"] == "oracle" and r["unit"] == "mp-op/s"
    assert r["value"] > 0 and 1 <= r["cores"] <= 16
    assert "QD GEMM rows 0.." in r["sample"] and "64x64x64" in r["sample"]
    one = r["single_thread"]
    assert one["cores"] == 1 and one["value"] > 0 and one["unit"] == "mp-op/s"


def test_bench_exact_dot_matches_the_exact_checker():
    """The benchmark's own exact sum of products (used for the Ozaki error
    comparison, so the timed script needs nothing from the oracle) equals the
    exact-rational checker's, and the relative error it reports is that of
    the checker."""
    import numpy as np
    from oracle import exact
    from paper_2603_14926_amd import synth
    bench = _bench()
    for K, n, dist in ((2, 300, "W"), (4, 257, "U"), (3, 1, "U")):
        a = synth.mp_array(K, n, 70 + K, dist)
        b = synth.mp_array(K, n, 80 + K, dist)
        assert bench.exact_dot(a, b) == exact.dot(a, b)
    A = synth.mp_array(2, (5, 64), 91, "W", phi=8.0)
    B = synth.mp_array(2, (64, 4), 92, "W", phi=8.0)
    C = np.zeros((2, 5, 4))
    C[0] = A[0] @ B[0]                                   # binary64 product: a visible error
    rows, cols = np.array([0, 3, 4]), np.array([1, 0, 3])
    d = [abs(exact.value(C[:, i, j]) - exact.dot(np.ascontiguousarray(A[:, i, :]),
                                                 np.ascontiguousarray(B[:, :, j]))) for i, j in zip(rows, cols)]
    want_sum = max(float(e) / exact.abs_dot(A[:, i, :], B[:, :, j]) for e, i, j in zip(d, rows, cols))
    want_rel = max(float(e / abs(exact.dot(np.ascontiguousarray(A[:, i, :]), np.ascontiguousarray(B[:, :, j]))))
                   for e, i, j in zip(d, rows, cols))
    import torch
    got = bench.ExactSample(A, B, rows, cols).errors(torch, torch.from_numpy(C))
    assert got == {"sum_norm": want_sum, "rel": want_rel}


def test_bench_sampled_entries_cover_tile_edges():
    import numpy as np
    bench = _bench()
    rows, cols = bench.sampled_entries(4096, 64, np.random.default_rng(0))
    assert rows.size == cols.size == 64
    for e in (0, 15, 16, 31, 32, 2047, 2048, 4095):
        assert e in rows[:18] and e in cols[:18]
    assert rows.min() >= 0 and rows.max() < 4096 and cols.min() >= 0 and cols.max() < 4096
