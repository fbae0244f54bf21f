"""GPU parity of the batched GEMM (many ragged products in one persistent
launch) against the oracle's product of each problem: bit-exact for every
tiling, empty problems included, and under HIP-graph replay."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2603_14926_amd import mpx, synth
from tests.gpu_util import bits_equal, first_mismatch, to_gpu, to_np

pytestmark = pytest.mark.gpu

PRECS = [("dd", 2, np.float64), ("td", 3, np.float64), ("qd", 4, np.float64), ("ff", 2, np.float32)]


def _batch(K, dt, count, seed, lo=1, hi=70):
    rng = np.random.default_rng(seed)
    ms, ns, ks = (rng.integers(lo, hi, count) for _ in range(3))
    ms[3] = 0; ns[5] = 0; ks[7] = 0          # empty products and an all-zero C block
    As = [synth.mp_array(K, (int(m), int(k)), seed + 10 + i, "W", dtype=dt) for i, (m, k) in enumerate(zip(ms, ks))]
    Bs = [synth.mp_array(K, (int(k), int(n)), seed + 5000 + i, "W", dtype=dt) for i, (k, n) in enumerate(zip(ks, ns))]
    return ms, ns, ks, As, Bs


def _pack(K, dt, blocks):
    flat = [b.reshape(K, -1) for b in blocks]
    return np.ascontiguousarray(np.concatenate(flat, axis=1) if flat else np.zeros((K, 0), dt))


def _want(p, K, As, Bs):
    out = []
    for A, B in zip(As, Bs):
        if A.shape[1] == 0:
            out.append(np.zeros((K, A.shape[1], B.shape[2]), A.dtype))
        else:
            out.append(oracle.ff_gemm(A, B) if p == "ff" else oracle.gemm(K, A, B))
    return out


@pytest.mark.parametrize("p,K,dt", PRECS)
def test_batched_bit_exact_every_tiling(p, K, dt):
    ms, ns, ks, As, Bs = _batch(K, dt, 40, 100 + K)
    plan = mpx.GemmBatchPlan(p, ms, ns, ks)
    A = to_gpu(_pack(K, dt, As)); B = to_gpu(_pack(K, dt, Bs))
    _, _, c_off, (_, _, tc) = plan.offsets()
    want = _want(p, K, As, Bs)
    for v in range(plan.variant_count()):
        Cm = torch.full((K, tc), float("nan"), dtype=A.dtype, device="cuda")
        plan.set_variant(v)
        got = to_np(plan.run(A, B, Cm))
        for i, w in enumerate(want):
            g = got[:, c_off[i]:c_off[i] + w.shape[1] * w.shape[2]].reshape(w.shape)
            assert bits_equal(np.ascontiguousarray(g), w), (v, i, first_mismatch(np.ascontiguousarray(g), w))
    v, ms_best = plan.autotune(A, B, torch.empty((K, tc), dtype=A.dtype, device="cuda"), reps=1)
    assert 0 <= v < plan.variant_count() and ms_best > 0


def test_batched_matches_single_gemm_at_larger_sizes():
    """Products of 60..300 (edge strips of hundreds of entries: several flat
    64-entry waves per strip) on every tiling equal mpx_gemm's bits."""
    K = 4
    ms, ns, ks, As, Bs = _batch(K, np.float64, 12, 7, lo=60, hi=300)
    plan = mpx.GemmBatchPlan("qd", ms, ns, ks)
    A = to_gpu(_pack(K, np.float64, As)); B = to_gpu(_pack(K, np.float64, Bs))
    _, _, c_off, (_, _, tc) = plan.offsets()
    singles = [to_np(mpx.gemm("qd", to_gpu(Ai), to_gpu(Bi))) for Ai, Bi in zip(As, Bs)]
    for v in range(plan.variant_count()):
        plan.set_variant(v)
        Cm = torch.full((K, tc), float("nan"), dtype=torch.float64, device="cuda")
        got = to_np(plan.run(A, B, Cm))
        for i, (Ai, Bi) in enumerate(zip(As, Bs)):
            m, n = Ai.shape[1], Bi.shape[2]
            g = np.ascontiguousarray(got[:, c_off[i]:c_off[i] + m * n].reshape(K, m, n))
            assert bits_equal(g, singles[i]), (v, i)


def test_batched_graph_replay():
    K = 3
    ms, ns, ks, As, Bs = _batch(K, np.float64, 25, 9)
    plan = mpx.GemmBatchPlan("td", ms, ns, ks)
    A = to_gpu(_pack(K, np.float64, As)); B = to_gpu(_pack(K, np.float64, Bs))
    _, _, c_off, (_, _, tc) = plan.offsets()
    Cm = torch.empty((K, tc), dtype=torch.float64, device="cuda")
    plan.run(A, B, Cm)
    torch.cuda.synchronize()
    want = _pack(K, np.float64, _want("td", K, As, Bs))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run(A, B, Cm)
    for rep in range(3):
        Cm.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _ = (torch.ones(1000, device="cuda") * 2).sum().item()
        assert bits_equal(to_np(Cm), want), rep


def test_batched_argument_errors():
    with pytest.raises(mpx.MpxError):
        mpx.GemmBatchPlan("qd_nobf", [2], [2], [2])
    with pytest.raises(mpx.MpxError):
        mpx.GemmBatchPlan("qd", [2, -1], [2, 2], [2, 2])
    plan = mpx.GemmBatchPlan("dd", [4], [4], [4])
    small = torch.zeros((2, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        plan.run(small, small, small)        # the binding: 16 elements per plane
    # the library itself: plane stride 8 < 16, rejected before any launch
    p8 = mpx._ptr(small)
    assert mpx.lib().mpx_gemm_batched(plan._h, p8, 8, p8, 8, p8, 8, None) == -1
    with pytest.raises(mpx.MpxError):
        plan.set_variant(99)


def test_batched_bench_configuration_sampled():
    """The benchmark's batch: 4096 QD products, m, n, k uniform in [16, 128],
    every tiling; 12 products (the extremes of m, n and k among them) checked
    whole against the oracle's GEMM."""
    K, count = 4, 4096
    rng = np.random.default_rng(synth.seed_for(1, 50))
    ms, ns, ks = (rng.integers(16, 129, count) for _ in range(3))
    plan = mpx.GemmBatchPlan("qd", ms, ns, ks)
    a_off, b_off, c_off, (ta, tb, tc) = plan.offsets()
    A_np = synth.mp_array(K, int(ta), 81, "U")
    B_np = synth.mp_array(K, int(tb), 82, "U")
    A, B = to_gpu(A_np), to_gpu(B_np)
    pick = sorted({int(np.argmax(ms)), int(np.argmin(ms)), int(np.argmax(ns)), int(np.argmin(ns)),
                   int(np.argmax(ks)), int(np.argmin(ks)), 0, count - 1,
                   *rng.integers(0, count, 4).tolist()})
    want = {}
    for i in pick:
        Ai = np.ascontiguousarray(A_np[:, a_off[i]:a_off[i] + ms[i] * ks[i]].reshape(K, ms[i], ks[i]))
        Bi = np.ascontiguousarray(B_np[:, b_off[i]:b_off[i] + ks[i] * ns[i]].reshape(K, ks[i], ns[i]))
        want[i] = oracle.gemm(K, Ai, Bi)
    for v in range(plan.variant_count()):
        plan.set_variant(v)
        Cm = torch.full((K, int(tc)), float("nan"), dtype=torch.float64, device="cuda")
        got = to_np(plan.run(A, B, Cm))
        for i in pick:
            g = np.ascontiguousarray(got[:, c_off[i]:c_off[i] + ms[i] * ns[i]].reshape(K, ms[i], ns[i]))
            assert bits_equal(g, want[i]), (v, i)
