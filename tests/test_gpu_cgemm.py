"""GPU parity of the complex 3M GEMM (Section 3.2) against the oracle's 3M
implementation: bit-exact (same real-GEMM sequence and the same additions),
and the paper's complex accuracy at a larger size, checked exactly."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from tests import paper_values
from oracle import exact
from paper_2603_14926_amd import mpx, synth
from tests.gpu_util import bits_equal, first_mismatch, to_gpu, to_np

pytestmark = pytest.mark.gpu


def _cx(K, shape, seed, dt=np.float64):
    return (synth.mp_array(K, shape, seed, "W", phi=1.0, dtype=dt),
            synth.mp_array(K, shape, seed + 1, "W", phi=1.0, dtype=dt))


@pytest.mark.parametrize("p,K", [("dd", 2), ("td", 3), ("qd", 4)])
@pytest.mark.parametrize("mnk", [(1, 1, 1), (33, 20, 47), (64, 70, 65)])
def test_cgemm_3m_bit_exact(p, K, mnk):
    m, n, k = mnk
    Are, Aim = _cx(K, (m, k), 10 + m)
    Bre, Bim = _cx(K, (k, n), 20 + n)
    wr, wi = oracle.cgemm_3m(K, Are, Aim, Bre, Bim)
    gr, gi = mpx.cgemm_3m(p, to_gpu(Are), to_gpu(Aim), to_gpu(Bre), to_gpu(Bim))
    assert bits_equal(to_np(gr), wr), first_mismatch(to_np(gr), wr)
    assert bits_equal(to_np(gi), wi), first_mismatch(to_np(gi), wi)


PAPER_COMPLEX_DIGITS = paper_values.gemm_digits("complex")   # tests/golden/gemm_digits.txt


@pytest.mark.parametrize("p,K", [("dd", 2), ("td", 3), ("qd", 4)])
def test_cgemm_3m_paper_accuracy_1024(p, K):
    """n = 1024 complex matrices of Section 3.2: norm-wise relative error of
    sampled entries of each part against the exact product meets the digits
    the paper reports at n = 2049."""
    n = 1024
    Are, Aim = _cx(K, (n, n), 30)
    Bre, Bim = _cx(K, (n, n), 40)
    gr, gi = mpx.cgemm_3m(p, to_gpu(Are), to_gpu(Aim), to_gpu(Bre), to_gpu(Bim))
    R, I = to_np(gr), to_np(gi)
    rng = np.random.default_rng(1)
    worst = {"re": 0.0, "im": 0.0}; scale = {"re": 0.0, "im": 0.0}
    for i, j in zip(rng.integers(0, n, 12), rng.integers(0, n, 12)):
        ar, ai = np.ascontiguousarray(Are[:, i, :]), np.ascontiguousarray(Aim[:, i, :])
        br, bi = np.ascontiguousarray(Bre[:, :, j]), np.ascontiguousarray(Bim[:, :, j])
        ex_re = exact.dot(ar, br) - exact.dot(ai, bi)
        ex_im = exact.dot(ar, bi) + exact.dot(ai, br)
        for part, got, ex in (("re", R[:, i, j], ex_re), ("im", I[:, i, j], ex_im)):
            worst[part] = max(worst[part], abs(float(exact.value(got) - ex)))
            scale[part] = max(scale[part], abs(float(ex)))
    digits = min(-math.log10(worst[q] / scale[q]) if worst[q] else 99.0 for q in worst)
    assert digits >= PAPER_COMPLEX_DIGITS[K], digits


@pytest.mark.parametrize("n", [2048, 2049])
def test_cgemm_3m_bench_size_sampled_bit_exact(n):
    """The benchmark sizes (QD, n = 2048 and the paper's 2049): sampled
    entries, tile edges and corners included, bit-exact against the oracle's
    3M steps evaluated entry by entry."""
    K = 4
    Are, Aim = _cx(K, (n, n), 70)
    Bre, Bim = _cx(K, (n, n), 72)
    gr, gi = mpx.cgemm_3m("qd", to_gpu(Are), to_gpu(Aim), to_gpu(Bre), to_gpu(Bim))
    rng = np.random.default_rng(n)
    rows = np.concatenate([[0, 0, n - 1, n - 1, 31, 32, n // 2], rng.integers(0, n, 13)])
    cols = np.concatenate([[0, n - 1, 0, n - 1, 32, 31, n // 2 + 1], rng.integers(0, n, 13)])
    wr, wi = oracle.cgemm_3m_entries(K, Are, Aim, Bre, Bim, rows, cols)
    assert bits_equal(np.ascontiguousarray(to_np(gr)[:, rows, cols]), wr)
    assert bits_equal(np.ascontiguousarray(to_np(gi)[:, rows, cols]), wi)
