"""GPU parity of Strassen's product (mpx_gemm_strassen) against the oracle's
recursion: bit-exact on whole matrices (odd, rectangular, several levels,
both arithmetics) and on sampled entries at the benchmark size."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle import strassen
from paper_2603_14926_amd import mpx, synth
from tests.gpu_util import bits_equal, first_mismatch, to_gpu, to_np

pytestmark = pytest.mark.gpu

PRECS = [("dd", 2), ("td", 3), ("qd", 4)]


@pytest.mark.parametrize("p,K", PRECS)
@pytest.mark.parametrize("mkn,cutoff", [((64, 64, 64), 16), ((65, 65, 65), 32), ((100, 129, 70), 20),
                                        ((33, 65, 17), 8), ((40, 40, 40), 64), ((2, 2, 2), 2)])
def test_strassen_bit_exact(p, K, mkn, cutoff):
    m, k, n = mkn
    A = synth.mp_array(K, (m, k), 10 + m, "W")
    B = synth.mp_array(K, (k, n), 20 + n, "W")
    want = strassen.gemm(K, A, B, cutoff)
    got = to_np(mpx.gemm_strassen(p, to_gpu(A), to_gpu(B), cutoff))
    assert bits_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("p,K,mode", [("qd_nobf", 4, "nobf"), ("td_nobf", 3, "nobf"),
                                      ("dd_nobf", 2, "nobf"), ("dd_nobf_acc", 2, "nobf_acc")])
def test_strassen_conventional_bit_exact(p, K, mode):
    A = synth.mp_array(K, (67, 50), 31, "U")
    B = synth.mp_array(K, (50, 45), 32, "U")
    with oracle.arith(mode):
        want = strassen.gemm(K, A, B, 12)
    got = to_np(mpx.gemm_strassen(p, to_gpu(A), to_gpu(B), 12))
    assert bits_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("p,K", [("qd", 4), ("dd", 2)])
def test_strassen_2048_one_level_sampled(p, K):
    """The benchmark shape: n = 2048, cutoff 2048 (one level, leaves 1024^3);
    20 sampled entries recomputed by the oracle's entry-wise recursion."""
    n = 2048
    A = synth.mp_array(K, (n, n), 90, "U")
    B = synth.mp_array(K, (n, n), 91, "U")
    got = to_np(mpx.gemm_strassen(p, to_gpu(A), to_gpu(B), 2048))
    rng = np.random.default_rng(5)
    rows = np.concatenate([[0, 0, n - 1, n - 1, 1023, 1024], rng.integers(0, n, 14)])
    cols = np.concatenate([[0, n - 1, 0, n - 1, 1024, 1023], rng.integers(0, n, 14)])
    want = strassen.entries(K, A, B, rows, cols, 2048)
    assert bits_equal(np.ascontiguousarray(got[:, rows, cols]), want)


def test_strassen_argument_errors():
    A = torch.zeros((4, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(mpx.MpxError):
        mpx.gemm_strassen("qd", A, A, 1)                       # cutoff < 2
    with pytest.raises(mpx.MpxError):
        mpx.gemm_strassen("qd", A, A, 2, ws=torch.empty(8, dtype=torch.uint8, device="cuda"))
    F = torch.zeros((2, 8, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(mpx.MpxError):
        mpx.gemm_strassen("ff", F, F, 4)
