"""Pins of the oracle's Strassen product (Section 3.1 runs its matrix
benchmarks with Strassen's algorithm, recursion stopped below 32 x 32):
the classical product when no split happens, exactness on integer data,
Higham's norm-wise error bound for Strassen's method, the paper's reported
accuracy on its real test matrices, and agreement of the whole-matrix and
entry-by-entry evaluations on odd and rectangular shapes."""
import math

import numpy as np
import pytest

import oracle
from tests import paper_values
from oracle import exact, strassen
from paper_2603_14926_amd import synth

# per-operation unit roundoff of the multicomponent arithmetic (largest of
# the add / mul ceilings)
U = {2: 2.0 ** -103, 3: 2.0 ** -155, 4: 2.0 ** -208}


def test_no_split_is_the_classical_product():
    K = 4
    A = synth.mp_array(K, (20, 31), 1, "W")
    B = synth.mp_array(K, (31, 9), 2, "W")
    assert np.array_equal(strassen.gemm(K, A, B, 10), oracle.gemm(K, A, B))
    assert np.array_equal(strassen.gemm(K, A, B, 32), oracle.gemm(K, A, B))


@pytest.mark.parametrize("K", [2, 3, 4])
def test_integer_matrices_are_exact(K):
    rng = np.random.default_rng(3 + K)
    A = np.zeros((K, 37, 29)); B = np.zeros((K, 29, 41))
    A[0] = rng.integers(-50, 51, (37, 29))
    B[0] = rng.integers(-50, 51, (29, 41))
    C = strassen.gemm(K, A, B, 4)
    assert np.array_equal(C, oracle.gemm(K, A, B))
    assert np.array_equal(C[0], A[0] @ B[0]) and np.all(C[1:] == 0)


def _higham_bound(n, n0):
    # Higham, Accuracy and Stability of Numerical Algorithms (2002), Thm 23.2:
    # ||C - C_hat|| <= [(n/n0)^log2(12) (n0^2 + 5 n0) - 5 n] u ||A|| ||B||
    return (n / n0) ** math.log2(12) * (n0 * n0 + 5 * n0) - 5 * n


@pytest.mark.parametrize("K", [2, 3, 4])
def test_normwise_error_within_higham_bound(K):
    n, cutoff = 64, 16          # 64 -> 32 -> 16 -> leaves of 8
    A = synth.mp_array(K, (n, n), 10 + K, "W")
    B = synth.mp_array(K, (n, n), 20 + K, "W")
    C = strassen.gemm(K, A, B, cutoff)
    na = max(abs(float(exact.value(A[:, i, j]))) for i in range(n) for j in range(n))
    nb = max(abs(float(exact.value(B[:, i, j]))) for i in range(n) for j in range(n))
    worst = 0.0
    for i in range(0, n, 3):
        for j in range(0, n, 5):
            ex = exact.dot(A[:, i, :], np.ascontiguousarray(B[:, :, j]))
            worst = max(worst, abs(float(exact.value(C[:, i, j]) - ex)))
    bound = _higham_bound(n, 8) * U[K] * n * na * nb
    assert worst <= bound, (worst, bound)
    # and it is a real multicomponent result, far below binary64 accuracy
    assert worst <= 2.0 ** -(53 * K - 20) * n * na * nb


PAPER_DIGITS = paper_values.gemm_digits("real")   # tests/golden/gemm_digits.txt


@pytest.mark.parametrize("K", [2, 3, 4])
@pytest.mark.parametrize("n", [64, 65])
def test_paper_matrices_meet_reported_digits(K, n):
    """a_ij = sqrt5 (i+j-1), b_ij = sqrt3 (n-i+1), Strassen with cutoff 32:
    the paper reports 29.0 / 45.5 / 61.7 or more significant digits."""
    A, B = synth.paper_real_gemm(K, n)
    rows = np.array([0, 7, n // 2, n - 1]); cols = np.array([0, n - 1, 5, n // 2 + 1])
    got = strassen.entries(K, A, B, rows, cols, 32)
    s15 = synth.sqrt_fraction(15, bits=400)
    for t in range(rows.size):
        ex = s15 * synth.paper_real_gemm_exact(n, int(rows[t]), int(cols[t]))
        rel = abs(exact.value(got[:, t]) - ex) / ex
        digits = -math.log10(float(rel)) if rel > 0 else 99.0
        assert digits >= PAPER_DIGITS[K], (K, n, t, digits)


@pytest.mark.parametrize("mkn,cutoff", [((9, 7, 11), 3), ((33, 65, 17), 8), ((50, 50, 50), 4),
                                        ((64, 64, 64), 16)])
def test_whole_and_entrywise_evaluations_agree(mkn, cutoff):
    K = 3
    m, k, n = mkn
    A = synth.mp_array(K, (m, k), 30, "U")
    B = synth.mp_array(K, (k, n), 31, "U")
    C = strassen.gemm(K, A, B, cutoff)
    rows = np.concatenate([np.arange(m), [m - 1, 0]])
    cols = np.concatenate([(np.arange(m) * 7) % n, [n - 1, n - 1]])
    assert np.array_equal(strassen.entries(K, A, B, rows, cols, cutoff), C[:, rows, cols])


def test_one_level_blocks_by_hand():
    """One split of 2 x 2 scalars reproduces Strassen's seven products."""
    K = 2
    a = np.array([[3.0, -1.0], [2.0, 5.0]]); b = np.array([[1.0, 4.0], [-2.0, 0.5]])
    A = np.zeros((K, 2, 2)); B = np.zeros((K, 2, 2))
    A[0], B[0] = a, b
    C = strassen.gemm(K, A, B, 2)
    assert np.array_equal(C[0], a @ b)
    with pytest.raises(ValueError):
        strassen.gemm(K, A, B, 1)


def test_conventional_arithmetic_follows_the_same_recursion():
    K = 4
    A = synth.mp_array(K, (24, 24), 40, "U")
    B = synth.mp_array(K, (24, 24), 41, "U")
    with oracle.arith("nobf"):
        C = strassen.gemm(K, A, B, 6)
        E = strassen.entries(K, A, B, [0, 23, 11], [23, 0, 12], 6)
    assert np.array_equal(E, C[:, [0, 23, 11], [23, 0, 12]])
    assert not np.array_equal(C, strassen.gemm(K, A, B, 6))
