"""Pins of the oracle's vector / matrix layer (elementwise, AXPY, dot, GEMV,
GEMM; Section 3.1) against exact rational arithmetic, closed forms and the
accuracy the paper reports for its real test matrices."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests import paper_values
from oracle import exact
from paper_2603_14926_amd import synth

BITS = {2: 104, 3: 155, 4: 208}


def _bound(K, n, scale):
    return n * 2.0 ** -BITS[K] * scale


@pytest.mark.parametrize("K", [2, 3, 4])
def test_elementwise_planes_match_single_ops(K):
    x = synth.mp_array(K, 257, 1, "W")
    y = synth.mp_array(K, 257, 2, "W")
    z = oracle.add(K, x, y)
    w = oracle.mul(K, x, y)
    for i in range(257):
        assert np.array_equal(z[:, i], oracle.op1(K, "add", x[:, i], y[:, i]))
        assert np.array_equal(w[:, i], oracle.op1(K, "mul", x[:, i], y[:, i]))


@pytest.mark.parametrize("K", [2, 3, 4])
def test_axpy_is_mul_then_add_and_accurate(K):
    n = 300
    alpha = synth.mp_array(K, 1, 3, "U")[:, 0]
    x = synth.mp_array(K, n, 4, "U")
    y = synth.mp_array(K, n, 5, "U")
    r = oracle.axpy(K, alpha, x, y)
    va = exact.value(alpha)
    for i in range(n):
        ex = va * exact.value(x[:, i]) + exact.value(y[:, i])
        scale = abs(float(va * exact.value(x[:, i]))) + abs(float(exact.value(y[:, i])))
        assert abs(exact.value(r[:, i]) - ex) <= Fraction(2 * 2.0 ** -BITS[K] * scale)


@pytest.mark.parametrize("K", [2, 3, 4])
@pytest.mark.parametrize("n", [0, 1, 2, 17, 1000])
def test_dot_within_bound_of_exact(K, n):
    x = synth.mp_array(K, n, 10 + n, "W")
    y = synth.mp_array(K, n, 20 + n, "W")
    r = oracle.dot(K, x, y)
    if n == 0:
        assert np.all(r == 0)
        return
    ex = exact.dot(x, y)
    err = abs(exact.value(r) - ex)
    assert err <= Fraction(_bound(K, n, exact.abs_dot(x, y)))


@pytest.mark.parametrize("K", [2, 3, 4])
def test_dot_of_integers_is_exact(K):
    rng = np.random.default_rng(7)
    n = 500
    x = np.zeros((K, n)); y = np.zeros((K, n))
    x[0] = rng.integers(-2 ** 20, 2 ** 20, n)
    y[0] = rng.integers(-2 ** 20, 2 ** 20, n)
    r = oracle.dot(K, x, y)
    assert exact.value(r) == exact.dot(x, y)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_gemv_entries_and_transpose(K):
    m, n = 37, 53
    A = synth.mp_array(K, (m, n), 30, "W")
    x = synth.mp_array(K, n, 31, "U")
    xt = synth.mp_array(K, m, 32, "U")
    y = oracle.gemv(K, A, x)
    for i in range(m):
        ex = exact.dot(A[:, i, :], x)
        assert abs(exact.value(y[:, i]) - ex) <= Fraction(_bound(K, n, exact.abs_dot(A[:, i, :], x)))
    yt = oracle.gemv(K, A, xt, trans=True)
    At = np.ascontiguousarray(A.transpose(0, 2, 1))
    assert np.array_equal(yt, oracle.gemv(K, At, xt))


@pytest.mark.parametrize("K", [2, 3, 4])
def test_gemm_small_against_exact(K):
    m, n, k = 9, 11, 29
    A = synth.mp_array(K, (m, k), 40, "W")
    B = synth.mp_array(K, (k, n), 41, "W")
    Cm = oracle.gemm(K, A, B)
    for i in range(m):
        for j in range(n):
            ex = exact.dot(A[:, i, :], B[:, :, j])
            sc = exact.abs_dot(A[:, i, :], B[:, :, j])
            assert abs(exact.value(Cm[:, i, j]) - ex) <= Fraction(_bound(K, k, sc))


@pytest.mark.parametrize("K", [2, 3, 4])
def test_gemm_is_sequential_dot_and_transposes(K):
    m, n, k = 13, 7, 19
    A = synth.mp_array(K, (m, k), 50, "U")
    B = synth.mp_array(K, (k, n), 51, "U")
    Cm = oracle.gemm(K, A, B)
    for i in range(m):
        for j in range(n):
            assert np.array_equal(Cm[:, i, j], oracle.dot(K, A[:, i, :], B[:, :, j]))
    At = np.ascontiguousarray(A.transpose(0, 2, 1))
    Bt = np.ascontiguousarray(B.transpose(0, 2, 1))
    assert np.array_equal(oracle.gemm(K, At, B, tA=True), Cm)
    assert np.array_equal(oracle.gemm(K, A, Bt, tB=True), Cm)
    assert np.array_equal(oracle.gemm(K, At, Bt, tA=True, tB=True), Cm)
    rows = np.array([0, 12, 5, 3]); cols = np.array([6, 0, 2, 6])
    e = oracle.gemm_entries(K, A, B, rows, cols)
    assert np.array_equal(e, Cm[:, rows, cols])


@pytest.mark.parametrize("K", [2, 3, 4])
def test_gemm_identity_reproduces_value(K):
    n = 12
    Id = np.zeros((K, n, n)); Id[0] = np.eye(n)
    B = synth.mp_array(K, (n, n), 60, "W")
    Cm = oracle.gemm(K, Id, B)
    for i in range(n):
        for j in range(n):
            assert exact.value(Cm[:, i, j]) == exact.value(B[:, i, j])


# Section 3.1: accuracy of the real test matrices a_ij = sqrt5 (i+j-1),
# b_ij = sqrt3 (n-i+1) is 29.0 / 45.5 / 61.7 significant digits or better.
PAPER_DIGITS = paper_values.gemm_digits("real")      # tests/golden/gemm_digits.txt


@pytest.mark.parametrize("K", [2, 3, 4])
def test_paper_real_matrices_digits(K):
    n = 48
    A, B = synth.paper_real_gemm(K, n)
    rows = np.array([0, 7, 23, 47]); cols = np.array([0, 31, 5, 47])
    got = oracle.gemm_entries(K, A, B, rows, cols)
    s15 = synth.sqrt_fraction(15, bits=400)
    for t in range(rows.size):
        S = synth.paper_real_gemm_exact(n, int(rows[t]), int(cols[t]))
        ex = s15 * S
        rel = abs(exact.value(got[:, t]) - ex) / ex
        digits = -math.log10(float(rel)) if rel > 0 else 99.0
        assert digits >= PAPER_DIGITS[K], (K, t, digits)


def test_ff_layer_against_exact():
    n = 200
    x = synth.mp_array(2, n, 70, "U", dtype=np.float32)
    y = synth.mp_array(2, n, 71, "U", dtype=np.float32)
    r = oracle.ff_dot(x, y)
    ex = exact.dot(x.astype(np.float64), y.astype(np.float64))
    sc = exact.abs_dot(x, y)
    assert abs(exact.value(r.astype(np.float64)) - ex) <= Fraction(n * 2.0 ** -46 * sc)
    z = oracle.ff_add(x, y)
    w = oracle.ff_mul(x, y)
    for i in range(n):
        assert np.array_equal(z[:, i], oracle.ff_op1("add", x[:, i], y[:, i]))
        assert np.array_equal(w[:, i], oracle.ff_op1("mul", x[:, i], y[:, i]))
    A = synth.mp_array(2, (8, 33), 72, "U", dtype=np.float32)
    B = synth.mp_array(2, (33, 5), 73, "U", dtype=np.float32)
    Cm = oracle.ff_gemm(A, B)
    for i in range(8):
        for j in range(5):
            assert np.array_equal(Cm[:, i, j], oracle.ff_dot(A[:, i, :], B[:, :, j]))
    Bt = np.ascontiguousarray(B.transpose(0, 2, 1))
    assert np.array_equal(oracle.ff_gemm(A, Bt, tB=True), Cm)
    yv = oracle.ff_gemv(A, y[:, :33])
    for i in range(8):
        assert np.array_equal(yv[:, i], oracle.ff_dot(A[:, i, :], y[:, :33]))


# Section 3.2: complex matrices a = exp(r_n)(r_u - 1/2) + i exp(r_n')(r_u' - 1/2)
# multiplied by the 3M method reach at least 23.2 / 39.2 / 55.8 significant
# digits (DD / TD / QD, minimum over real and imaginary parts, n = 2049).
PAPER_COMPLEX_DIGITS = paper_values.gemm_digits("complex")


def _complex_inputs(K, n, seed):
    mk = lambda s: synth.mp_array(K, (n, n), s, "W", phi=1.0)
    return mk(seed), mk(seed + 1), mk(seed + 2), mk(seed + 3)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_cgemm_3m_matches_definition_and_paper_digits(K):
    n = 40
    Are, Aim, Bre, Bim = _complex_inputs(K, n, 300 + K)
    Cre, Cim = oracle.cgemm_3m(K, Are, Aim, Bre, Bim)
    # the steps of eq. cgemm_3m with the oracle's own real GEMM and additions
    C1 = oracle.gemm(K, Are, Bre); C2 = oracle.gemm(K, Aim, Bim)
    SA = oracle.add(K, Are.reshape(K, -1), Aim.reshape(K, -1)).reshape(K, n, n)
    SB = oracle.add(K, Bre.reshape(K, -1), Bim.reshape(K, -1)).reshape(K, n, n)
    C3 = oracle.gemm(K, SA, SB)
    assert np.array_equal(Cre.reshape(K, -1), oracle.add(K, C1.reshape(K, -1), -C2.reshape(K, -1)))
    t = oracle.add(K, C3.reshape(K, -1), -C1.reshape(K, -1))
    assert np.array_equal(Cim.reshape(K, -1), oracle.add(K, t, -C2.reshape(K, -1)))
    # accuracy against the exact complex product (norm-wise, per part)
    worst = {"re": 0.0, "im": 0.0}
    scale = {"re": 0.0, "im": 0.0}
    for i in range(0, n, 7):
        for j in range(0, n, 5):
            ar, ai = np.ascontiguousarray(Are[:, i, :]), np.ascontiguousarray(Aim[:, i, :])
            br, bi = np.ascontiguousarray(Bre[:, :, j]), np.ascontiguousarray(Bim[:, :, j])
            ex_re = exact.dot(ar, br) - exact.dot(ai, bi)
            ex_im = exact.dot(ar, bi) + exact.dot(ai, br)
            for part, got, ex in (("re", Cre[:, i, j], ex_re), ("im", Cim[:, i, j], ex_im)):
                worst[part] = max(worst[part], abs(float(exact.value(got) - ex)))
                scale[part] = max(scale[part], abs(float(ex)))
    digits = min(-math.log10(worst[p] / scale[p]) if worst[p] else 99.0 for p in worst)
    assert digits >= PAPER_COMPLEX_DIGITS[K], (K, digits)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_cgemm_3m_entries_match_the_whole_product(K):
    """The entry-wise 3M evaluation (used at sizes where the whole product is
    too slow for the oracle) reproduces the whole-matrix one bit for bit."""
    Are, Aim = synth.mp_array(K, (9, 13), 60, "W"), synth.mp_array(K, (9, 13), 61, "W")
    Bre, Bim = synth.mp_array(K, (13, 7), 62, "W"), synth.mp_array(K, (13, 7), 63, "W")
    Cre, Cim = oracle.cgemm_3m(K, Are, Aim, Bre, Bim)
    rows, cols = np.divmod(np.arange(9 * 7), 7)
    re, im = oracle.cgemm_3m_entries(K, Are, Aim, Bre, Bim, rows, cols)
    assert np.array_equal(re.view(np.uint64), Cre.reshape(K, -1).view(np.uint64))
    assert np.array_equal(im.view(np.uint64), Cim.reshape(K, -1).view(np.uint64))
