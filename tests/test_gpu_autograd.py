"""GPU checks of the hand-written backward passes behind torch.autograd:
QD / DD GEMM (dA = dC B^T, dB = A^T dC) and Horner (coefficient and x
gradients), against the oracle gradient (bit-exact: same kernels' sequential
order) and against central finite differences evaluated by the oracle in
the same precision (the GEMM and the coefficient map are linear, so the
difference quotient has no truncation error; for the x-gradient the step is
small enough that its truncation error lies far below the tolerance)."""
from fractions import Fraction

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle import exact
from paper_2603_14926_amd import autograd as ag
from paper_2603_14926_amd import mpx, synth
from tests.gpu_util import bits_equal, to_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("p,K", [("qd", 4), ("dd", 2), ("td", 3)])
@pytest.mark.parametrize("mnk", [(33, 47, 29), (128, 64, 96)])
def test_gemm_backward_matches_oracle_gradient(p, K, mnk):
    m, n, k = mnk
    A = synth.mp_array(K, (m, k), 1, "U")
    B = synth.mp_array(K, (k, n), 2, "U")
    G = synth.mp_array(K, (m, n), 3, "U")
    tA = to_gpu(A).requires_grad_(True)
    tB = to_gpu(B).requires_grad_(True)
    Cm = ag.gemm(tA, tB, p)
    Cm.backward(to_gpu(G))
    assert bits_equal(to_np(Cm.detach()), oracle.gemm(K, A, B))
    Bt = np.ascontiguousarray(B.transpose(0, 2, 1))
    At = np.ascontiguousarray(A.transpose(0, 2, 1))
    assert bits_equal(to_np(tA.grad), oracle.gemm(K, G, Bt))
    assert bits_equal(to_np(tB.grad), oracle.gemm(K, At, G))


def _qd_scalar_mul(K, a, s):
    return oracle.op1(K, "mul", a, np.array([s] + [0.0] * (K - 1)))


def test_gemm_backward_finite_differences_qd():
    """dL/dA_il for L = sum_ij G_ij C_ij by central differences in QD:
    only row i of C changes, C(A +- h e_il) row = (A_i +- h e_l) B."""
    K, m, n, k = 4, 6, 9, 11
    A = synth.mp_array(K, (m, k), 4, "U")
    B = synth.mp_array(K, (k, n), 5, "U")
    G = synth.mp_array(K, (m, n), 6, "U")
    tA = to_gpu(A).requires_grad_(True)
    tB = to_gpu(B).requires_grad_(True)
    ag.gemm(tA, tB, "qd").backward(to_gpu(G))
    dA, dB = to_np(tA.grad), to_np(tB.grad)
    h = 2.0 ** -40
    for (i, l) in ((0, 0), (3, 7), (5, 10)):
        rows = []
        for sgn in (1, -1):
            Ap = A[:, i:i + 1, :].copy()
            Ap[:, 0, l] = oracle.op1(K, "add", Ap[:, 0, l], np.array([sgn * h] + [0.0] * (K - 1)))
            rows.append(oracle.gemm(K, Ap, B)[:, 0, :])
        diff = oracle.add(K, rows[0], -rows[1])
        fd = oracle.dot(K, G[:, i, :], diff)
        fd = fd / (2 * h)   # exact power-of-two scaling
        want = exact.value(fd)
        got = exact.value(dA[:, i, l])
        assert abs(got - want) <= abs(want) * Fraction(2.0 ** -150) + Fraction(2.0 ** -180)
    # dB_lj = sum_i A_il G_ij (oracle gradient, exact check of one entry)
    ex = exact.dot(np.ascontiguousarray(A[:, :, 2]), np.ascontiguousarray(G[:, :, 4]))
    assert abs(exact.value(dB[:, 2, 4]) - ex) <= Fraction(m * 2.0 ** -208) * Fraction(exact.abs_dot(A[:, :, 2], G[:, :, 4]))


@pytest.mark.parametrize("p,K", [("qd", 4), ("dd", 2)])
def test_gemm_backward_2048_sampled(p, K):
    """config size: QD and DD GEMM 2048 forward + backward through autograd,
    sampled entries of C, dA, dB checked bit for bit against the oracle."""
    n = 2048
    A = synth.mp_array(K, (n, n), synth.seed_for(3, 0), "U")
    B = synth.mp_array(K, (n, n), synth.seed_for(3, 1), "U")
    G = synth.mp_array(K, (n, n), synth.seed_for(3, 2), "U")
    tA = to_gpu(A).requires_grad_(True)
    tB = to_gpu(B).requires_grad_(True)
    Cm = ag.gemm(tA, tB, p)
    Cm.backward(to_gpu(G))
    rows = np.array([0, 17, 1024, 2047]); cols = np.array([5, 2047, 1023, 0])
    assert bits_equal(to_np(Cm.detach())[:, rows, cols], oracle.gemm_entries(K, A, B, rows, cols))
    Bt = np.ascontiguousarray(B.transpose(0, 2, 1))
    At = np.ascontiguousarray(A.transpose(0, 2, 1))
    assert bits_equal(to_np(tA.grad)[:, rows, cols], oracle.gemm_entries(K, G, B, rows, cols, tB=True))
    assert bits_equal(to_np(tB.grad)[:, rows, cols], oracle.gemm_entries(K, A, G, rows, cols, tA=True))
    del At, Bt


@pytest.mark.parametrize("p,K", [("qd", 4), ("dd", 2)])
def test_polyval_autograd(p, K):
    batch, deg = 1024, 1024
    coef = synth.mp_array(K, (batch, deg + 1), synth.seed_for(3, 10), "U")
    x = synth.mp_array(K, batch, synth.seed_for(3, 11), "U")
    g = synth.mp_array(K, batch, synth.seed_for(3, 12), "U")
    tc = to_gpu(coef).requires_grad_(True)
    tx = to_gpu(x).requires_grad_(True)
    y = ag.polyval(tc, tx, p)
    y.backward(to_gpu(g))
    wc, wx = oracle.polyval_backward(K, coef, x, g)
    assert bits_equal(to_np(y.detach()), oracle.polyval(K, coef, x))
    assert bits_equal(to_np(tc.grad), wc)
    assert bits_equal(to_np(tx.grad), wx)


def test_polyval_coefficient_gradient_finite_differences():
    """p is linear in its coefficients: (p(a + h e_i) - p(a - h e_i)) / 2h = x^i
    exactly up to QD rounding."""
    K, batch, deg = 4, 4, 30
    coef = synth.mp_array(K, (batch, deg + 1), 20, "U")
    x = synth.mp_array(K, batch, 21, "U")
    g = np.zeros((K, batch)); g[0] = 1.0
    tc = to_gpu(coef).requires_grad_(True)
    ag.polyval(tc, to_gpu(x), "qd").backward(to_gpu(g))
    grad = to_np(tc.grad)
    h = 2.0 ** -30
    for b, i in ((0, 0), (1, 7), (3, 30)):
        ys = []
        for sgn in (1, -1):
            c2 = coef.copy()
            c2[:, b, i] = oracle.op1(K, "add", c2[:, b, i], np.array([sgn * h, 0, 0, 0.0]))
            ys.append(oracle.polyval(K, c2, x)[:, b])
        fd = oracle.op1(K, "add", ys[0], -ys[1]) / (2 * h)
        want = exact.value(fd)
        got = exact.value(grad[:, b, i])
        assert abs(got - want) <= Fraction(2.0 ** -160) * (1 + abs(want))


def test_polyval_x_gradient_finite_differences_and_exact_derivative():
    """x-gradient of Horner in QD against (i) central differences
    (p(x + h) - p(x - h)) / 2h evaluated by the oracle in QD with h = 2^-70,
    whose truncation error h^2 |p'''| / 6 stays below 2^-120 relative, and
    (ii) the exact derivative sum_i i a_i x^(i-1) in rational arithmetic."""
    K, batch, deg = 4, 6, 30
    coef = synth.mp_array(K, (batch, deg + 1), 22, "U")
    x = synth.mp_array(K, batch, 23, "U")
    g = np.zeros((K, batch)); g[0] = 1.0
    tx = to_gpu(x).requires_grad_(True)
    ag.polyval(to_gpu(coef), tx, "qd").backward(to_gpu(g))
    gx = to_np(tx.grad)
    h = 2.0 ** -70
    step = np.array([h, 0.0, 0.0, 0.0])
    xp = np.stack([oracle.op1(K, "add", x[:, b], step) for b in range(batch)], 1)
    xm = np.stack([oracle.op1(K, "add", x[:, b], -step) for b in range(batch)], 1)
    yp, ym = oracle.polyval(K, coef, xp), oracle.polyval(K, coef, xm)
    for b in range(batch):
        fd = oracle.op1(K, "add", yp[:, b], -ym[:, b]) / (2 * h)   # exact power-of-two scaling
        want = exact.value(fd)
        got = exact.value(gx[:, b])
        assert abs(got - want) <= Fraction(2.0 ** -120) * (1 + abs(want)), b
        xv = exact.value(x[:, b])
        terms = [i * exact.value(coef[:, b, i]) * xv ** (i - 1) for i in range(1, deg + 1)]
        d = sum(terms)
        assert abs(got - d) <= Fraction(2.0 ** -200) * (1 + sum(abs(t) for t in terms)), b


@pytest.mark.parametrize("p,K", [("qd", 4), ("dd", 2)])
def test_plain_torch_loss_through_to_value(p, K):
    """A loss built from plain torch operations reaches the multicomponent
    backward through to_value(): the cotangent is (1, 0, ..., 0) per entry,
    so A.grad = ones B^T and B.grad = A^T ones, bit for bit; summing the raw
    planes instead hands in the number K (the documented convention)."""
    m, n, k = 19, 23, 31
    A = synth.mp_array(K, (m, k), 41, "U")
    B = synth.mp_array(K, (k, n), 42, "U")
    ones = np.zeros((K, m, n)); ones[0] = 1.0
    Bt = np.ascontiguousarray(B.transpose(0, 2, 1))
    At = np.ascontiguousarray(A.transpose(0, 2, 1))
    tA = to_gpu(A).requires_grad_(True)
    tB = to_gpu(B).requires_grad_(True)
    ag.to_value(ag.gemm(tA, tB, p)).sum().backward()
    assert bits_equal(to_np(tA.grad), oracle.gemm(K, ones, Bt))
    assert bits_equal(to_np(tB.grad), oracle.gemm(K, At, ones))
    tA2 = to_gpu(A).requires_grad_(True)
    ag.gemm(tA2, to_gpu(B), p).sum().backward()
    # every plane's gradient 1 is read as one multicomponent cotangent, the number K
    assert bits_equal(to_np(tA2.grad), oracle.gemm(K, np.ones((K, m, n)), Bt))
    assert np.allclose(to_np(tA2.grad)[0], K * to_np(tA.grad)[0], rtol=1e-12, atol=0)
