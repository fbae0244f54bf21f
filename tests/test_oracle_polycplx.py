"""Pins of the oracle's real-coefficient polynomial evaluation at complex
arguments (Section 4.1, second benchmark), Horner and Estrin: exact rational
evaluation, conjugate symmetry, reduction to the real-argument evaluators on
the real axis, and the closed forms at degree 0 and 1."""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_2603_14926_amd import synth

BITS = {2: 104, 3: 155, 4: 208}


def _exact_eval(a, zr, zi):
    """Exact p(z) = sum a_i z^i for rational coefficients and point."""
    pr, pi = Fraction(0), Fraction(0)
    for ai in reversed(a):
        pr, pi = pr * zr - pi * zi + ai, pr * zi + pi * zr
    return pr, pi


@pytest.mark.parametrize("K", [2, 3, 4])
@pytest.mark.parametrize("method", ["horner", "estrin"])
def test_against_exact_evaluation(K, method):
    deg, batch = 21, 12
    coef = synth.mp_array(K, (batch, deg + 1), 5 + K, "U")
    xr = synth.mp_array(K, batch, 6 + K, "U")
    xi = synth.mp_array(K, batch, 7 + K, "U")
    yr, yi = oracle.polyval_cplx(K, coef, xr, xi, method)
    for b in range(batch):
        a = [exact.value(coef[:, b, i]) for i in range(deg + 1)]
        zr, zi = exact.value(xr[:, b]), exact.value(xi[:, b])
        er, ei = _exact_eval(a, zr, zi)
        absz = abs(complex(float(zr), float(zi)))
        scale = sum(abs(float(ai)) * absz ** i for i, ai in enumerate(a))
        tol = Fraction(8 * (deg + 1) * 2.0 ** -BITS[K] * scale)
        assert abs(exact.value(yr[:, b]) - er) <= tol, b
        assert abs(exact.value(yi[:, b]) - ei) <= tol, b


@pytest.mark.parametrize("K", [2, 3, 4])
@pytest.mark.parametrize("method", ["horner", "estrin"])
def test_conjugate_symmetry_and_real_axis(K, method):
    coef = synth.mp_array(K, (40, 37), 20 + K, "W")
    xr = synth.mp_array(K, 40, 21 + K, "U")
    xi = synth.mp_array(K, 40, 22 + K, "U")
    yr, yi = oracle.polyval_cplx(K, coef, xr, xi, method)
    cr, ci = oracle.polyval_cplx(K, coef, xr, -xi, method)
    assert np.array_equal(cr, yr) and np.array_equal(ci, -yi)
    # on the real axis the evaluation is the real-argument one, bit for bit
    rr, ri = oracle.polyval_cplx(K, coef, xr, np.zeros_like(xi), method)
    real = oracle.polyval(K, coef, xr) if method == "horner" else oracle.polyval_estrin(K, coef, xr)
    assert np.array_equal(rr, real) and np.all(ri == 0)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_degree_zero_and_one_closed_forms(K):
    coef0 = synth.mp_array(K, (5, 1), 30, "U")
    xr = synth.mp_array(K, 5, 31, "U")
    xi = synth.mp_array(K, 5, 32, "U")
    for method in ("horner", "estrin"):
        yr, yi = oracle.polyval_cplx(K, coef0, xr, xi, method)
        assert np.array_equal(yr, coef0[:, :, 0]) and np.all(yi == 0)
    coef1 = synth.mp_array(K, (5, 2), 33, "U")
    yr, yi = oracle.polyval_cplx(K, coef1, xr, xi, "estrin")
    for b in range(5):
        a0, a1 = coef1[:, b, 0], coef1[:, b, 1]
        want_r = oracle.op1(K, "add", a0, oracle.op1(K, "mul", a1, xr[:, b]))
        want_i = oracle.op1(K, "mul", a1, xi[:, b])
        assert np.array_equal(yr[:, b], want_r) and np.array_equal(yi[:, b], want_i)


@pytest.mark.parametrize("K", [3, 4])
def test_estrin_and_horner_agree_within_bound(K):
    deg, batch = 300, 8
    coef = synth.mp_array(K, (batch, deg + 1), 40 + K, "U")
    xr = synth.mp_array(K, batch, 41 + K, "U") * 0.7
    xi = synth.mp_array(K, batch, 42 + K, "U") * 0.7
    hr, hi = oracle.polyval_cplx(K, coef, xr, xi, "horner")
    er, ei = oracle.polyval_cplx(K, coef, xr, xi, "estrin")
    for b in range(batch):
        absz = abs(complex(xr[0, b], xi[0, b]))
        scale = sum(abs(coef[0, b, i]) * absz ** i for i in range(deg + 1))
        tol = 16 * (deg + 1) * 2.0 ** -BITS[K] * scale
        assert abs(float(exact.value(hr[:, b]) - exact.value(er[:, b]))) <= tol
        assert abs(float(exact.value(hi[:, b]) - exact.value(ei[:, b]))) <= tol
