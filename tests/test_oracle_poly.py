"""Pins of the oracle's polynomial layer: Horner evaluation and its backward
(Section 4.1), Newton division, and the Durand-Kerner iteration with the
Aberth start (Section 4.2), against exact rationals and closed forms."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_2603_14926_amd import synth

BITS = {2: 104, 3: 155, 4: 208}


@pytest.mark.parametrize("K", [2, 3, 4])
def test_polyval_against_exact(K):
    batch, deg = 6, 25
    coef = synth.mp_array(K, (batch, deg + 1), 1, "U")
    x = synth.mp_array(K, batch, 2, "U")
    y = oracle.polyval(K, coef, x)
    for b in range(batch):
        xs = exact.value(x[:, b])
        cs = [exact.value(coef[:, b, i]) for i in range(deg + 1)]
        ex = exact.horner_real(cs, xs)
        scale = sum(abs(float(c)) * abs(float(xs)) ** i for i, c in enumerate(cs))
        assert abs(exact.value(y[:, b]) - ex) <= Fraction(2 * deg * 2.0 ** -BITS[K] * scale)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_polyval_backward_against_exact(K):
    batch, deg = 5, 20
    coef = synth.mp_array(K, (batch, deg + 1), 3, "U")
    x = synth.mp_array(K, batch, 4, "U")
    g = synth.mp_array(K, batch, 5, "U")
    gc, gx = oracle.polyval_backward(K, coef, x, g)
    for b in range(batch):
        xs, gs = exact.value(x[:, b]), exact.value(g[:, b])
        for i in range(deg + 1):
            ex = gs * xs ** i
            assert abs(exact.value(gc[:, b, i]) - ex) <= abs(ex) * Fraction((i + 1) * 2.0 ** -BITS[K])
        cs = [exact.value(coef[:, b, i]) for i in range(deg + 1)]
        dp = sum(i * cs[i] * xs ** (i - 1) for i in range(1, deg + 1))
        scale = sum(i * abs(float(cs[i])) * abs(float(xs)) ** (i - 1) for i in range(1, deg + 1))
        ex = gs * dp
        assert abs(exact.value(gx[:, b]) - ex) <= Fraction(4 * deg * 2.0 ** -BITS[K] * scale * abs(float(gs)))


def test_polyval_backward_degree_zero():
    K = 4
    coef = synth.mp_array(K, (3, 1), 6, "U")
    x = synth.mp_array(K, 3, 7, "U")
    g = synth.mp_array(K, 3, 8, "U")
    gc, gx = oracle.polyval_backward(K, coef, x, g)
    assert np.array_equal(gc[:, :, 0], g)
    assert np.all(gx == 0)
    assert np.array_equal(oracle.polyval(K, coef, x), coef[:, :, 0])


@pytest.mark.parametrize("K", [2, 3, 4])
def test_newton_reciprocal(K):
    d = synth.mp_array(K, 300, 9, "W", phi=6.0)
    for i in range(300):
        if d[0, i] == 0:
            continue
        y = oracle.recip(K, d[:, i])
        err = abs(exact.value(y) * exact.value(d[:, i]) - 1)
        assert err <= Fraction(2.0 ** -(BITS[K] - 2)), (K, i, float(err))


@pytest.mark.parametrize("K", [2, 3, 4])
def test_complex_division(K):
    q = [synth.mp_array(K, 200, 10 + t, "U") for t in range(4)]
    for i in range(200):
        zr, zi = oracle.cdiv(K, q[0][:, i], q[1][:, i], q[2][:, i], q[3][:, i])
        a = (exact.value(q[0][:, i]), exact.value(q[1][:, i]))
        b = (exact.value(q[2][:, i]), exact.value(q[3][:, i]))
        den = b[0] ** 2 + b[1] ** 2
        ex = ((a[0] * b[0] + a[1] * b[1]) / den, (a[1] * b[0] - a[0] * b[1]) / den)
        mag = math.hypot(float(ex[0]), float(ex[1]))
        tol = Fraction(16 * 2.0 ** -BITS[K] * mag)
        assert abs(exact.value(zr) - ex[0]) <= tol
        assert abs(exact.value(zi) - ex[1]) <= tol


def _exact_monic(K, are, aim):
    n = are.shape[1] - 1
    A = [(exact.value(are[:, i]), exact.value(aim[:, i])) for i in range(n + 1)]
    an = A[n]
    den = an[0] ** 2 + an[1] ** 2
    return [((a[0] * an[0] + a[1] * an[1]) / den, (a[1] * an[0] - a[0] * an[1]) / den) for a in A[:n]]


@pytest.mark.parametrize("K", [2, 3, 4])
def test_dk_one_sweep_against_exact(K):
    """One Jacobi sweep z_i - q(z_i)/prod_{j!=i}(z_i - z_j) (equation for the
    DK iteration), every term evaluated exactly from the same iterate."""
    n = 5
    are = synth.mp_array(K, n + 1, 20, "N")
    aim = synth.mp_array(K, n + 1, 21, "N")
    zr = synth.mp_array(K, n, 22, "U") * 1.5
    zi = synth.mp_array(K, n, 23, "U") * 1.5
    deg = np.array([n], np.int32)
    nr, ni, st = oracle.polyroots(K, deg, are, aim, zr, zi, iters=1, init=False)
    assert st[0] == 0
    c = _exact_monic(K, are, aim) + [(Fraction(1), Fraction(0))]
    Z = [(exact.value(zr[:, i]), exact.value(zi[:, i])) for i in range(n)]
    for i in range(n):
        q = exact.cpoly(c, Z[i])
        P = (Fraction(1), Fraction(0))
        for j in range(n):
            if j != i:
                P = exact.cmul(P, (Z[i][0] - Z[j][0], Z[i][1] - Z[j][1]))
        den = P[0] ** 2 + P[1] ** 2
        w = ((q[0] * P[0] + q[1] * P[1]) / den, (q[1] * P[0] - q[0] * P[1]) / den)
        ex = (Z[i][0] - w[0], Z[i][1] - w[1])
        mag = math.hypot(float(ex[0]), float(ex[1])) + math.hypot(float(w[0]), float(w[1]))
        tol = Fraction(2.0 ** -(BITS[K] - 14) * mag)
        assert abs(exact.value(nr[:, i]) - ex[0]) <= tol, (K, i)
        assert abs(exact.value(ni[:, i]) - ex[1]) <= tol, (K, i)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_dk_horner_rescaled_value(K):
    n = 40
    cre = synth.mp_array(K, n, 30, "N")
    cim = synth.mp_array(K, n, 31, "N")
    zr = synth.mp_array(K, 4, 32, "U") * 6.0
    zi = synth.mp_array(K, 4, 33, "U") * 6.0
    qr, qi, E = oracle.dk_horner(K, cre, cim, zr, zi)
    c = [(exact.value(cre[:, i]), exact.value(cim[:, i])) for i in range(n)] + [(Fraction(1), Fraction(0))]
    for t in range(4):
        z = (exact.value(zr[:, t]), exact.value(zi[:, t]))
        ex = exact.cpoly(c, z)
        got = (exact.value(qr[:, t]) * Fraction(2) ** int(E[t]), exact.value(qi[:, t]) * Fraction(2) ** int(E[t]))
        az = math.hypot(float(z[0]), float(z[1]))
        scale = sum(math.hypot(float(a), float(b)) * az ** i for i, (a, b) in enumerate(c))
        tol = Fraction(8 * n * 2.0 ** -BITS[K] * scale)
        assert abs(got[0] - ex[0]) <= tol and abs(got[1] - ex[1]) <= tol
        # the rescaled leading component lies below 1 (rescaling only scales down)
        assert max(abs(qr[0, t]), abs(qi[0, t])) < 1.0 and E[t] >= 0


def test_aberth_start_geometry():
    """Start values lie on a circle of the stated radius around -c_{n-1}/n with
    angles 2(i-1)pi/n + 3/(2n) (equation for the Aberth initial values)."""
    K, n = 4, 12
    are = synth.mp_array(K, n + 1, 40, "N")
    aim = synth.mp_array(K, n + 1, 41, "N")
    zr, zi, st = oracle.polyroots(K, np.array([n], np.int32), are, aim, iters=0, init=True)
    cre, cim = oracle.dk_monic(K, are, aim)
    c = cre[0] + 1j * cim[0]
    centre = -c[n - 1] / n
    r = max(abs(n * c[i]) ** (1.0 / (n - i)) for i in range(n))
    z = zr[0] + 1j * zi[0]
    assert np.allclose(np.abs(z - centre), r, rtol=1e-13)
    ang = np.angle((z - centre) / r)
    want = np.angle(np.exp(1j * (2 * np.pi * np.arange(n) / n + 3.0 / (2 * n))))
    assert np.allclose(np.exp(1j * ang), np.exp(1j * want), atol=1e-12)
    assert np.all(zr[1:] == 0) and np.all(zi[1:] == 0)
    # every true root lies inside the start circle's bounding radius 2r
    roots = np.roots((c.tolist() + [1.0])[::-1])
    assert np.all(np.abs(roots - centre) <= 2 * r + np.abs(centre))


# Chebyshev integration (Section 4.2): the nodes for n = 2..5 are classical.
CHEB_NODES = {
    2: [-1 / math.sqrt(3), 1 / math.sqrt(3)],
    3: [-1 / math.sqrt(2), 0.0, 1 / math.sqrt(2)],
    4: [-0.7946544722917661, -0.1875924740850799, 0.1875924740850799, 0.7946544722917661],
    5: [-0.8324974870009819, -0.3745414095535811, 0.0, 0.3745414095535811, 0.8324974870009819],
}


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_chebyshev_roots(n):
    K = 4
    a = synth.chebyshev_coefficients(n)
    are = np.stack([synth.round_greedy(v, K) for v in a], axis=1)
    aim = np.zeros_like(are)
    zr, zi, st = oracle.polyroots(K, np.array([n], np.int32), are, aim, iters=120, init=True)
    assert st[0] == 0
    got = sorted(zr[0] + 1j * zi[0], key=lambda v: v.real)
    for g, w in zip(got, CHEB_NODES[n]):
        assert abs(g.real - w) < 1e-14 and abs(g.imag) < 1e-14
    # and at QD level: the computed roots annihilate the exact polynomial
    for i in range(n):
        z = (exact.value(zr[:, i]), exact.value(zi[:, i]))
        q = exact.cpoly([(v, Fraction(0)) for v in a], z)
        assert math.hypot(float(q[0]), float(q[1])) < 1e-58


def test_chebyshev_coefficients_closed_form():
    # x^2 - 1/3 ; x^3 - x/2 ; x^4 - 2/3 x^2 + 1/45 (textbook Chebyshev quadrature)
    assert synth.chebyshev_coefficients(2) == [Fraction(-1, 3), 0, 1]
    assert synth.chebyshev_coefficients(3) == [0, Fraction(-1, 2), 0, 1]
    assert synth.chebyshev_coefficients(4) == [Fraction(1, 45), 0, Fraction(-2, 3), 0, 1]


def test_known_root_polynomials_converge():
    K = 4
    deg, cre, cim, known = synth.dk_batch(K, 3, 16, 16, seed=77, n_known=3, known_degree=16)
    zr, zi, st = oracle.polyroots(K, deg, cre, cim, iters=200, init=True)
    assert np.all(st == 0)
    coff, roff = synth.offsets(deg)
    for b in range(3):
        z = zr[0, roff[b]:roff[b + 1]] + 1j * zi[0, roff[b]:roff[b + 1]]
        for r in known[b]:
            assert np.min(np.abs(z - r)) < 1e-13


def test_polyroots_status_flags_coincident_start():
    K = 2
    are = synth.mp_array(K, 4, 50, "N")
    aim = synth.mp_array(K, 4, 51, "N")
    zr = np.zeros((K, 3)); zi = np.zeros((K, 3))
    zr[0] = [0.5, 0.5, -0.3]           # two coincident start values
    _, _, st = oracle.polyroots(K, np.array([3], np.int32), are, aim, zr, zi, iters=2, init=False)
    assert st[0] == 1


@pytest.mark.parametrize("K", [2, 3, 4])
@pytest.mark.parametrize("deg", [0, 1, 2, 5, 31, 100])
def test_estrin_against_exact(K, deg):
    batch = 4
    coef = synth.mp_array(K, (batch, deg + 1), 70 + deg, "U")
    x = synth.mp_array(K, batch, 71 + deg, "U")
    y = oracle.polyval_estrin(K, coef, x)
    for b in range(batch):
        xs = exact.value(x[:, b])
        cs = [exact.value(coef[:, b, i]) for i in range(deg + 1)]
        ex = exact.horner_real(cs, xs)
        scale = sum(abs(float(c)) * abs(float(xs)) ** i for i, c in enumerate(cs))
        levels = max(1, (deg).bit_length())
        assert abs(exact.value(y[:, b]) - ex) <= Fraction(4 * levels * 2.0 ** -BITS[K] * scale)


def test_estrin_small_cases_by_hand():
    """deg 1: a0 + a1 x; deg 2 (padded to 4): (a0 + a1 x) + (a2 + 0 x) x^2."""
    K = 2
    coef = np.zeros((K, 1, 3)); coef[0, 0] = [1.5, -2.0, 0.25]
    x = np.zeros((K, 1)); x[0, 0] = 3.0
    assert oracle.polyval_estrin(K, coef, x)[0, 0] == 1.5 - 6.0 + 0.25 * 9.0
    assert oracle.polyval_estrin(K, coef[:, :, :2], x)[0, 0] == 1.5 - 6.0
