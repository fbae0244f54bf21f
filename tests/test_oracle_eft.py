"""Pins of the oracle's EFT primitives and branch-free DD/TD/QD/FF operations
against exact rational arithmetic, the operation counts of Tables 1 and 2,
and algebraic invariants (Section 2)."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from tests import paper_values
from oracle import exact
from paper_2603_14926_amd import synth

# Relative-error ceilings (log2) for one BF operation; the BF algorithms are
# stated to be accurate to about the working precision 2^-(53K) (Section 2);
# the ceilings leave two bits of slack over that.
CEIL = {2: (-104, -103), 3: (-157, -155), 4: (-210, -208)}


def _inputs(K, n, seed):
    """Random, wide-spread and cancelling operand pairs."""
    a = synth.mp_array(K, n, seed, "U")
    b = synth.mp_array(K, n, seed + 1, "U")
    w1 = synth.mp_array(K, n, seed + 2, "W", phi=8.0)
    w2 = synth.mp_array(K, n, seed + 3, "W", phi=8.0)
    # cancellation: b = -(a with a perturbed tail)
    c1 = synth.mp_array(K, n, seed + 4, "U")
    c2 = -c1.copy()
    t = synth.mp_array(K, n, seed + 5, "U")
    c2[K - 1] = t[0] * np.abs(c1[K - 1]) + 0.0
    pairs = [(a, b), (w1, w2), (c1, c2)]
    return pairs


def test_two_sum_exact_and_error_bound():
    x = synth.mp_array(1, 4000, 11, "W", phi=10.0)[0]
    y = synth.mp_array(1, 4000, 12, "W", phi=10.0)[0]
    for a, b in zip(x, y):
        s, e = oracle.eft("two_sum", a, b)
        assert Fraction(s) + Fraction(e) == Fraction(a) + Fraction(b)
        assert s == a + b
        assert abs(e) <= exact.ulp(s) / 2


def test_quick_two_sum_exact_when_ordered():
    x = synth.mp_array(1, 4000, 13, "W", phi=10.0)[0]
    y = synth.mp_array(1, 4000, 14, "W", phi=10.0)[0]
    for a, b in zip(x, y):
        if abs(a) < abs(b):
            a, b = b, a
        s, e = oracle.eft("quick_two_sum", a, b)
        assert Fraction(s) + Fraction(e) == Fraction(a) + Fraction(b)


def test_two_prod_exact_and_unique():
    x = synth.mp_array(1, 4000, 15, "W", phi=10.0)[0]
    y = synth.mp_array(1, 4000, 16, "W", phi=10.0)[0]
    for a, b in zip(x, y):
        p, e = oracle.eft("two_prod", a, b)
        assert Fraction(p) + Fraction(e) == Fraction(a) * Fraction(b)
        assert p == a * b
        # e is the unique binary64 with p + e == a*b: the exact error is a float
        assert Fraction(e) == Fraction(a) * Fraction(b) - Fraction(p)


# Table 1 and Table 2 (BF rows) and the operation lists of DWBFAdd / DWBFMul
# (tests/golden/bf_operation_counts.txt).
COUNTS = paper_values.bf_operation_counts()


@pytest.mark.parametrize("key", sorted(COUNTS))
def test_operation_counts_match_tables(key):
    K, op = key
    assert oracle.op_counts(K, op) == COUNTS[key]


@pytest.mark.parametrize("K", [2, 3, 4])
@pytest.mark.parametrize("op", ["add", "mul"])
def test_bf_error_against_exact(K, op):
    worst = -math.inf
    for (a, b) in _inputs(K, 1500, 100 + K):
        for i in range(a.shape[1]):
            c = oracle.op1(K, op, a[:, i], b[:, i])
            va, vb = exact.value(a[:, i]), exact.value(b[:, i])
            ex = va + vb if op == "add" else va * vb
            assert exact.nonoverlapping(c), (K, op, i)
            if ex == 0:
                assert exact.value(c) == 0
                continue
            worst = max(worst, exact.log2_rel(c, ex))
    ceil = CEIL[K][0 if op == "add" else 1]
    assert worst <= ceil, (K, op, worst)
    # and the accuracy is really multicomponent (not one or two components)
    assert worst <= -(53 * K - 10)


@pytest.mark.parametrize("op", ["add", "mul"])
def test_ff_error_against_exact(op):
    a = synth.mp_array(2, 3000, 21, "U", dtype=np.float32)
    b = synth.mp_array(2, 3000, 22, "U", dtype=np.float32)
    worst = -math.inf
    for i in range(a.shape[1]):
        c = oracle.ff_op1(op, a[:, i], b[:, i])
        va, vb = exact.value(a[:, i]), exact.value(b[:, i])
        ex = va + vb if op == "add" else va * vb
        assert c[0] + c[1] == c[0]
        worst = max(worst, exact.log2_rel(c.astype(np.float64), ex))
    assert worst <= (-46 if op == "add" else -45), worst
    assert worst <= -44


@pytest.mark.parametrize("K", [2, 3, 4])
def test_bitwise_commutative_and_sign_symmetric(K):
    a = synth.mp_array(K, 400, 31, "W", phi=4.0)
    b = synth.mp_array(K, 400, 32, "W", phi=4.0)
    for op in ("add", "mul"):
        for i in range(a.shape[1]):
            ab = oracle.op1(K, op, a[:, i], b[:, i])
            ba = oracle.op1(K, op, b[:, i], a[:, i])
            assert np.array_equal(ab.view(np.int64), ba.view(np.int64))
            nn = oracle.op1(K, op, -a[:, i], -b[:, i])
            want = -ab if op == "add" else ab
            assert np.array_equal(nn, want)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_power_of_two_scaling_invariance(K):
    a = synth.mp_array(K, 300, 41, "U")
    b = synth.mp_array(K, 300, 42, "U")
    for i in range(a.shape[1]):
        s = oracle.op1(K, "add", a[:, i], b[:, i])
        s2 = oracle.op1(K, "add", a[:, i] * 2.0 ** 37, b[:, i] * 2.0 ** 37)
        assert np.array_equal(s * 2.0 ** 37, s2)
        p = oracle.op1(K, "mul", a[:, i], b[:, i])
        p2 = oracle.op1(K, "mul", a[:, i] * 2.0 ** 20, b[:, i] * 2.0 ** -9)
        assert np.array_equal(p * 2.0 ** 11, p2)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_zero_tail_reduces_to_eft(K):
    """With zero lower components the BF add / mul return the TwoSum /
    TwoProd pair (textbook special case)."""
    x = synth.mp_array(1, 500, 51, "W", phi=6.0)[0]
    y = synth.mp_array(1, 500, 52, "W", phi=6.0)[0]
    for a0, b0 in zip(x, y):
        a = np.zeros(K); b = np.zeros(K)
        a[0], b[0] = a0, b0
        s = oracle.op1(K, "add", a, b)
        ts = oracle.eft("two_sum", a0, b0)
        assert exact.value(s) == Fraction(ts[0]) + Fraction(ts[1])
        assert s[0] == ts[0]
        p = oracle.op1(K, "mul", a, b)
        tp = oracle.eft("two_prod", a0, b0)
        assert exact.value(p) == Fraction(tp[0]) + Fraction(tp[1])
        assert p[0] == tp[0]


@pytest.mark.parametrize("K", [2, 3, 4])
def test_small_integers_are_exact(K):
    rng = np.random.default_rng(5)
    for _ in range(300):
        a = np.zeros(K); b = np.zeros(K)
        # |a| < 2^30 with a tail below 2^-30: the exact sum spans < 106 bits,
        # the exact product < 140 bits, so TD and QD must represent it exactly.
        a[0] = float(rng.integers(-2 ** 30, 2 ** 30))
        b[0] = float(rng.integers(-2 ** 30, 2 ** 30))
        a[1] = float(rng.integers(-1000, 1000)) * 2.0 ** -40
        b[1] = float(rng.integers(-1000, 1000)) * 2.0 ** -40
        s = oracle.op1(K, "add", a, b)
        assert exact.value(s) == exact.value(a) + exact.value(b)
        p = oracle.op1(K, "mul", a, b)
        if K >= 3:
            assert exact.value(p) == exact.value(a) * exact.value(b)
