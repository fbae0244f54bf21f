"""Pins of the oracle's conventional ("NoBF") arithmetic, the baseline the
paper measures its branch-free algorithms against (Sections 2.1-2.3):
DWAdd, DWAccurateAdd and DWMul as printed, TWAdd / TWMul, their
four-component forms, and the TW/QW renormalisation.  Checked against exact
rational arithmetic, the published error bound of the accurate double-word
addition, hand-derived renormalisation cases and algebraic invariants."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_2603_14926_amd import synth
from tests.test_oracle_eft import _inputs

# log2 ceilings of the relative error of one operation (the BF ceilings):
# the conventional TD / QD operations keep the working precision 2^-(53K).
CEIL = {3: (-157, -155), 4: (-210, -208)}


def _err(K, op, a, b, c):
    va, vb = exact.value(a), exact.value(b)
    ex = va + vb if op == "add" else va * vb
    return abs(exact.value(c) - ex), ex, (abs(va) + abs(vb) if op == "add" else abs(va * vb))


def test_dw_mul_is_the_bf_mul_sequence():
    """DWMul (the QD default) and DWBFMul perform the same operations; the
    only difference is the order of the two operands of one addition, so the
    results are bit-identical."""
    for a, b in _inputs(2, 3000, 500):
        with oracle.arith("nobf"):
            conv = oracle.mul(2, a, b)
        assert np.array_equal(conv, oracle.mul(2, a, b))


def test_dw_operation_counts_follow_the_printed_algorithms():
    # DWAdd: TwoSum (2 add, 4 sub) + 2 add + QuickTwoSum (1 add, 2 sub)
    # DWAccurateAdd: 2 TwoSum + 2 add + 2 QuickTwoSum
    # DWMul: TwoProd (1 mul, 1 fma) + 2 mul + 2 add + QuickTwoSum
    a = synth.mp_array(2, 1, 7, "U")[:, 0]
    b = synth.mp_array(2, 1, 8, "U")[:, 0]
    with oracle.arith("nobf"):
        assert oracle.op_counts(2, "add", a, b) == (5, 6, 0, 0)
        assert oracle.op_counts(2, "mul", a, b) == (3, 2, 3, 1)
    with oracle.arith("nobf_acc"):
        assert oracle.op_counts(2, "add", a, b) == (8, 12, 0, 0)


def test_dw_sloppy_add_bound_and_cancellation():
    """DWAdd is accurate relative to |a| + |b| but not to |a + b|: the hand
    case a = 1 + 2^-60, b = -1 + 2^-113 loses the 2^-113 (relative error
    2^-53), which DWAccurateAdd keeps."""
    worst = -999.0
    for a, b in _inputs(2, 2000, 600):
        with oracle.arith("nobf"):
            c = oracle.add(2, a, b)
        for i in range(a.shape[1]):
            err, _, sc = _err(2, "add", a[:, i], b[:, i], c[:, i])
            if err:
                worst = max(worst, math.log2(err / sc))
    assert worst <= -104
    a = np.array([1.0, 2.0 ** -60])
    b = np.array([-1.0, 2.0 ** -113])
    with oracle.arith("nobf"):
        sl = oracle.op1(2, "add", a, b)
    with oracle.arith("nobf_acc"):
        ac = oracle.op1(2, "add", a, b)
    assert list(sl) == [2.0 ** -60, 0.0]
    assert list(ac) == [2.0 ** -60, 2.0 ** -113]


def test_dw_accurate_add_relative_bound():
    """DWAccurateAdd: relative error at most 3u^2 / (1 - 4u), u = 2^-53
    (Joldes, Muller and Popescu, ACM TOMS 44(2), 2017), cancellation
    included."""
    bound = Fraction(3, 2 ** 106) / (1 - Fraction(4, 2 ** 53))
    for a, b in _inputs(2, 2000, 700):
        with oracle.arith("nobf_acc"):
            c = oracle.add(2, a, b)
        for i in range(a.shape[1]):
            err, ex, _ = _err(2, "add", a[:, i], b[:, i], c[:, i])
            assert err <= bound * abs(ex), i


@pytest.mark.parametrize("K", [3, 4])
@pytest.mark.parametrize("op", ["add", "mul"])
def test_tw_qw_conventional_error_and_nonoverlap(K, op):
    lim = CEIL[K][0 if op == "add" else 1]
    worst = -999.0
    for a, b in _inputs(K, 1200, 800 + K):
        with oracle.arith("nobf"):
            c = (oracle.add if op == "add" else oracle.mul)(K, a, b)
        for i in range(a.shape[1]):
            err, ex, _ = _err(K, op, a[:, i], b[:, i], c[:, i])
            assert exact.nonoverlapping(c[:, i]), i
            if err:
                worst = max(worst, math.log2(err / abs(ex)))
    assert worst <= lim, worst


@pytest.mark.parametrize("K", [2, 3, 4])
@pytest.mark.parametrize("mode", ["nobf", "nobf_acc"])
def test_conventional_invariants(K, mode):
    """Addition is bitwise commutative; both operations are odd in each
    operand and invariant under power-of-two scaling."""
    a = synth.mp_array(K, 400, 900 + K, "W", phi=6.0)
    b = synth.mp_array(K, 400, 950 + K, "W", phi=6.0)
    with oracle.arith(mode):
        s = oracle.add(K, a, b)
        assert np.array_equal(s, oracle.add(K, b, a))
        assert np.array_equal(-s, oracle.add(K, -a, -b))
        p = oracle.mul(K, a, b)
        assert np.array_equal(-p, oracle.mul(K, -a, b))
        assert np.array_equal(p, oracle.mul(K, -a, -b))
        assert np.array_equal(s * 2.0 ** 40, oracle.add(K, a * 2.0 ** 40, b * 2.0 ** 40))
        assert np.array_equal(p * 2.0 ** -70, oracle.mul(K, a * 2.0 ** -30, b * 2.0 ** -40))


@pytest.mark.parametrize("K", [2, 3, 4])
def test_conventional_zero_tail_reduces_to_eft(K):
    x = synth.mp_array(1, 300, 41, "W", phi=8.0)[0]
    y = synth.mp_array(1, 300, 42, "W", phi=8.0)[0]
    with oracle.arith("nobf"):
        for u, v in zip(x, y):
            a = np.zeros(K); a[0] = u
            b = np.zeros(K); b[0] = v
            s, e = oracle.eft("two_sum", u, v)
            c = oracle.op1(K, "add", a, b)
            assert exact.value(c) == Fraction(u) + Fraction(v)
            assert c[0] == s and np.all(c[2:] == 0)
            p, pe = oracle.eft("two_prod", u, v)
            c = oracle.op1(K, "mul", a, b)
            assert c[0] == p and c[1] == pe and np.all(c[2:] == 0)


def test_renormalize_hand_cases():
    """Hand-traced cases of the two-pass renormalisation, including the
    zero-error path that skips an emission."""
    t = 2.0
    assert list(oracle.renormalize(4, [1.0, t ** -60, 0.0, t ** -130, 0.0])) == \
        [1.0, t ** -60, t ** -130, 0.0]
    assert list(oracle.renormalize(4, [1.0, 0.0, 0.0, 0.0, 0.0])) == [1.0, 0.0, 0.0, 0.0]
    assert list(oracle.renormalize(4, [1.0, 1.0, 1.0, 1.0, 1.0])) == [5.0, 0.0, 0.0, 0.0]
    assert list(oracle.renormalize(3, [3.0, t ** -60, 0.0, 0.0])) == [3.0, t ** -60, 0.0]
    # every first-pass sum is a tie that rounds to even; the last term is
    # folded into the third component and rounds away
    assert list(oracle.renormalize(3, [1.0, t ** -53, t ** -106, t ** -159])) == \
        [1.0, t ** -53, t ** -106]


@pytest.mark.parametrize("K", [3, 4])
def test_renormalize_keeps_the_sum_and_is_idempotent(K):
    """On K+1 terms of decreasing magnitude with overlap, the output is
    non-overlapping, differs from the exact sum by at most one ulp of its last
    component, and renormalising a renormalised value changes nothing."""
    rng = np.random.default_rng(5 + K)
    for _ in range(500):
        x = np.empty(K + 1)
        x[0] = rng.uniform(-1, 1)
        for j in range(1, K + 1):
            x[j] = x[j - 1] * rng.uniform(-1, 1) * 2.0 ** -int(rng.integers(40, 56))
        c = oracle.renormalize(K, x)
        assert exact.nonoverlapping(c)
        err = abs(exact.value(c) - exact.value(x))
        assert err <= Fraction(exact.ulp(c[K - 1])), (x, c)
        c2 = oracle.renormalize(K, np.append(c, 0.0))
        assert np.array_equal(c, c2)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_conventional_dot_and_gemm_are_sequential_definitions(K):
    """Under the conventional arithmetic the vector and matrix routines are
    the same sequential loops over the conventional operations, and stay
    within the dot-product bound of the exact result."""
    bits = {2: 104, 3: 155, 4: 208}[K]
    A = synth.mp_array(K, (6, 17), 60 + K, "W")
    B = synth.mp_array(K, (17, 5), 70 + K, "W")
    with oracle.arith("nobf"):
        C = oracle.gemm(K, A, B)
        for i in range(6):
            for j in range(5):
                acc = np.zeros(K)
                for l in range(17):
                    acc = oracle.op1(K, "add", acc, oracle.op1(K, "mul", A[:, i, l], B[:, l, j]))
                assert np.array_equal(C[:, i, j], acc)
                assert np.array_equal(C[:, i, j], oracle.dot(K, A[:, i, :], B[:, :, j]))
                ex = exact.dot(A[:, i, :], B[:, :, j])
                sc = exact.abs_dot(A[:, i, :], B[:, :, j])
                assert abs(exact.value(C[:, i, j]) - ex) <= Fraction(17 * 2.0 ** -bits * sc)
