"""Pins of the oracle's Ozaki-style split DD GEMM (the scheme is only named in
Section 3.1; the reading implemented is described in the oracle source):
error-free splitting, exact slice products, and the final error against
exact rational arithmetic."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact
from paper_2603_14926_amd import synth


@pytest.mark.parametrize("phi,beta", [(1.0, 20), (8.0, 20), (1.0, 22), (8.0, 22), (1.0, 23), (8.0, 23)])
def test_split_is_error_free_and_bounded(phi, beta):
    s = 9
    A = synth.mp_array(2, (6, 40), 1, "W", phi=phi)
    # adversarial: a row maximum just below a power of two, and values that
    # round up in every slice
    A[0, 0, :] = np.nextafter(2.0 ** 5, 0.0) * np.where(np.arange(40) % 2, 1.0, -1.0)
    A[1, 0, :] = 0.0
    A[0, 1, :] = 1.0 - 2.0 ** -53
    A[1, 1, :] = -2.0 ** -80
    e, sl = oracle.ozaki_split_rows(A, s, beta)
    for i in range(6):
        mx = np.max(np.abs(A[0, i]))
        assert mx < 2.0 ** e[i] and (mx >= 2.0 ** (e[i] - 1))
        for l in range(40):
            m = sl[:, i, l]
            assert np.all(m == np.rint(m))                 # integers
            # the magnitudes behind the exactness bound of the level sums
            assert abs(m[0]) <= 2 ** beta
            assert np.all(np.abs(m[1:]) <= 2 ** (beta - 1))
            rec = sum(Fraction(int(m[p])) * Fraction(2) ** (int(e[i]) - (p + 1) * beta) for p in range(s))
            resid = exact.value(A[:, i, l]) - rec
            # what is left after s slices is below half a unit of the last slice
            assert abs(resid) <= Fraction(2) ** (int(e[i]) - s * beta - 1) * Fraction(1 + 2.0 ** -50)
    # enough slices reproduce a DD value exactly (its span is at most ~2^107
    # below the row maximum for phi = 1 inputs of this size)
    if phi == 1.0:
        e, sl = oracle.ozaki_split_rows(A, 12, beta)
        for i in range(6):
            for l in range(40):
                rec = sum(Fraction(int(sl[p, i, l])) * Fraction(2) ** (int(e[i]) - (p + 1) * beta)
                          for p in range(12))
                if abs(A[0, i, l]) > 2.0 ** (int(e[i]) - 100):
                    assert rec == exact.value(A[:, i, l])


def test_split_cols_matches_rows_of_transpose():
    B = synth.mp_array(2, (30, 7), 2, "W", phi=4.0)
    f, sb = oracle.ozaki_split_cols(B, 6, 20)
    Bt = np.ascontiguousarray(B.transpose(0, 2, 1))
    e, sa = oracle.ozaki_split_rows(Bt, 6, 20)
    assert np.array_equal(f, e)
    assert np.array_equal(sb, sa.transpose(0, 2, 1))


@pytest.mark.parametrize("phi", [1.0, 4.0])
def test_ozaki_error_decreases_to_dd_level(phi):
    m = n = 5
    k = 300
    A = synth.mp_array(2, (m, k), 3, "W", phi=phi)
    B = synth.mp_array(2, (k, n), 4, "W", phi=phi)
    rows = np.repeat(np.arange(m), n); cols = np.tile(np.arange(n), m)
    errs = []
    for s in (3, 5, 7, 9, 11):
        out = oracle.ozaki_entries(A, B, rows, cols, s=s, beta=20, kblk=128)
        worst = 0.0
        for t in range(rows.size):
            ex = exact.dot(A[:, rows[t], :], B[:, :, cols[t]])
            sc = exact.abs_dot(A[:, rows[t], :], B[:, :, cols[t]])
            worst = max(worst, float(abs(exact.value(out[:, t]) - ex)) / sc)
        errs.append(worst)
    assert all(errs[i + 1] <= errs[i] * 1.01 + 1e-300 for i in range(len(errs) - 1)), errs
    # with enough slices the result is within the reduction bound k 2^-104
    assert errs[-1] <= k * 2.0 ** -104, errs
    assert errs[0] > errs[-1] * 2 ** 20


def test_ozaki_level_sums_are_exact_products():
    """With one slice per operand (s = 1) the product is a single exact level
    sum: compare with the exact integer dot product of the slices."""
    A = synth.mp_array(2, (3, 64), 5, "U")
    B = synth.mp_array(2, (64, 3), 6, "U")
    e, sa = oracle.ozaki_split_rows(A, 1, 20)
    f, sb = oracle.ozaki_split_cols(B, 1, 20)
    out = oracle.ozaki_entries(A, B, np.arange(3), np.arange(3), s=1, beta=20, kblk=64)
    for t in range(3):
        S = sum(int(sa[0, t, l]) * int(sb[0, l, t]) for l in range(64))
        ex = Fraction(S) * Fraction(2) ** (int(e[t]) + int(f[t]) - 40)
        assert exact.value(out[:, t]) == ex
