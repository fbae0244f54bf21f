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


@pytest.mark.parametrize("phi,beta,kblk", [(1.0, 20, 40), (8.0, 20, 16), (1.0, 22, 16), (8.0, 22, 40),
                                           (1.0, 23, 64), (8.0, 23, 16)])
def test_split_is_error_free_and_bounded(phi, beta, kblk):
    s = 9
    A = synth.mp_array(2, (6, 40), 1, "W", phi=phi)
    # adversarial: a row maximum just below a power of two, and values that
    # round up in every slice
    A[0, 0, :] = np.nextafter(2.0 ** 5, 0.0) * np.where(np.arange(40) % 2, 1.0, -1.0)
    A[1, 0, :] = 0.0
    A[0, 1, :] = 1.0 - 2.0 ** -53
    A[1, 1, :] = -2.0 ** -80
    e, sl = oracle.ozaki_split_rows(A, s, beta, kblk)
    nb = -(-40 // kblk)
    assert e.shape == (6, nb)
    for i in range(6):
        for b in range(nb):
            blk = slice(b * kblk, min(40, (b + 1) * kblk))
            mx = np.max(np.abs(A[0, i, blk]))
            # the block exponent: the block maximum lies in [2^(e-1), 2^e)
            assert mx < 2.0 ** e[i, b] and (mx >= 2.0 ** (e[i, b] - 1))
        for l in range(40):
            ei = int(e[i, l // kblk])
            m = sl[:, i, l]
            assert np.all(m == np.rint(m))                 # integers
            # the magnitudes behind the exactness bound of the level sums
            assert abs(m[0]) <= 2 ** beta
            assert np.all(np.abs(m[1:]) <= 2 ** (beta - 1))
            rec = sum(Fraction(int(m[p])) * Fraction(2) ** (ei - (p + 1) * beta) for p in range(s))
            resid = exact.value(A[:, i, l]) - rec
            # what is left after s slices is below half a unit of the last slice
            assert abs(resid) <= Fraction(2) ** (ei - s * beta - 1) * Fraction(1 + 2.0 ** -50)
    # enough slices reproduce a DD value exactly (its span is at most ~2^107
    # below the block maximum for phi = 1 inputs of this size)
    if phi == 1.0:
        e, sl = oracle.ozaki_split_rows(A, 12, beta, kblk)
        for i in range(6):
            for l in range(40):
                ei = int(e[i, l // kblk])
                rec = sum(Fraction(int(sl[p, i, l])) * Fraction(2) ** (ei - (p + 1) * beta)
                          for p in range(12))
                if abs(A[0, i, l]) > 2.0 ** (ei - 100):
                    assert rec == exact.value(A[:, i, l])


def test_block_exponents_follow_each_block():
    """Blocks of very different magnitude get their own exponents; with one
    block spanning k they reduce to the row maximum's exponent; an all-zero
    block gets 0 and all-zero slices."""
    A = synth.mp_array(2, (3, 48), 7, "U")
    A[:, 0, 16:32] *= 2.0 ** -40
    A[:, 1, 32:] = 0.0
    e, sl = oracle.ozaki_split_rows(A, 4, 20, 16)
    e1, _ = oracle.ozaki_split_rows(A, 4, 20, 48)
    for i in range(3):
        for b in range(3):
            mx = np.max(np.abs(A[0, i, 16 * b:16 * b + 16]))
            want = 0 if mx == 0 else math.frexp(mx)[1]
            assert e[i, b] == want
        assert e1[i, 0] == math.frexp(np.max(np.abs(A[0, i])))[1]
    assert e[0, 1] <= e[0, 0] - 35
    assert np.all(sl[:, 1, 32:] == 0.0)


def test_split_cols_matches_rows_of_transpose():
    B = synth.mp_array(2, (30, 7), 2, "W", phi=4.0)
    f, sb = oracle.ozaki_split_cols(B, 6, 20, 8)
    Bt = np.ascontiguousarray(B.transpose(0, 2, 1))
    e, sa = oracle.ozaki_split_rows(Bt, 6, 20, 8)
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


def test_block_scaling_needs_fewer_slices_for_wide_ranges():
    """With k-blocks of very different magnitude, per-block exponents make
    the error of s slices relative to each block, so one block of tiny
    entries loses nothing: the product with the small block alone is as
    accurate as with the large ones."""
    m = n = 3
    k = 64
    A = synth.mp_array(2, (m, k), 8, "U")
    B = synth.mp_array(2, (k, n), 9, "U")
    A[:, :, 32:] *= 2.0 ** -60          # the second k-block is 2^60 smaller
    rows = np.repeat(np.arange(m), n); cols = np.tile(np.arange(n), m)
    out = oracle.ozaki_entries(A, B, rows, cols, s=5, beta=20, kblk=32)
    A2 = A.copy(); A2[:, :, :32] = 0.0  # the small block's own contribution
    out2 = oracle.ozaki_entries(A2, B, rows, cols, s=5, beta=20, kblk=32)
    for t in range(rows.size):
        ex2 = exact.dot(A2[:, rows[t], :], B[:, :, cols[t]])
        sc2 = exact.abs_dot(A2[:, rows[t], :], B[:, :, cols[t]])
        # the small block alone is resolved to the level of s = 5 slices
        assert float(abs(exact.value(out2[:, t]) - ex2)) <= sc2 * 2.0 ** -75
        ex = exact.dot(A[:, rows[t], :], B[:, :, cols[t]])
        sc = exact.abs_dot(A[:, rows[t], :], B[:, :, cols[t]])
        assert float(abs(exact.value(out[:, t]) - ex)) <= sc * 2.0 ** -75


def test_ozaki_level_sums_are_exact_products():
    """With one slice per operand (s = 1) the product is a single exact level
    sum: compare with the exact integer dot product of the slices."""
    A = synth.mp_array(2, (3, 64), 5, "U")
    B = synth.mp_array(2, (64, 3), 6, "U")
    e, sa = oracle.ozaki_split_rows(A, 1, 20, 64)
    f, sb = oracle.ozaki_split_cols(B, 1, 20, 64)
    out = oracle.ozaki_entries(A, B, np.arange(3), np.arange(3), s=1, beta=20, kblk=64)
    for t in range(3):
        S = sum(int(sa[0, t, l]) * int(sb[0, l, t]) for l in range(64))
        ex = Fraction(S) * Fraction(2) ** (int(e[t, 0]) + int(f[t, 0]) - 40)
        assert exact.value(out[:, t]) == ex


def test_two_blocks_scale_their_level_sums_separately():
    """s = 1, two k-blocks of different magnitude: the result is the exact
    sum of the two blocks' integer dot products, each scaled by its own
    block exponents (the fold adds exact DD terms of bounded span)."""
    A = synth.mp_array(2, (2, 32), 10, "U")
    B = synth.mp_array(2, (32, 2), 11, "U")
    A[:, :, 16:] *= 2.0 ** -9
    B[:, 16:, :] *= 2.0 ** 5
    e, sa = oracle.ozaki_split_rows(A, 1, 20, 16)
    f, sb = oracle.ozaki_split_cols(B, 1, 20, 16)
    assert e[0, 1] != e[0, 0] and f[0, 1] != f[0, 0]
    out = oracle.ozaki_entries(A, B, np.arange(2), np.arange(2), s=1, beta=20, kblk=16)
    for t in range(2):
        ex = Fraction(0)
        for b in range(2):
            S = sum(int(sa[0, t, l]) * int(sb[0, l, t]) for l in range(16 * b, 16 * b + 16))
            ex += Fraction(S) * Fraction(2) ** (int(e[t, b]) + int(f[t, b]) - 40)
        assert abs(exact.value(out[:, t]) - ex) <= abs(ex) * Fraction(2) ** -104
