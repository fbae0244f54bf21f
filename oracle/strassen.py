"""Strassen's matrix product over the oracle's multicomponent arithmetic
(TEST INFRASTRUCTURE ONLY, like the rest of this package).

Section 3.1 uses Strassen's algorithm for its matrix benchmarks and stops the
recursion once a block is smaller than 32 x 32; the paper does not print the
algorithm.  This is the classic form (Strassen, Numer. Math. 13, 1969):

    M1 = (A11 + A22)(B11 + B22)      M5 = (A11 + A12) B22
    M2 = (A21 + A22) B11             M6 = (A21 - A11)(B11 + B12)
    M3 = A11 (B12 - B22)             M7 = (A12 - A22)(B21 + B22)
    M4 = A22 (B21 - B11)
    C11 = ((M1 + M4) - M5) + M7      C12 = M3 + M5
    C21 = M2 + M4                    C22 = ((M1 - M2) + M3) + M6

with these readings of what the paper leaves open:
  * a product of shape (m, k) x (k, n) is split while min(m, k, n) >= cutoff
    (cutoff 32 in the paper; at least 2); otherwise it is the classical
    product, each entry the sequential sum of the naive triple loop;
  * each dimension d splits into a leading half ceil(d/2) and a trailing
    half floor(d/2); trailing blocks are padded with zeros to the leading
    block's shape (a padded sum adds the zeros with the multicomponent
    addition; a padded single block is a zero-extended copy);
  * subtraction is addition of the negation; the C blocks are formed in the
    left-to-right order written above and then cut to their true shape.

``gemm`` evaluates the recursion on whole matrices; ``entries`` follows the
same recursion for single entries (only the rows and columns each entry
depends on are formed), so full-size results can be checked at sampled
positions.  Both use only the oracle's add / dot / gemm.
"""
from __future__ import annotations

import numpy as np

from . import add as _add, dot as _dot, gemm as _gemm, op1 as _op1


def _halves(d):
    return (d + 1) // 2, d // 2


def split(m, k, n, cutoff):
    if cutoff < 2:
        raise ValueError("cutoff must be at least 2 (a dimension of 1 cannot split)")
    return min(m, k, n) >= cutoff


def _pad(X, r, c):
    """Zero-extend a (K, rows, cols) block to (K, r, c)."""
    K = X.shape[0]
    out = np.zeros((K, r, c))
    out[:, :X.shape[1], :X.shape[2]] = X
    return out


def _addm(K, X, Y, sign=1.0):
    sh = X.shape
    return _add(K, X.reshape(K, -1), (sign * Y).reshape(K, -1)).reshape(sh)


def gemm(K, A, B, cutoff):
    """C = A B by the recursion above; A (K, m, k), B (K, k, n)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    m, k = A.shape[1:]
    n = B.shape[2]
    if not split(m, k, n, cutoff):
        return _gemm(K, A, B)
    m1, m2 = _halves(m)
    k1, k2 = _halves(k)
    n1, n2 = _halves(n)
    A11, A12 = A[:, :m1, :k1], _pad(A[:, :m1, k1:], m1, k1)
    A21, A22 = _pad(A[:, m1:, :k1], m1, k1), _pad(A[:, m1:, k1:], m1, k1)
    B11, B12 = B[:, :k1, :n1], _pad(B[:, :k1, n1:], k1, n1)
    B21, B22 = _pad(B[:, k1:, :n1], k1, n1), _pad(B[:, k1:, n1:], k1, n1)
    M1 = gemm(K, _addm(K, A11, A22), _addm(K, B11, B22), cutoff)
    M2 = gemm(K, _addm(K, A21, A22), B11, cutoff)
    M3 = gemm(K, A11, _addm(K, B12, B22, -1.0), cutoff)
    M4 = gemm(K, A22, _addm(K, B21, B11, -1.0), cutoff)
    M5 = gemm(K, _addm(K, A11, A12), B22, cutoff)
    M6 = gemm(K, _addm(K, A21, A11, -1.0), _addm(K, B11, B12), cutoff)
    M7 = gemm(K, _addm(K, A12, A22, -1.0), _addm(K, B21, B22), cutoff)
    C11 = _addm(K, _addm(K, _addm(K, M1, M4), M5, -1.0), M7)
    C12 = _addm(K, M3, M5)
    C21 = _addm(K, M2, M4)
    C22 = _addm(K, _addm(K, _addm(K, M1, M2, -1.0), M3), M6)
    C = np.empty((K, m, n))
    C[:, :m1, :n1] = C11
    C[:, :m1, n1:] = C12[:, :, :n2]
    C[:, m1:, :n1] = C21[:, :m2, :]
    C[:, m1:, n1:] = C22[:, :m2, :n2]
    return C


# --------------------------------------------------------- single entries --

class _Rows:
    """Row provider of a virtual left operand: row(r) -> (K, cols)."""

    def __init__(self, K, cols, fn):
        self.K, self.cols, self.fn = K, cols, fn

    def __call__(self, r):
        return self.fn(r)


def _block_rows(P, rows_true, cols_true, r0, c0, r1, c1):
    """Row provider of the (r1 x c1) block at (r0, c0) of provider P (whose
    true shape is rows_true x cols_true), zero beyond the true shape."""
    K = P.K

    def fn(r):
        out = np.zeros((K, c1))
        rr = r0 + r
        if rr < rows_true:
            w = max(0, min(c1, cols_true - c0))
            if w:
                out[:, :w] = P(rr)[:, c0:c0 + w]
        return out
    return _Rows(K, c1, fn)


def _sum_rows(K, X, Y, sign):
    return _Rows(K, X.cols, lambda r: _add(K, X(r), sign * Y(r)))


def _entry(K, L, R, m, k, n, i, j, cutoff):
    """C[i, j] of L (m x k, row provider) times R (k x n, given as the row
    provider of R^T, i.e. a column provider)."""
    if not split(m, k, n, cutoff):
        return _dot(K, L(i), R(j))
    m1, _ = _halves(m)
    k1, _ = _halves(k)
    n1, _ = _halves(n)
    A = {(a, b): _block_rows(L, m, k, a * m1, b * k1, m1, k1) for a in (0, 1) for b in (0, 1)}
    # column providers of B's blocks: block (a, b) of B is block (b, a) of B^T
    Bt = {(a, b): _block_rows(R, n, k, b * n1, a * k1, n1, k1) for a in (0, 1) for b in (0, 1)}

    def one(X):
        return X

    prods = {
        1: (_sum_rows(K, A[0, 0], A[1, 1], 1.0), _sum_rows(K, Bt[0, 0], Bt[1, 1], 1.0)),
        2: (_sum_rows(K, A[1, 0], A[1, 1], 1.0), one(Bt[0, 0])),
        3: (one(A[0, 0]), _sum_rows(K, Bt[0, 1], Bt[1, 1], -1.0)),
        4: (one(A[1, 1]), _sum_rows(K, Bt[1, 0], Bt[0, 0], -1.0)),
        5: (_sum_rows(K, A[0, 0], A[0, 1], 1.0), one(Bt[1, 1])),
        6: (_sum_rows(K, A[1, 0], A[0, 0], -1.0), _sum_rows(K, Bt[0, 0], Bt[0, 1], 1.0)),
        7: (_sum_rows(K, A[0, 1], A[1, 1], -1.0), _sum_rows(K, Bt[1, 0], Bt[1, 1], 1.0)),
    }
    ii = i - m1 if i >= m1 else i
    jj = j - n1 if j >= n1 else j

    def M(t):
        return _entry(K, prods[t][0], prods[t][1], m1, k1, n1, ii, jj, cutoff)

    def ad(x, y, s=1.0):
        return _op1(K, "add", x, s * y)
    blk = (int(i >= m1), int(j >= n1))
    if blk == (0, 0):
        return ad(ad(ad(M(1), M(4)), M(5), -1.0), M(7))
    if blk == (0, 1):
        return ad(M(3), M(5))
    if blk == (1, 0):
        return ad(M(2), M(4))
    return ad(ad(ad(M(1), M(2), -1.0), M(3)), M(6))


def entries(K, A, B, rows, cols, cutoff):
    """C[rows[t], cols[t]] of the Strassen product, entry by entry."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    Bt = np.ascontiguousarray(np.asarray(B, dtype=np.float64).transpose(0, 2, 1))
    m, k = A.shape[1:]
    n = Bt.shape[1]
    L = _Rows(K, k, lambda r: A[:, r, :])
    R = _Rows(K, k, lambda c: Bt[:, c, :])
    out = np.empty((K, len(rows)))
    for t, (i, j) in enumerate(zip(rows, cols)):
        out[:, t] = _entry(K, L, R, m, k, n, int(i), int(j), cutoff)
    return out
