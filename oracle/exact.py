"""Exact rational arithmetic used to pin the oracle (test infrastructure only).

Every binary64 (binary32) value is a dyadic rational N * 2^E, so sums and
products of them are computed exactly here with Python integers / Fractions.
Nothing in this module performs the branch-free algorithms; it evaluates the
plain mathematical definitions (a sum, a product, a dot product, a polynomial)
exactly, so it can judge the oracle independently.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np


def frac(x) -> Fraction:
    return Fraction(float(x))


def value(comps) -> Fraction:
    """Exact value of an unevaluated sum of floats."""
    return sum((Fraction(float(c)) for c in np.ravel(comps)), Fraction(0))


def ulp(x: float) -> float:
    return float(np.spacing(abs(np.float64(x))))


def nonoverlapping(comps) -> bool:
    """fl(x_c + x_{c+1}) == x_c for all adjacent components (the usual
    non-overlap test of a renormalised expansion)."""
    c = np.asarray(comps)
    return all(c[i] + c[i + 1] == c[i] for i in range(len(c) - 1))


def _dyadic_ints(planes: np.ndarray):
    """Exact integer values (Python ints, object array over the trailing axes)
    of sum_c planes[c] scaled by 2^-E0; returns (ints, E0)."""
    planes = np.asarray(planes, dtype=np.float64)
    mant, ex = np.frexp(planes)
    N = (mant * 2.0 ** 53).astype(np.int64)
    E = ex.astype(np.int64) - 53
    nz = N != 0
    E0 = int(E[nz].min()) if nz.any() else 0
    sh = np.where(nz, E - E0, 0)
    tot = None
    for c in range(planes.shape[0]):
        term = N[c].astype(object) * np.left_shift(np.ones_like(sh[c], dtype=object),
                                                   sh[c].astype(object))
        tot = term if tot is None else tot + term
    return tot, E0


def dot(x: np.ndarray, y: np.ndarray) -> Fraction:
    """Exact sum_i x_i y_i for K-component vectors x, y of shape (K, n)."""
    X, ex = _dyadic_ints(x)
    Y, ey = _dyadic_ints(y)
    s = int(np.sum(X * Y)) if X.size else 0
    e = ex + ey
    return Fraction(s) * Fraction(2) ** e


def abs_dot(x: np.ndarray, y: np.ndarray) -> float:
    """sum_i |x_i| |y_i| from the leading components (a bound scale only)."""
    return float(np.sum(np.abs(np.asarray(x[0], np.float64)) * np.abs(np.asarray(y[0], np.float64))))


def rel_err(approx_comps, exact: Fraction, scale: float) -> float:
    """|value(approx) - exact| / scale as a float (scale > 0)."""
    d = value(approx_comps) - exact
    return float(abs(d) / Fraction(scale)) if scale > 0 else float(abs(d))


def log2_rel(approx_comps, exact: Fraction) -> float:
    """log2 of the relative error (or -inf if exact)."""
    d = abs(value(approx_comps) - exact)
    if d == 0:
        return -math.inf
    return math.log2(d / abs(exact)) if exact != 0 else math.inf


def horner_real(coefs, x) -> Fraction:
    """Exact p(x) = sum a_i x^i, coefficients given as exact values, ascending."""
    h = Fraction(0)
    for a in reversed(list(coefs)):
        h = h * x + a
    return h


def cmul(a, b):
    return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])


def cpoly(coefs, z):
    """Exact complex polynomial value; coefs list of (re, im) ascending."""
    h = (Fraction(0), Fraction(0))
    for (cr, ci) in reversed(coefs):
        h = cmul(h, z)
        h = (h[0] + cr, h[1] + ci)
    return h
