"""Seeded synthetic inputs for the multicomponent kernels.

This module holds none of the method's arithmetic: it never runs an error-free
transformation or a branch-free add/multiply.  It builds inputs directly in
the component-plane layout (numpy arrays of shape (K, ...), component first),
and is shared by the tests, the benchmark and the smoke check so that the HIP
path and the CPU oracle see the same bytes.

Generator (SplitMix64, Steele, Lea & Flood, OOPSLA 2014): one stream per array,
seeded with ``2603149260 + 1000*config + array_id``.  u01 = (x >> 11) * 2^-53.

Multicomponent values (component 0 drawn from the stated distribution, each
lower component the previous one times 2^-53 (binary32: 2^-24) times an
independent uniform in [-1, 1)).  "Renormalised to non-overlapping" is read as:
a lower component is halved (an exact power-of-two scaling) until adding it to
the component above no longer changes that component, i.e. until
fl(x_{c-1} + x_c) == x_{c-1}.  The result is a non-overlapping expansion whose
components follow the stated distribution up to a factor of two.

Exact-rational workloads of the paper (the real test matrices of Section 3.1,
the Chebyshev integration polynomial of Section 4.2, polynomials with known
roots) are built in exact rational arithmetic and rounded greedily to K
components: x_0 = RN(v), x_1 = RN(v - x_0), ...
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

BASE_SEED = 2603149260
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def seed_for(config: int, array_id: int) -> int:
    return BASE_SEED + 1000 * config + array_id


def splitmix64(seed: int, n: int) -> np.ndarray:
    """First n outputs of SplitMix64 started at state `seed`."""
    with np.errstate(over="ignore"):
        i = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed % (1 << 64)) + i * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def u01(seed: int, n: int) -> np.ndarray:
    """Uniform doubles in [0, 1), multiples of 2^-53."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def uniform_pm1(seed: int, n: int) -> np.ndarray:
    """Uniform doubles in [-1, 1) (exact transform of u01)."""
    return 2.0 * u01(seed, n) - 1.0


def normal(seed: int, n: int) -> np.ndarray:
    """Standard normals by Box-Muller from two halves of one stream."""
    u = u01(seed, 2 * n)
    u1 = 1.0 - u[:n]          # in (0, 1]
    u2 = u[n:]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def _lower_components(lead: np.ndarray, K: int, seed: int, dtype) -> np.ndarray:
    n = lead.size
    out = np.zeros((K,) + lead.shape, dtype=dtype)
    out[0] = lead
    shift = 2.0 ** -53 if dtype == np.float64 else 2.0 ** -24
    for c in range(1, K):
        u = uniform_pm1(seed + 7919 * c, n).reshape(lead.shape).astype(dtype)
        prev = out[c - 1]
        x = (prev * u) * dtype(shift)
        with np.errstate(over="ignore", invalid="ignore"):
            for _ in range(4):
                bad = (prev + x) != prev
                if not bad.any():
                    break
                x = np.where(bad, x * dtype(0.5), x)
        out[c] = x
    return out


def mp_array(K: int, shape, seed: int, dist: str = "U", phi: float = 4.0,
             dtype=np.float64) -> np.ndarray:
    """K-component array of the given shape.

    dist "U": component 0 uniform in [-1, 1).
    dist "W": component 0 = (u - 0.5) * exp(phi * z), u uniform [0,1), z ~ N(0,1)
              (wide exponent spread).
    dist "N": component 0 standard normal.
    """
    shape = (shape,) if isinstance(shape, int) else tuple(shape)
    n = int(np.prod(shape)) if shape else 1
    if dist == "U":
        lead = uniform_pm1(seed, n)
    elif dist == "W":
        lead = (u01(seed, n) - 0.5) * np.exp(phi * normal(seed + 104729, n))
    elif dist == "N":
        lead = normal(seed, n)
    else:
        raise ValueError(dist)
    lead = lead.astype(dtype).reshape(shape)
    return _lower_components(lead, K, seed, dtype)


# ------------------------------------------------------- exact workloads ----

def round_greedy(v: Fraction, K: int, dtype=np.float64) -> np.ndarray:
    """K non-overlapping components of the exact rational v: x_c = RN(v - sum)."""
    out = np.zeros(K, dtype=dtype)
    r = Fraction(v)
    for c in range(K):
        x = float(r) if dtype == np.float64 else _round_f32(r)
        out[c] = x
        r -= Fraction(x)
    return out


def _round_f32(r: Fraction) -> float:
    if r == 0:
        return 0.0
    f = float(np.float32(float(r)))
    # float(r) is RN to binary64; the double rounding to binary32 is fixed up
    # by comparing neighbours exactly.
    cands = [np.float32(f), np.nextafter(np.float32(f), np.float32(np.inf)),
             np.nextafter(np.float32(f), np.float32(-np.inf))]
    best = min(cands, key=lambda c: (abs(Fraction(float(c)) - r),
                                     int(np.float32(c).view(np.uint32)) & 1))
    return float(best)


def sqrt_fraction(m: int, bits: int = 320) -> Fraction:
    """sqrt(m) to within 2^-bits (floor), as an exact rational."""
    return Fraction(math.isqrt(m << (2 * bits)), 1 << bits)


def paper_real_gemm(K: int, n: int):
    """The real test matrices of Section 3.1:
    a_ij = sqrt(5)(i+j-1), b_ij = sqrt(3)(n-i+1), i, j = 1..n, as K-component
    planes (K, n, n).  sqrt is evaluated to 320 bits and rounded greedily."""
    s5, s3 = sqrt_fraction(5), sqrt_fraction(3)
    avals = np.stack([round_greedy(s5 * t, K) for t in range(1, 2 * n)], axis=1)
    bvals = np.stack([round_greedy(s3 * t, K) for t in range(1, n + 1)], axis=1)
    i = np.arange(n)[:, None]
    j = np.arange(n)[None, :]
    A = avals[:, (i + j)]                            # i+j-1 with 1-based i, j
    B = np.broadcast_to(bvals[:, (n - 1 - np.arange(n))][:, :, None], (K, n, n)).copy()
    return A, B


def paper_real_gemm_exact(n: int, i: int, j: int) -> Fraction:
    """Closed form of (AB)_ij for the Section 3.1 matrices, 0-based i, j:
    sqrt(15) * sum_{k=1..n} (i+k)(n-k+1), returned as sqrt(15) * S with S an
    integer: returns S."""
    i1 = i + 1
    return sum((i1 + k - 1) * (n - k + 1) for k in range(1, n + 1))


def chebyshev_coefficients(n: int):
    """Exact coefficients a_0..a_n of the Chebyshev integration polynomial of
    Section 4.2 (a_n = 1, odd-offset coefficients zero), from Newton's
    identities with power sums n/(2j+1) of the even powers:
    a_{n-2k} = -(n/(2k)) sum_{j=1..k} a_{n-2(k-j)} / (2j+1)."""
    a = [Fraction(0)] * (n + 1)
    a[n] = Fraction(1)
    for k in range(1, n // 2 + 1):
        s = sum(a[n - 2 * (k - j)] / (2 * j + 1) for j in range(1, k + 1))
        a[n - 2 * k] = -Fraction(n, 2 * k) * s
    return a


def poly_from_roots(roots):
    """Exact complex coefficients (list of (re, im) Fractions, ascending) of
    prod_j (z - r_j) for binary64 roots given as (re, im) float pairs."""
    coef = [(Fraction(1), Fraction(0))]
    for (rr, ri) in roots:
        rr, ri = Fraction(rr), Fraction(ri)
        new = [(Fraction(0), Fraction(0))] * (len(coef) + 1)
        for k, (cr, ci) in enumerate(coef):
            # multiply by z: shift up
            nr, ni = new[k + 1]
            new[k + 1] = (nr + cr, ni + ci)
            # multiply by -r
            nr, ni = new[k]
            new[k] = (nr - (cr * rr - ci * ri), ni - (cr * ri + ci * rr))
        coef = new
    return coef


def dk_batch(K: int, count: int, deg_lo: int, deg_hi: int, seed: int,
             n_known: int = 0, known_degree: int = 16):
    """Batch of complex polynomials for the root solver.

    Degrees uniform in [deg_lo, deg_hi]; coefficient real and imaginary
    leading parts standard normal with lower components as in mp_array.
    The first n_known polynomials instead have known_degree roots
    (cos t, sin t), t = 2 pi u, in binary64; their coefficients are expanded
    exactly and rounded greedily.

    Returns (degrees int32 (count,), coef_re (K, total), coef_im (K, total),
    known_roots list of arrays (n_known entries, complex128))."""
    span = deg_hi - deg_lo + 1
    deg = (deg_lo + np.floor(span * u01(seed, count))).astype(np.int32)
    deg[:n_known] = known_degree
    total = int((deg.astype(np.int64) + 1).sum())
    cre = mp_array(K, total, seed + 1, "N")
    cim = mp_array(K, total, seed + 2, "N")
    known = []
    off = 0
    for b in range(count):
        n = int(deg[b])
        if b < n_known:
            th = 2.0 * np.pi * u01(seed + 10 + b, n)
            roots = [(float(np.cos(t)), float(np.sin(t))) for t in th]
            coef = poly_from_roots(roots)
            for i, (vr, vi) in enumerate(coef):
                cre[:, off + i] = round_greedy(vr, K)
                cim[:, off + i] = round_greedy(vi, K)
            known.append(np.array([complex(r, i) for r, i in roots]))
        off += n + 1
    return deg, cre, cim, known


def offsets(degrees):
    """(coef_off, root_off) int64 arrays of length count+1."""
    d = np.asarray(degrees, np.int64)
    coef_off = np.concatenate([[0], np.cumsum(d + 1)])
    root_off = np.concatenate([[0], np.cumsum(d)])
    return coef_off, root_off
