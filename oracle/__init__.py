"""CPU oracle for branch-free DD / TD / QD / float-float arithmetic.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product path (the HIP library
and its Python binding) never does, and shares no code with it.

The arithmetic lives in ``mpx_oracle.c`` (plain sequential C, binary64 with
round-to-nearest-even, ``-ffp-contract=off``, explicit ``fma``); this module
only marshals numpy arrays.  Multicomponent arrays are numpy arrays whose
first axis is the component: shape ``(K, n)`` for vectors, ``(K, m, n)`` for
row-major matrices, float64 (float32 for float-float).

Parity notes (functions whose results no independent pin fixes are marked
"parity unpinned" in their docstrings): every function here is pinned by the
tests in ``tests/test_oracle_*.py``; see the docstrings for which pin.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None
_CLIB = None

_i64 = C.c_int64
_i32 = C.c_int
_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)
_vp = C.c_void_p


def _load(name):
    # MPX_ORACLE_LIBRARY names another build of liboracle.so (the CPU tests
    # run the oracle's pins against an AddressSanitizer build this way)
    alt = os.environ.get("MPX_ORACLE_LIBRARY")
    if alt and name == "liboracle.so":
        return C.CDLL(alt)
    path = os.path.join(_HERE, name)
    if not os.path.exists(path):
        from . import build as _b  # noqa: WPS433  (oracle's own build step)
        _b.build()
    return C.CDLL(path)


def lib():
    global _LIB
    if _LIB is None:
        _LIB = _load("liboracle.so")
    return _LIB


def count_lib():
    global _CLIB
    if _CLIB is None:
        _CLIB = _load("liboracle_count.so")
    return _CLIB


def _p(a):
    return a.ctypes.data_as(_vp)


def _chk(a, K=None, dtype=np.float64):
    a = np.ascontiguousarray(a, dtype=dtype)
    if K is not None and a.shape[0] != K:
        raise ValueError(f"expected {K} components, got shape {a.shape}")
    return a


def set_threads(t: int) -> None:
    lib().orc_set_threads(_i32(t))


def get_threads() -> int:
    return int(lib().orc_get_threads())


ARITH = {"bf": 0, "nobf": 1, "nobf_acc": 2}


class arith:
    """Context manager selecting the arithmetic of every K-generic oracle
    routine: "bf" (the paper's branch-free algorithms, the default), "nobf"
    (the conventional algorithms of Sections 2.1-2.3 with the sloppy DWAdd)
    or "nobf_acc" (conventional with DWAccurateAdd; TD and QD as "nobf").
    Float-float routines are unaffected.  Not thread-safe."""

    def __init__(self, mode: str):
        self.mode = ARITH[mode]

    def __enter__(self):
        self.prev = [int(L.orc_get_arith()) for L in (lib(), count_lib())]
        for L in (lib(), count_lib()):
            L.orc_set_arith(_i32(self.mode))
        return self

    def __exit__(self, *exc):
        for L, m in zip((lib(), count_lib()), self.prev):
            L.orc_set_arith(_i32(m))
        return False


def renormalize(K: int, x):
    """TWRenormalize (K = 3) / QWRenormalize (K = 4) of K+1 doubles: the
    two-pass QuickTwoSum renormalisation with data-dependent emission."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.shape != (K + 1,):
        raise ValueError("renormalize takes K+1 doubles")
    c = np.zeros(K)
    lib().orc_renormalize(_i32(K), _p(x), _p(c))
    return c


# ---------------------------------------------------------------- scalars ----

def eft(which: str, a: float, b: float):
    """QuickTwoSum / TwoSum / TwoProd (Section 2, the three EFT algorithms)."""
    w = {"quick_two_sum": 0, "two_sum": 1, "two_prod": 2}[which]
    s, e = C.c_double(), C.c_double()
    lib().orc_eft(_i32(w), C.c_double(a), C.c_double(b), C.byref(s), C.byref(e))
    return s.value, e.value


def op1(K: int, op: str, a, b, counting: bool = False):
    """One BF addition or multiplication of two K-component numbers
    (DWBFAdd/DWBFMul, TWBFAdd/TWBFMul, QWBFAdd/QDBFMul)."""
    a = _chk(a, K); b = _chk(b, K)
    c = np.zeros(K)
    L = count_lib() if counting else lib()
    L.orc_op1(_i32(K), _i32(0 if op == "add" else 1), _p(a), _p(b), _p(c))
    return c


def ff_op1(op: str, a, b):
    """DWBFAdd / DWBFMul on binary32 components (float-float)."""
    a = _chk(a, 2, np.float32); b = _chk(b, 2, np.float32)
    c = np.zeros(2, np.float32)
    lib().orc_ff_op1(_i32(0 if op == "add" else 1), _p(a), _p(b), _p(c))
    return c


def op_counts(K: int, op: str, a=None, b=None):
    """(add, sub, mul, fma) counts of one BF operation, from the counting build."""
    L = count_lib()
    a = np.ones(K) if a is None else a
    b = np.ones(K) if b is None else b
    L.orc_count_reset()
    op1(K, op, a, b, counting=True)
    out = (C.c_longlong * 4)()
    L.orc_count_get(out)
    return tuple(int(v) for v in out)


# ---------------------------------------------------------------- vectors ----

def _vec_args(x):
    return _p(x), _i64(x.shape[1] if x.ndim == 2 else 0)


def add(K, x, y):
    x = _chk(x, K); y = _chk(y, K)
    n = x.shape[1]
    z = np.zeros((K, n))
    lib().orc_add(_i32(K), _i64(n), _p(x), _i64(n), _p(y), _i64(n), _p(z), _i64(n))
    return z


def mul(K, x, y):
    x = _chk(x, K); y = _chk(y, K)
    n = x.shape[1]
    z = np.zeros((K, n))
    lib().orc_mul(_i32(K), _i64(n), _p(x), _i64(n), _p(y), _i64(n), _p(z), _i64(n))
    return z


def axpy(K, alpha, x, y):
    """Returns alpha*x + y (BF product, then BF sum), y untouched."""
    alpha = _chk(alpha, K); x = _chk(x, K); y = np.array(_chk(y, K))
    n = x.shape[1]
    lib().orc_axpy(_i32(K), _i64(n), _p(alpha), _p(x), _i64(n), _p(y), _i64(n))
    return y


def dot(K, x, y):
    x = _chk(x, K); y = _chk(y, K)
    n = x.shape[1]
    r = np.zeros(K)
    lib().orc_dot(_i32(K), _i64(n), _p(x), _i64(n), _p(y), _i64(n), _p(r))
    return r


def gemv(K, A, x, trans=False):
    A = _chk(A, K); x = _chk(x, K)
    m, n = A.shape[1], A.shape[2]
    rows = n if trans else m
    y = np.zeros((K, rows))
    lib().orc_gemv(_i32(K), _i32(int(trans)), _i64(m), _i64(n), _p(A), _i64(n), _i64(m * n),
                   _p(x), _i64(x.shape[1]), _p(y), _i64(rows))
    return y


def _gemm_dims(A, B, tA, tB):
    m = A.shape[2] if tA else A.shape[1]
    k = A.shape[1] if tA else A.shape[2]
    n = B.shape[1] if tB else B.shape[2]
    k2 = B.shape[2] if tB else B.shape[1]
    if k != k2:
        raise ValueError("inner dimensions differ")
    return m, n, k


def gemm(K, A, B, tA=False, tB=False):
    """C = op(A) op(B) by the naive triple loop, k ascending per entry."""
    A = _chk(A, K); B = _chk(B, K)
    m, n, k = _gemm_dims(A, B, tA, tB)
    Cm = np.zeros((K, m, n))
    lib().orc_gemm(_i32(K), _i32(int(tA)), _i32(int(tB)), _i64(m), _i64(n), _i64(k),
                   _p(A), _i64(A.shape[2]), _i64(A.shape[1] * A.shape[2]),
                   _p(B), _i64(B.shape[2]), _i64(B.shape[1] * B.shape[2]),
                   _p(Cm), _i64(n), _i64(m * n))
    return Cm


def gemm_entries(K, A, B, rows, cols, tA=False, tB=False):
    """Selected entries of op(A) op(B); returns (K, len(rows))."""
    A = _chk(A, K); B = _chk(B, K)
    m, n, k = _gemm_dims(A, B, tA, tB)
    rows = np.ascontiguousarray(rows, np.int64); cols = np.ascontiguousarray(cols, np.int64)
    out = np.zeros((K, rows.size))
    lib().orc_gemm_entries(_i32(K), _i32(int(tA)), _i32(int(tB)), _i64(k),
                           _p(A), _i64(A.shape[2]), _i64(A.shape[1] * A.shape[2]),
                           _p(B), _i64(B.shape[2]), _i64(B.shape[1] * B.shape[2]),
                           _i64(rows.size), _p(rows), _p(cols), _p(out))
    return out


def cgemm_3m(K, Are, Aim, Bre, Bim):
    """Complex product by the 3M method (Section 3.2); returns (Cre, Cim)."""
    Are, Aim, Bre, Bim = (_chk(v, K) for v in (Are, Aim, Bre, Bim))
    m, k = Are.shape[1], Are.shape[2]
    n = Bre.shape[2]
    Cre = np.zeros((K, m, n)); Cim = np.zeros((K, m, n))
    lib().orc_cgemm_3m(_i32(K), _i64(m), _i64(n), _i64(k), _p(Are), _p(Aim), _p(Bre), _p(Bim),
                       _p(Cre), _p(Cim))
    return Cre, Cim


def cgemm_3m_entries(K, Are, Aim, Bre, Bim, rows, cols):
    """Selected entries (rows[t], cols[t]) of the 3M complex product, by the
    steps of cgemm_3m restricted to those entries: the operand sums
    Are + Aim and Bre + Bim, the three real products C1 = Are Bre,
    C2 = Aim Bim, C3 = (Are + Aim)(Bre + Bim), then Re = C1 - C2 and
    Im = (C3 - C1) - C2.  Returns (re, im), each (K, len(rows))."""
    Are, Aim, Bre, Bim = (_chk(v, K) for v in (Are, Aim, Bre, Bim))
    SA = add(K, Are.reshape(K, -1), Aim.reshape(K, -1)).reshape(Are.shape)
    SB = add(K, Bre.reshape(K, -1), Bim.reshape(K, -1)).reshape(Bre.shape)
    c1 = gemm_entries(K, Are, Bre, rows, cols)
    c2 = gemm_entries(K, Aim, Bim, rows, cols)
    c3 = gemm_entries(K, SA, SB, rows, cols)
    re = np.zeros_like(c1); im = np.zeros_like(c1)
    for t in range(c1.shape[1]):
        re[:, t] = op1(K, "add", c1[:, t], -c2[:, t])
        im[:, t] = op1(K, "add", op1(K, "add", c3[:, t], -c1[:, t]), -c2[:, t])
    return re, im


# ------------------------------------------------------------ float-float ----

def ff_add(x, y):
    x = _chk(x, 2, np.float32); y = _chk(y, 2, np.float32)
    n = x.shape[1]
    z = np.zeros((2, n), np.float32)
    lib().orc_ff_add(_i64(n), _p(x), _i64(n), _p(y), _i64(n), _p(z), _i64(n))
    return z


def ff_mul(x, y):
    x = _chk(x, 2, np.float32); y = _chk(y, 2, np.float32)
    n = x.shape[1]
    z = np.zeros((2, n), np.float32)
    lib().orc_ff_mul(_i64(n), _p(x), _i64(n), _p(y), _i64(n), _p(z), _i64(n))
    return z


def ff_axpy(alpha, x, y):
    alpha = _chk(alpha, 2, np.float32); x = _chk(x, 2, np.float32)
    y = np.array(_chk(y, 2, np.float32))
    n = x.shape[1]
    lib().orc_ff_axpy(_i64(n), _p(alpha), _p(x), _i64(n), _p(y), _i64(n))
    return y


def ff_dot(x, y):
    x = _chk(x, 2, np.float32); y = _chk(y, 2, np.float32)
    n = x.shape[1]
    r = np.zeros(2, np.float32)
    lib().orc_ff_dot(_i64(n), _p(x), _i64(n), _p(y), _i64(n), _p(r))
    return r


def ff_gemv(A, x, trans=False):
    A = _chk(A, 2, np.float32); x = _chk(x, 2, np.float32)
    m, n = A.shape[1], A.shape[2]
    rows = n if trans else m
    y = np.zeros((2, rows), np.float32)
    lib().orc_ff_gemv(_i32(int(trans)), _i64(m), _i64(n), _p(A), _i64(n), _i64(m * n),
                      _p(x), _i64(x.shape[1]), _p(y), _i64(rows))
    return y


def ff_gemm(A, B, tA=False, tB=False):
    A = _chk(A, 2, np.float32); B = _chk(B, 2, np.float32)
    m, n, k = _gemm_dims(A, B, tA, tB)
    Cm = np.zeros((2, m, n), np.float32)
    lib().orc_ff_gemm(_i32(int(tA)), _i32(int(tB)), _i64(m), _i64(n), _i64(k),
                      _p(A), _i64(A.shape[2]), _i64(A.shape[1] * A.shape[2]),
                      _p(B), _i64(B.shape[2]), _i64(B.shape[1] * B.shape[2]),
                      _p(Cm), _i64(n), _i64(m * n))
    return Cm


def ff_gemm_entries(A, B, rows, cols, tA=False, tB=False):
    A = _chk(A, 2, np.float32); B = _chk(B, 2, np.float32)
    m, n, k = _gemm_dims(A, B, tA, tB)
    rows = np.ascontiguousarray(rows, np.int64); cols = np.ascontiguousarray(cols, np.int64)
    out = np.zeros((2, rows.size), np.float32)
    lib().orc_ff_gemm_entries(_i32(int(tA)), _i32(int(tB)), _i64(k),
                              _p(A), _i64(A.shape[2]), _i64(A.shape[1] * A.shape[2]),
                              _p(B), _i64(B.shape[2]), _i64(B.shape[1] * B.shape[2]),
                              _i64(rows.size), _p(rows), _p(cols), _p(out))
    return out


# ------------------------------------------------------------ polynomials ----

def polyval(K, coef, x):
    """Horner (Section 4.1). coef: (K, batch, deg+1) ascending powers; x: (K, batch)."""
    coef = _chk(coef, K); x = _chk(x, K)
    batch, d1 = coef.shape[1], coef.shape[2]
    y = np.zeros((K, batch))
    lib().orc_polyval(_i32(K), _i64(batch), _i64(d1 - 1), _p(coef), _i64(batch * d1),
                      _p(x), _i64(batch), _p(y), _i64(batch))
    return y


def polyval_estrin(K, coef, x):
    """Estrin's method on zero-padded power-of-two coefficient lists."""
    coef = _chk(coef, K); x = _chk(x, K)
    batch, d1 = coef.shape[1], coef.shape[2]
    y = np.zeros((K, batch))
    lib().orc_polyval_estrin(_i32(K), _i64(batch), _i64(d1 - 1), _p(coef), _i64(batch * d1),
                             _p(x), _i64(batch), _p(y), _i64(batch))
    return y


def polyval_cplx(K, coef, xre, xim, method="horner"):
    """Real-coefficient polynomials (coef (K, batch, deg+1)) at complex
    points (xre, xim each (K, batch)) by Horner or Estrin; returns (yre, yim)."""
    coef = _chk(coef, K); xre = _chk(xre, K); xim = _chk(xim, K)
    batch, d1 = coef.shape[1], coef.shape[2]
    yre = np.zeros((K, batch)); yim = np.zeros((K, batch))
    fn = lib().orc_polyval_cplx if method == "horner" else lib().orc_polyval_cplx_estrin
    fn(_i32(K), _i64(batch), _i64(d1 - 1), _p(coef), _i64(batch * d1), _p(xre), _p(xim),
       _i64(batch), _p(yre), _p(yim), _i64(batch))
    return yre, yim


def polyval_backward(K, coef, x, g, want_coef=True, want_x=True):
    """Gradients of sum_b g_b p_b(x_b): (dcoef (K,batch,deg+1), dx (K,batch))."""
    coef = _chk(coef, K); x = _chk(x, K); g = _chk(g, K)
    batch, d1 = coef.shape[1], coef.shape[2]
    gc = np.zeros((K, batch, d1)) if want_coef else None
    gx = np.zeros((K, batch)) if want_x else None
    lib().orc_polyval_backward(
        _i32(K), _i64(batch), _i64(d1 - 1), _p(coef), _i64(batch * d1), _p(x), _i64(batch),
        _p(g), _i64(batch), _p(gc) if gc is not None else None, _i64(batch * d1),
        _p(gx) if gx is not None else None, _i64(batch))
    return gc, gx


def recip(K, d):
    """1/d by Newton's method (Section 2: division through Newton iteration)."""
    d = _chk(d, K)
    y = np.zeros(K)
    lib().orc_recip(_i32(K), _p(d), _p(y))
    return y


def cdiv(K, xr, xi, yr, yi):
    xr, xi, yr, yi = (_chk(v, K) for v in (xr, xi, yr, yi))
    zr, zi = np.zeros(K), np.zeros(K)
    lib().orc_cdiv(_i32(K), _p(xr), _p(xi), _p(yr), _p(yi), _p(zr), _p(zi))
    return zr, zi


def dk_monic(K, are, aim):
    """c_i = a_i / a_n for one polynomial; are/aim: (K, n+1)."""
    are = _chk(are, K); aim = _chk(aim, K)
    n = are.shape[1] - 1
    cre, cim = np.zeros((K, n)), np.zeros((K, n))
    lib().orc_dk_monic(_i32(K), _i64(n), _p(are), _p(aim), _i64(n + 1), _p(cre), _p(cim), _i64(n))
    return cre, cim


def dk_horner(K, cre, cim, zr, zi):
    """q(z) = z^n + sum c_i z^i with power-of-two rescaling: returns
    (qr, qi, E) with q = (qr + i qi) * 2^E."""
    cre = _chk(cre, K); cim = _chk(cim, K); zr = _chk(zr, K); zi = _chk(zi, K)
    n = cre.shape[1]; npts = zr.shape[1]
    qr, qi = np.zeros((K, npts)), np.zeros((K, npts))
    E = np.zeros(npts, np.int64)
    lib().orc_dk_horner(_i32(K), _i64(n), _p(cre), _p(cim), _i64(n), _i64(npts),
                        _p(zr), _p(zi), _i64(npts), _p(qr), _p(qi), _i64(npts), _p(E))
    return qr, qi, E


def polyroots(K, degrees, coef_re, coef_im, roots_re=None, roots_im=None, iters=200,
              init=True):
    """Batched Durand-Kerner (Section 4.2). Coefficients of polynomial b are
    columns coef_off[b] .. coef_off[b]+deg[b] of coef_re/coef_im (K, total);
    roots are columns root_off[b] .. of (K, sum deg).  Returns
    (roots_re, roots_im, status)."""
    degrees = np.ascontiguousarray(degrees, np.int32)
    coef_off = np.concatenate([[0], np.cumsum(degrees.astype(np.int64) + 1)])
    root_off = np.concatenate([[0], np.cumsum(degrees.astype(np.int64))])
    coef_re = _chk(coef_re, K); coef_im = _chk(coef_im, K)
    nr = int(root_off[-1])
    zr = np.zeros((K, nr)) if roots_re is None else np.array(_chk(roots_re, K))
    zi = np.zeros((K, nr)) if roots_im is None else np.array(_chk(roots_im, K))
    status = np.zeros(degrees.size, np.int32)
    lib().orc_polyroots(_i32(K), _i64(degrees.size), _p(degrees), _p(coef_off), _p(root_off),
                        _p(coef_re), _p(coef_im), _i64(coef_re.shape[1]), _p(zr), _p(zi),
                        _i64(nr), _i32(iters), _i32(1 if init else 0), _p(status))
    return zr, zi, status


# ------------------------------------------------------------------ Ozaki ----

def ozaki_split_rows(A, s, beta, kblk):
    """Block exponents (m, nb) -- one per row and k-block of kblk columns --
    and integer slices (s, m, k) of a DD matrix (2, m, k)."""
    A = _chk(A, 2)
    m, k = A.shape[1], A.shape[2]
    nb = -(-k // kblk)
    e = np.zeros((m, nb), np.int32)
    sl = np.zeros((s, m, k))
    lib().orc_ozaki_split_rows(_i64(m), _i64(k), _p(A), _i64(k), _i64(m * k), _i32(s),
                               _i32(beta), _i64(kblk), _p(e), _p(sl))
    return e, sl


def ozaki_split_cols(B, s, beta, kblk):
    """Block exponents (n, nb) -- one per column and k-block of kblk rows --
    and integer slices (s, k, n) of a DD matrix (2, k, n)."""
    B = _chk(B, 2)
    k, n = B.shape[1], B.shape[2]
    nb = -(-k // kblk)
    f = np.zeros((n, nb), np.int32)
    sl = np.zeros((s, k, n))
    lib().orc_ozaki_split_cols(_i64(k), _i64(n), _p(B), _i64(n), _i64(k * n), _i32(s),
                               _i32(beta), _i64(kblk), _p(f), _p(sl))
    return f, sl


def ozaki_entries(A, B, rows, cols, s, beta, kblk):
    """Selected entries (2, cnt) of the Ozaki-split DD product.  A row's split
    depends only on that row (its own maximum), a column's only on that
    column, so only the rows / columns asked for are split."""
    A = _chk(A, 2); B = _chk(B, 2)
    rows = np.ascontiguousarray(rows, np.int64); cols = np.ascontiguousarray(cols, np.int64)
    ur, ri = np.unique(rows, return_inverse=True)
    uc, ci = np.unique(cols, return_inverse=True)
    As = np.ascontiguousarray(A[:, ur, :])
    Bs = np.ascontiguousarray(B[:, :, uc])
    m, k = As.shape[1], As.shape[2]
    n = Bs.shape[2]
    e, sa = ozaki_split_rows(As, s, beta, kblk)
    f, sb = ozaki_split_cols(Bs, s, beta, kblk)
    r2 = np.ascontiguousarray(ri.astype(np.int64)); c2 = np.ascontiguousarray(ci.astype(np.int64))
    out = np.zeros((2, rows.size))
    lib().orc_ozaki_entries(_i64(m), _i64(n), _i64(k), _i32(s), _i32(beta), _i64(kblk),
                            _p(e), _p(sa), _p(f), _p(sb), _i64(rows.size), _p(r2), _p(c2),
                            _p(out))
    return out
