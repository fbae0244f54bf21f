"""Python binding of libmpx (argument marshalling only).

Multicomponent tensors are torch tensors on the GPU whose FIRST axis is the
component: (K, n) vectors, (K, rows, cols) row-major matrices; dtype float64
for DD / TD / QD (K = 2 / 3 / 4) and float32 for FF (K = 2).  Every function
here validates shapes, picks pointers and strides, and calls the C ABI
declared in include/mpx.h on torch's current stream; all arithmetic runs in
the HIP kernels of libmpx.so.  There is no fallback: if the library is
missing or a call fails, an exception is raised.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# MPX_LIBRARY names another build of the library (the CPU tests load an
# AddressSanitizer build of the host code this way).
LIB_PATH = os.environ.get("MPX_LIBRARY") or os.path.join(_HERE, "libmpx.so")

DD, TD, QD, FF = 2, 3, 4, 0x102
# Arithmetic flags OR-ed into DD / TD / QD: the conventional (non-branch-free)
# operations, with the sloppy or (DD only) the accurate double-word addition.
NOBF, NOBF_ACC = 0x1000, 0x2000
PRECS = {"dd": DD, "td": TD, "qd": QD, "ff": FF,
         "dd_nobf": DD | NOBF, "td_nobf": TD | NOBF, "qd_nobf": QD | NOBF,
         "dd_nobf_acc": DD | NOBF_ACC}
_K = {DD: 2, TD: 3, QD: 4, FF: 2, DD | NOBF: 2, TD | NOBF: 3, QD | NOBF: 4, DD | NOBF_ACC: 2}

OP_DOT, OP_GEMV, OP_GEMM, OP_OZAKI, OP_CGEMM, OP_STRASSEN = 1, 2, 3, 4, 5, 6

_lib = None


class MpxError(RuntimeError):
    pass


def lib():
    """The loaded libmpx.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MpxError(f"{LIB_PATH} not found: build it with `python -m paper_2603_14926_amd.build`")
        L = C.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


_i = C.c_int
_l = C.c_int64
_v = C.c_void_p
_z = C.c_size_t


def _declare(L):
    def sig(name, res, *args):
        f = getattr(L, name)
        f.restype = res
        f.argtypes = list(args)
    sig("mpx_version", _i)
    sig("mpx_status_string", C.c_char_p, _i)
    sig("mpx_add", _i, _i, _l, _v, _l, _v, _l, _v, _l, _v)
    sig("mpx_mul", _i, _i, _l, _v, _l, _v, _l, _v, _l, _v)
    sig("mpx_axpy", _i, _i, _l, _v, _v, _l, _v, _l, _v)
    sig("mpx_workspace_size", _z, _i, _i, _l, _l, _l, _l)
    sig("mpx_dot", _i, _i, _l, _v, _l, _v, _l, _v, _v, _z, _v)
    sig("mpx_gemv", _i, _i, _i, _l, _l, _v, _l, _l, _v, _l, _v, _l, _v, _z, _v)
    sig("mpx_gemm", _i, _i, _i, _i, _l, _l, _l, _v, _l, _l, _v, _l, _l, _v, _l, _l, _v)
    sig("mpx_gemm_variant", _i, _i, _i, _i, _i, _l, _l, _l, _v, _l, _l, _v, _l, _l, _v, _l, _l, _v)
    sig("mpx_gemm_variant_count", _i, _i)
    sig("mpx_gemm_variant_name", C.c_char_p, _i, _i)
    sig("mpx_gemm_autotune", _i, _i, _i, _i, _l, _l, _l, _v, _l, _l, _v, _l, _l, _v, _l, _l, _i,
        C.POINTER(C.c_float), _v)
    sig("mpx_gemm_autotune_reset", None)
    sig("mpx_gemm_ozaki_dd", _i, _l, _l, _l, _v, _l, _l, _v, _l, _l, _v, _l, _l, _i, _i, _l, _v, _z, _v)
    sig("mpx_gemm_ozaki_set_variant", _i, _i)
    sig("mpx_probe_threads", _l)
    sig("mpx_probe_valu", _i, _i, _l, _v, _l, _v)
    sig("mpx_probe_chains_threads", _l, _i)
    sig("mpx_probe_chains", _i, _i, _i, _l, _v, _l, _v)
    sig("mpx_gemm_batched_plan", _i, C.POINTER(_v), _i, _l, _v, _v, _v)
    sig("mpx_gemm_batched", _i, _v, _v, _l, _v, _l, _v, _l, _v)
    sig("mpx_gemm_batched_variant_count", _i, _v)
    sig("mpx_gemm_batched_set_variant", _i, _v, _i)
    sig("mpx_gemm_batched_autotune", _i, _v, _v, _l, _v, _l, _v, _l, _i, C.POINTER(C.c_float), _v)
    sig("mpx_gemm_plan_destroy", _i, _v)
    sig("mpx_gemm_strassen", _i, _i, _l, _l, _l, _v, _l, _l, _v, _l, _l, _v, _l, _l, _l, _v, _z, _v)
    sig("mpx_cgemm_3m", _i, _i, _l, _l, _l, _v, _v, _l, _l, _v, _v, _l, _l, _v, _v, _l, _l, _v, _z, _v)
    sig("mpx_polyval", _i, _i, _l, _l, _v, _l, _v, _l, _v, _l, _v)
    sig("mpx_polyval_estrin", _i, _i, _l, _l, _v, _l, _v, _l, _v, _l, _v)
    sig("mpx_polyval_cplx", _i, _i, _l, _l, _v, _l, _v, _v, _l, _v, _v, _l, _i, _v)
    sig("mpx_polyval_backward", _i, _i, _l, _l, _v, _l, _v, _l, _v, _l, _v, _l, _v, _l, _v)
    sig("mpx_polyroots_plan", _i, C.POINTER(_v), _i, _l, _v, _v, _v, _i, C.c_uint32)
    sig("mpx_dot_noalloc", _i, _i, _l, _v, _l, _v, _l, _v, _v)
    sig("mpx_gemm_selected_variant", _i, _i, _i, _i, _l, _l, _l)
    sig("mpx_tune_reload", _i)
    sig("mpx_polyroots", _i, _v, _v, _v, _l, _v, _v, _l, _v, _v)
    sig("mpx_plan_destroy", _i, _v)
    sig("mpx_polyroots_variant_count", _i)
    sig("mpx_polyroots_set_variant", _i, _v, _i)
    sig("mpx_polyroots_get_variant", _i, _v)
    sig("mpx_polyroots_autotune", _i, _v, _v, _v, _l, _v, _v, _l, _i, C.POINTER(C.c_float), _v)
    for name, res, args in _EXTRA_SIGS:
        if hasattr(L, name):
            sig(name, res, *args)


_EXTRA_SIGS = []


def _check(status: int, what: str):
    if status != 0:
        msg = lib().mpx_status_string(status)
        raise MpxError(f"{what} failed: {msg.decode() if msg else status}")


def prec_of(p) -> int:
    if isinstance(p, str):
        return PRECS[p.lower()]
    if p not in _K:
        raise ValueError(f"unknown precision {p!r}")
    return int(p)


def ncomp(p) -> int:
    return _K[prec_of(p)]


def dtype_of(p):
    return torch.float32 if prec_of(p) == FF else torch.float64


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr()) if t.numel() else None


def _planes(t: torch.Tensor, p, nd: int, name: str):
    """Check a (K, ...) component-plane tensor; return (plane stride, ld)."""
    K = ncomp(p)
    if t.dim() != nd + 1 or t.shape[0] != K:
        raise ValueError(f"{name}: expected shape (K={K}, ...) with {nd} trailing dims, got {tuple(t.shape)}")
    if t.dtype != dtype_of(p):
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype_of(p)}")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a GPU tensor")
    if t.numel() == 0:
        return max(t.stride(0), 0), (t.shape[2] if nd == 2 else 0)
    if nd == 1:
        if t.shape[1] > 1 and t.stride(1) != 1:
            raise ValueError(f"{name}: components must be contiguous")
        return t.stride(0), 0
    if t.shape[2] > 1 and t.stride(2) != 1:
        raise ValueError(f"{name}: rows must be contiguous")
    return t.stride(0), t.stride(1)


def _expect(t: torch.Tensor, shape, name: str):
    """An output (or an operand sized by the others) must have exactly the
    result's shape: the library writes the whole extent, so a smaller view
    would be written past its end."""
    if tuple(t.shape) != tuple(int(v) for v in shape):
        raise ValueError(f"{name}: expected shape {tuple(int(v) for v in shape)}, got {tuple(t.shape)}")


def _same_layout(t: torch.Tensor, ref: torch.Tensor, name: str, ref_name: str):
    """Real / imaginary parts share one plane stride and leading dimension."""
    if t.shape != ref.shape or t.stride() != ref.stride():
        raise ValueError(f"{name} must match {ref_name}'s shape and strides")


def workspace(op: int, p, m: int, n: int = 0, k: int = 0, extra: int = 0) -> torch.Tensor:
    nbytes = int(lib().mpx_workspace_size(op, prec_of(p), m, n, k, extra))
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device="cuda")


# ------------------------------------------------------------ elementwise ----

def _ew(fn, p, x, y, out):
    p = prec_of(p)
    psx, _ = _planes(x, p, 1, "x")
    psy, _ = _planes(y, p, 1, "y")
    n = x.shape[1]
    if y.shape[1] != n:
        raise ValueError("x and y lengths differ")
    if out is None:
        out = torch.empty_like(x)
    psz, _ = _planes(out, p, 1, "out")
    _expect(out, (ncomp(p), n), "out")
    _check(fn(p, n, _ptr(x), psx, _ptr(y), psy, _ptr(out), psz, _stream()), fn.__name__)
    return out


def add(p, x, y, out=None):
    """Elementwise BF addition of two (K, n) tensors."""
    return _ew(lib().mpx_add, p, x, y, out)


def mul(p, x, y, out=None):
    """Elementwise BF multiplication of two (K, n) tensors."""
    return _ew(lib().mpx_mul, p, x, y, out)


def axpy(p, alpha, x, y):
    """y := alpha * x + y in place; alpha is a sequence of K host floats."""
    p = prec_of(p)
    psx, _ = _planes(x, p, 1, "x")
    psy, _ = _planes(y, p, 1, "y")
    if x.shape[1] != y.shape[1]:
        raise ValueError("x and y lengths differ")
    K = ncomp(p)
    ctype = C.c_float if p == FF else C.c_double
    a = (ctype * K)(*[float(v) for v in alpha])
    _check(lib().mpx_axpy(p, x.shape[1], C.cast(a, C.c_void_p), _ptr(x), psx, _ptr(y), psy,
                          _stream()), "mpx_axpy")
    return y


def dot(p, x, y, out=None, ws=None):
    """K-component dot product of two (K, n) tensors -> (K,) tensor."""
    p = prec_of(p)
    psx, _ = _planes(x, p, 1, "x")
    psy, _ = _planes(y, p, 1, "y")
    n = x.shape[1]
    if y.shape[1] != n:
        raise ValueError("x and y lengths differ")
    if out is None:
        out = torch.empty(ncomp(p), dtype=dtype_of(p), device=x.device)
    _expect(out, (ncomp(p),), "out")
    if out.dtype != dtype_of(p) or not out.is_cuda or (out.numel() > 1 and out.stride(0) != 1):
        raise ValueError("out: expected K contiguous GPU values of the precision's dtype")
    if ws is None:
        ws = workspace(OP_DOT, p, n)
    _check(lib().mpx_dot(p, n, _ptr(x), psx, _ptr(y), psy, _ptr(out), _ptr(ws), ws.numel(),
                         _stream()), "mpx_dot")
    return out


def gemv(p, A, x, trans=False, out=None, ws=None):
    """op(A) x for a (K, m, n) matrix A."""
    p = prec_of(p)
    psA, lda = _planes(A, p, 2, "A")
    psx, _ = _planes(x, p, 1, "x")
    m, n = A.shape[1], A.shape[2]
    if x.shape[1] != (m if trans else n):
        raise ValueError("x length does not match op(A)")
    rows = n if trans else m
    if out is None:
        out = torch.empty((ncomp(p), rows), dtype=dtype_of(p), device=A.device)
    psy, _ = _planes(out, p, 1, "out")
    _expect(out, (ncomp(p), rows), "out")
    if ws is None:
        ws = workspace(OP_GEMV, p, m, n, int(trans))
    _check(lib().mpx_gemv(p, int(trans), m, n, _ptr(A), max(lda, n), psA, _ptr(x), psx,
                          _ptr(out), psy, _ptr(ws), ws.numel(), _stream()), "mpx_gemv")
    return out


def _gemm_shapes(A, B, tA, tB):
    m = A.shape[2] if tA else A.shape[1]
    k = A.shape[1] if tA else A.shape[2]
    n = B.shape[1] if tB else B.shape[2]
    kb = B.shape[2] if tB else B.shape[1]
    if k != kb:
        raise ValueError(f"inner dimensions differ: {k} vs {kb}")
    return m, n, k


def gemm(p, A, B, transA=False, transB=False, out=None, variant=None):
    """C = op(A) op(B) for (K, ., .) matrices; variant forces a kernel tiling."""
    p = prec_of(p)
    psA, lda = _planes(A, p, 2, "A")
    psB, ldb = _planes(B, p, 2, "B")
    m, n, k = _gemm_shapes(A, B, transA, transB)
    if out is None:
        out = torch.empty((ncomp(p), m, n), dtype=dtype_of(p), device=A.device)
    psC, ldc = _planes(out, p, 2, "out")
    _expect(out, (ncomp(p), m, n), "out")
    lda = max(lda, A.shape[2]); ldb = max(ldb, B.shape[2]); ldc = max(ldc, n)
    args = (int(transA), int(transB), m, n, k, _ptr(A), lda, psA, _ptr(B), ldb, psB,
            _ptr(out), ldc, psC, _stream())
    if variant is None:
        _check(lib().mpx_gemm(p, *args), "mpx_gemm")
    else:
        _check(lib().mpx_gemm_variant(p, int(variant), *args), "mpx_gemm_variant")
    return out


def gemm_ozaki_dd(A, B, slices, beta=20, kblk=256, out=None, ws=None):
    """DD product by the Ozaki-style split on FP64 MFMA; A (2, m, k), B (2, k, n)."""
    psA, lda = _planes(A, DD, 2, "A")
    psB, ldb = _planes(B, DD, 2, "B")
    m, n, k = _gemm_shapes(A, B, False, False)
    if out is None:
        out = torch.empty((2, m, n), dtype=torch.float64, device=A.device)
    psC, ldc = _planes(out, DD, 2, "out")
    _expect(out, (2, m, n), "out")
    if ws is None:
        ws = workspace(OP_OZAKI, DD, m, n, k, slices)
    _check(lib().mpx_gemm_ozaki_dd(m, n, k, _ptr(A), max(lda, k), psA, _ptr(B), max(ldb, n), psB,
                                   _ptr(out), max(ldc, n), psC, int(slices), int(beta), int(kblk),
                                   _ptr(ws), ws.numel(), _stream()), "mpx_gemm_ozaki_dd")
    return out


def cgemm_3m(p, Are, Aim, Bre, Bim, out=None, ws=None):
    """Complex product (Re, Im) = A B by the 3M method; parts are (K, ., .) tensors."""
    p = prec_of(p)
    psA, lda = _planes(Are, p, 2, "Are")
    psB, ldb = _planes(Bre, p, 2, "Bre")
    for t, ref, name in ((Aim, Are, "Aim"), (Bim, Bre, "Bim")):
        _planes(t, p, 2, name)
        _same_layout(t, ref, name, "the real part")
    m, n, k = _gemm_shapes(Are, Bre, False, False)
    if out is None:
        out = (torch.empty((ncomp(p), m, n), dtype=dtype_of(p), device=Are.device),
               torch.empty((ncomp(p), m, n), dtype=dtype_of(p), device=Are.device))
    Cre, Cim = out
    psC, ldc = _planes(Cre, p, 2, "Cre")
    _planes(Cim, p, 2, "Cim")
    _expect(Cre, (ncomp(p), m, n), "Cre")
    _same_layout(Cim, Cre, "Cim", "Cre")
    if ws is None:
        ws = workspace(OP_CGEMM, p, m, n, k)
    _check(lib().mpx_cgemm_3m(p, m, n, k, _ptr(Are), _ptr(Aim), max(lda, k), psA, _ptr(Bre),
                              _ptr(Bim), max(ldb, n), psB, _ptr(Cre), _ptr(Cim), max(ldc, n), psC,
                              _ptr(ws), ws.numel(), _stream()), "mpx_cgemm_3m")
    return Cre, Cim


def gemm_strassen(p, A, B, cutoff, out=None, ws=None):
    """C = A B by Strassen's recursion (split while min(m, k, n) >= cutoff)."""
    p = prec_of(p)
    psA, lda = _planes(A, p, 2, "A")
    psB, ldb = _planes(B, p, 2, "B")
    m, n, k = _gemm_shapes(A, B, False, False)
    if out is None:
        out = torch.empty((ncomp(p), m, n), dtype=dtype_of(p), device=A.device)
    psC, ldc = _planes(out, p, 2, "out")
    _expect(out, (ncomp(p), m, n), "out")
    if ws is None:
        ws = workspace(OP_STRASSEN, p, m, n, k, cutoff)
    _check(lib().mpx_gemm_strassen(p, m, n, k, _ptr(A), max(lda, k), psA, _ptr(B), max(ldb, n), psB,
                                   _ptr(out), max(ldc, n), psC, int(cutoff), _ptr(ws), ws.numel(),
                                   _stream()), "mpx_gemm_strassen")
    return out


PROBES = {"f64_add": 0, "f64_fma": 1, "f32_add": 2, "f32_fma": 3}


def probe_valu(kind: str, iters: int = 1 << 12, reps: int = 3, warmup: int = 1) -> float:
    """Measured VALU issue rate (lane-operations per second) of one
    instruction kind, from independent chains on 8 workgroups per CU: the
    median over `reps` launches after `warmup` untimed ones."""
    import statistics
    k = PROBES[kind]
    threads = int(lib().mpx_probe_threads())
    out = torch.empty(threads, dtype=torch.float64 if k < 2 else torch.float32, device="cuda")
    for _ in range(warmup):
        _check(lib().mpx_probe_valu(k, iters, _ptr(out), threads, _stream()), "mpx_probe_valu")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        _check(lib().mpx_probe_valu(k, iters, _ptr(out), threads, _stream()), "mpx_probe_valu")
        e1.record()
    torch.cuda.synchronize()
    ms = statistics.median(e0.elapsed_time(e1) for e0, e1 in ev)
    return threads * iters * 64.0 / (ms * 1e-3)


def probe_chains(chains: int, waves_per_simd: int, iters: int = 1 << 14, reps: int = 5,
                 warmup: int = 3) -> float:
    """FP64 addition rate (lane-operations per second) of `chains`
    independent dependency chains per lane at `waves_per_simd` waves per SIMD
    (one workgroup per CU): the median over `reps` launches after `warmup`
    untimed ones."""
    import statistics
    threads = int(lib().mpx_probe_chains_threads(waves_per_simd))
    if threads <= 0:
        raise ValueError("waves_per_simd must be 1..4")
    out = torch.empty(threads, dtype=torch.float64, device="cuda")
    run = lambda: _check(lib().mpx_probe_chains(chains, waves_per_simd, iters, _ptr(out), threads,
                                                _stream()), "mpx_probe_chains")
    for _ in range(warmup):
        run()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        run()
        e1.record()
    torch.cuda.synchronize()
    ms = statistics.median(e0.elapsed_time(e1) for e0, e1 in ev)
    return threads * iters * 8.0 * chains / (ms * 1e-3)


class GemmBatchPlan:
    """Plan for many independent products C_p = A_p B_p of ragged shapes in
    one persistent launch.  Operands are packed per component plane:
    A is (K, sum m_p k_p), A_p row-major at offsets()[0][p], likewise B and C."""

    def __init__(self, p, ms, ns, ks):
        import numpy as np
        self.p = prec_of(p)
        self.ms = np.ascontiguousarray(ms, dtype=np.int64)
        self.ns = np.ascontiguousarray(ns, dtype=np.int64)
        self.ks = np.ascontiguousarray(ks, dtype=np.int64)
        if not (self.ms.shape == self.ns.shape == self.ks.shape):
            raise ValueError("ms, ns, ks must have the same length")
        h = C.c_void_p()
        _check(lib().mpx_gemm_batched_plan(C.byref(h), self.p, self.ms.size,
                                           self.ms.ctypes.data_as(_v), self.ns.ctypes.data_as(_v),
                                           self.ks.ctypes.data_as(_v)), "mpx_gemm_batched_plan")
        self._h = h

    def offsets(self):
        """(a_off, b_off, c_off, totals) of the packed layout."""
        import numpy as np
        a = np.concatenate([[0], np.cumsum(self.ms * self.ks)])
        b = np.concatenate([[0], np.cumsum(self.ks * self.ns)])
        c = np.concatenate([[0], np.cumsum(self.ms * self.ns)])
        return a[:-1], b[:-1], c[:-1], (int(a[-1]), int(b[-1]), int(c[-1]))

    def _args(self, A, B, Cm):
        totals = self.offsets()[3]
        for t, name, tot in ((A, "A", totals[0]), (B, "B", totals[1]), (Cm, "C", totals[2])):
            if t.dim() != 2 or t.shape[0] != ncomp(self.p) or t.dtype != dtype_of(self.p) or not t.is_cuda:
                raise ValueError(f"{name}: expected a (K, total) GPU tensor of the plan's precision")
            if t.shape[1] > 1 and t.stride(1) != 1:
                raise ValueError(f"{name}: planes must be contiguous")
            _expect(t, (ncomp(self.p), tot), name)
        return (_ptr(A), A.stride(0), _ptr(B), B.stride(0), _ptr(Cm), Cm.stride(0))

    def run(self, A, B, Cm):
        a = self._args(A, B, Cm)
        _check(lib().mpx_gemm_batched(self._h, *a, _stream()), "mpx_gemm_batched")
        return Cm

    def variant_count(self):
        return int(lib().mpx_gemm_batched_variant_count(self._h))

    def set_variant(self, v):
        _check(lib().mpx_gemm_batched_set_variant(self._h, int(v)), "mpx_gemm_batched_set_variant")

    def autotune(self, A, B, Cm, reps=3):
        a = self._args(A, B, Cm)
        best = C.c_float()
        v = lib().mpx_gemm_batched_autotune(self._h, *a, int(reps), C.byref(best), _stream())
        if v < 0:
            _check(v, "mpx_gemm_batched_autotune")
        return v, best.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.mpx_gemm_plan_destroy(h)
            self._h = None


def gemm_ozaki_set_variant(v: int) -> None:
    _check(lib().mpx_gemm_ozaki_set_variant(int(v)), "mpx_gemm_ozaki_set_variant")


def gemm_variants(p):
    p = prec_of(p)
    return [lib().mpx_gemm_variant_name(p, i).decode() for i in range(lib().mpx_gemm_variant_count(p))]


def gemm_autotune(p, A, B, out, transA=False, transB=False, reps=3):
    """Time every GEMM tiling on these buffers, remember the fastest for this
    shape bucket; returns (variant index, ms)."""
    p = prec_of(p)
    psA, lda = _planes(A, p, 2, "A")
    psB, ldb = _planes(B, p, 2, "B")
    psC, ldc = _planes(out, p, 2, "out")
    m, n, k = _gemm_shapes(A, B, transA, transB)
    best = C.c_float()
    r = lib().mpx_gemm_autotune(p, int(transA), int(transB), m, n, k, _ptr(A), max(lda, A.shape[2]),
                                psA, _ptr(B), max(ldb, B.shape[2]), psB, _ptr(out), max(ldc, n),
                                psC, reps, C.byref(best), _stream())
    if r < 0:
        _check(r, "mpx_gemm_autotune")
    return r, best.value


# ------------------------------------------------------------ polynomials ----

def polyval(p, coef, x, out=None, method="horner"):
    """y_b = sum_i coef[:, b, i] x_b^i by Horner (or Estrin's method);
    coef (K, batch, deg+1), x (K, batch)."""
    p = prec_of(p)
    if p == FF:
        raise ValueError("polyval supports DD / TD / QD")
    K = ncomp(p)
    if coef.dim() != 3 or coef.shape[0] != K:
        raise ValueError("coef must be (K, batch, deg+1)")
    coef = coef.contiguous()
    psx, _ = _planes(x, p, 1, "x")
    batch, d1 = coef.shape[1], coef.shape[2]
    if x.shape[1] != batch:
        raise ValueError("x must have one point per polynomial")
    if out is None:
        out = torch.empty((K, batch), dtype=torch.float64, device=coef.device)
    psy, _ = _planes(out, p, 1, "out")
    _expect(out, (K, batch), "out")
    fn = {"horner": lib().mpx_polyval, "estrin": lib().mpx_polyval_estrin}[method]
    _check(fn(p, batch, d1 - 1, _ptr(coef), coef.stride(0), _ptr(x), psx, _ptr(out), psy,
              _stream()), f"polyval ({method})")
    return out


def polyval_cplx(p, coef, xre, xim, out=None, method="horner"):
    """Real-coefficient polynomials at complex points: coef (K, batch, deg+1),
    xre / xim (K, batch) -> (yre, yim) by Horner or Estrin's method."""
    p = prec_of(p)
    if p == FF:
        raise ValueError("polyval_cplx supports DD / TD / QD")
    K = ncomp(p)
    if coef.dim() != 3 or coef.shape[0] != K:
        raise ValueError("coef must be (K, batch, deg+1)")
    coef = coef.contiguous()
    psx, _ = _planes(xre, p, 1, "xre")
    _planes(xim, p, 1, "xim")
    _same_layout(xim, xre, "xim", "xre")
    batch, d1 = coef.shape[1], coef.shape[2]
    if xre.shape[1] != batch:
        raise ValueError("one point per polynomial")
    if out is None:
        out = (torch.empty((K, batch), dtype=torch.float64, device=coef.device),
               torch.empty((K, batch), dtype=torch.float64, device=coef.device))
    yre, yim = out
    psy, _ = _planes(yre, p, 1, "yre")
    _planes(yim, p, 1, "yim")
    _expect(yre, (K, batch), "yre")
    _same_layout(yim, yre, "yim", "yre")
    _check(lib().mpx_polyval_cplx(p, batch, d1 - 1, _ptr(coef), coef.stride(0), _ptr(xre), _ptr(xim),
                                  psx, _ptr(yre), _ptr(yim), psy, {"horner": 0, "estrin": 1}[method],
                                  _stream()), f"polyval_cplx ({method})")
    return yre, yim


def polyval_backward(p, coef, x, gy, want_coef=True, want_x=True):
    """(dL/dcoef, dL/dx) for L = sum_b gy_b p_b(x_b); entries None when not wanted."""
    p = prec_of(p)
    K = ncomp(p)
    if coef.dim() != 3 or coef.shape[0] != K:
        raise ValueError("coef must be (K, batch, deg+1)")
    coef = coef.contiguous()
    psx, _ = _planes(x, p, 1, "x")
    psg, _ = _planes(gy, p, 1, "gy")
    batch, d1 = coef.shape[1], coef.shape[2]
    _expect(x, (K, batch), "x")
    _expect(gy, (K, batch), "gy")
    gc = torch.empty_like(coef) if want_coef else None
    gx = torch.empty((K, batch), dtype=torch.float64, device=coef.device) if want_x else None
    _check(lib().mpx_polyval_backward(
        p, batch, d1 - 1, _ptr(coef), coef.stride(0), _ptr(x), psx, _ptr(gy), psg,
        _ptr(gc) if gc is not None else None, gc.stride(0) if gc is not None else 0,
        _ptr(gx) if gx is not None else None, gx.stride(0) if gx is not None else 0,
        _stream()), "mpx_polyval_backward")
    return gc, gx


DK_INIT, DK_GRAPH = 1, 2


class RootsPlan:
    """Plan for the batched Durand-Kerner solver (owns its device buffers).

    degrees: host sequence of polynomial degrees (>= 1).  By default the
    coefficient columns are packed: polynomial b occupies columns coef_off[b]
    .. coef_off[b] + deg[b] of (K, total_coef) planes, coef_off the prefix
    sums of deg + 1; roots likewise with (K, total_roots) and prefix sums of
    deg.  coef_off / root_off (host sequences of batch + 1 int64 offsets)
    place the polynomials elsewhere; the planes then need coef_off[-1] and
    root_off[-1] columns."""

    def __init__(self, p, degrees, iters=200, init=True, graph=True, coef_off=None, root_off=None):
        import numpy as np
        self.p = prec_of(p)
        if self.p == FF:
            raise ValueError("polyroots supports DD / TD / QD")
        self.K = ncomp(self.p)
        self.degrees = np.ascontiguousarray(degrees, dtype=np.int32)
        if (coef_off is None) != (root_off is None):
            raise ValueError("give both coef_off and root_off, or neither")
        offs = [None, None]
        if coef_off is not None:
            offs = [np.ascontiguousarray(o, dtype=np.int64) for o in (coef_off, root_off)]
            for o, name in zip(offs, ("coef_off", "root_off")):
                if o.shape != (self.degrees.size + 1,):
                    raise ValueError(f"{name}: expected {self.degrees.size + 1} offsets")
            self.total_coef, self.total_roots = int(offs[0][-1]), int(offs[1][-1])
        else:
            self.total_coef = int((self.degrees.astype(np.int64) + 1).sum())
            self.total_roots = int(self.degrees.astype(np.int64).sum())
        self.coef_off, self.root_off = offs
        flags = (DK_INIT if init else 0) | (DK_GRAPH if graph else 0)
        h = C.c_void_p()
        ptr = lambda o: None if o is None else o.ctypes.data_as(C.c_void_p)
        _check(lib().mpx_polyroots_plan(C.byref(h), self.p, self.degrees.size,
                                        self.degrees.ctypes.data_as(C.c_void_p), ptr(offs[0]), ptr(offs[1]),
                                        int(iters), flags),
               "mpx_polyroots_plan")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.mpx_plan_destroy(h)
            self._h = None

    def _args(self, cre, cim, zre, zim):
        for t, name, cols in ((cre, "coef_re", self.total_coef), (cim, "coef_im", self.total_coef),
                              (zre, "roots_re", self.total_roots), (zim, "roots_im", self.total_roots)):
            _planes(t, self.p, 1, name)
            if t.shape[1] != cols:
                raise ValueError(f"{name}: expected {cols} columns, got {t.shape[1]}")
        if cre.stride(0) != cim.stride(0) or zre.stride(0) != zim.stride(0):
            raise ValueError("real and imaginary planes must share a plane stride")

    def run(self, coef_re, coef_im, roots_re, roots_im, status=None):
        """Iterate in place on roots_re / roots_im; returns the status tensor."""
        self._args(coef_re, coef_im, roots_re, roots_im)
        if status is None:
            status = torch.zeros(self.degrees.size, dtype=torch.int32, device=coef_re.device)
        if status.dtype != torch.int32 or not status.is_cuda or status.dim() != 1 or \
                status.shape[0] != self.degrees.size or (status.numel() > 1 and status.stride(0) != 1):
            raise ValueError(f"status: expected a contiguous int32 GPU tensor of {self.degrees.size} values")
        _check(lib().mpx_polyroots(self._h, _ptr(coef_re), _ptr(coef_im), coef_re.stride(0),
                                   _ptr(roots_re), _ptr(roots_im), roots_re.stride(0),
                                   _ptr(status), _stream()), "mpx_polyroots")
        return status

    def set_variant(self, v):
        _check(lib().mpx_polyroots_set_variant(self._h, int(v)), "mpx_polyroots_set_variant")

    def variant(self):
        return int(lib().mpx_polyroots_get_variant(self._h))

    def autotune(self, coef_re, coef_im, roots_re, roots_im, iters_probe=2):
        self._args(coef_re, coef_im, roots_re, roots_im)
        best = C.c_float()
        r = lib().mpx_polyroots_autotune(self._h, _ptr(coef_re), _ptr(coef_im), coef_re.stride(0),
                                         _ptr(roots_re), _ptr(roots_im), roots_re.stride(0),
                                         int(iters_probe), C.byref(best), _stream())
        if r < 0:
            _check(r, "mpx_polyroots_autotune")
        return r, best.value


def polyroots_variant_count() -> int:
    return int(lib().mpx_polyroots_variant_count())
