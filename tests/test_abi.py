"""CPU-side checks of the C ABI: the library loads, exports every function
declared in include/mpx.h, and rejects bad arguments before any launch (no
GPU needed: argument errors return before the first HIP call)."""
import ctypes as C
import os
import re

import numpy as np

import pytest

from paper_2603_14926_amd import mpx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


def _declared():
    names = set()
    for h in HEADERS:
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"\b(mpx_[a-z0-9_]+)\s*\(", txt):
            names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    L = mpx.lib()
    names = _declared()
    assert len(names) >= 10
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing


def test_version_and_status_strings():
    L = mpx.lib()
    assert L.mpx_version() >= 100
    for s in (0, -1, -2, -3, -4, -5):
        assert L.mpx_status_string(s)


FAKE = C.c_void_p(0x1000)  # never dereferenced: every call below fails validation


def test_bad_precision_rejected():
    L = mpx.lib()
    assert L.mpx_add(7, 10, FAKE, 10, FAKE, 10, FAKE, 10, None) == -2
    assert L.mpx_gemm(5, 0, 0, 4, 4, 4, FAKE, 4, 16, FAKE, 4, 16, FAKE, 4, 16, None) == -2


def test_bad_sizes_and_strides_rejected():
    L = mpx.lib()
    assert L.mpx_add(4, -1, FAKE, 10, FAKE, 10, FAKE, 10, None) == -1
    assert L.mpx_add(4, 10, FAKE, 9, FAKE, 10, FAKE, 10, None) == -1      # plane stride < n
    assert L.mpx_add(4, 10, None, 10, FAKE, 10, FAKE, 10, None) == -1     # null pointer
    assert L.mpx_gemm(4, 0, 0, 4, 4, 4, FAKE, 3, 16, FAKE, 4, 16, FAKE, 4, 16, None) == -1  # lda < k
    assert L.mpx_gemm(4, 2, 0, 4, 4, 4, FAKE, 4, 16, FAKE, 4, 16, FAKE, 4, 16, None) == -1  # bad flag
    assert L.mpx_gemm(4, 0, 0, 4, 4, 4, FAKE, 4, 15, FAKE, 4, 16, FAKE, 4, 16, None) == -1  # psA small
    assert L.mpx_gemv(4, 0, 4, 4, FAKE, 4, 16, FAKE, 4, FAKE, 3, None, 0, None) == -1       # psy < m
    assert L.mpx_axpy(2, 4, None, FAKE, 4, FAKE, 4, None) == -1


def test_workspace_checked():
    L = mpx.lib()
    n = 1 << 20
    need = L.mpx_workspace_size(mpx.OP_DOT, 4, n, 0, 0, 0)
    assert need > 0
    assert L.mpx_dot(4, n, FAKE, n, FAKE, n, FAKE, FAKE, need - 1, None) == -4
    assert L.mpx_dot(4, n, FAKE, n, FAKE, n, FAKE, None, 0, None) == -4
    assert L.mpx_workspace_size(mpx.OP_DOT, 4, 100, 0, 0, 0) == 0   # small dot: one block
    assert L.mpx_workspace_size(99, 4, 100, 0, 0, 0) == 0


def test_empty_problems_are_noops():
    L = mpx.lib()
    assert L.mpx_add(4, 0, None, 0, None, 0, None, 0, None) == 0
    assert L.mpx_gemm(4, 0, 0, 0, 5, 5, None, 5, 0, FAKE, 5, 25, None, 5, 0, None) == 0


def test_arithmetic_flags_accepted_only_where_declared():
    """The conventional-arithmetic flags: DD / TD / QD (accurate addition: DD
    only) on the elementwise, dot, GEMM and Horner entry points; never on FF
    or on the other entry points (checked before any launch)."""
    L = mpx.lib()
    NOBF, ACC = mpx.NOBF, mpx.NOBF_ACC
    for p in (2 | NOBF, 3 | NOBF, 4 | NOBF, 2 | ACC):
        # the conventional arithmetic has exactly the branch-free tilings
        base = p & 0xFF
        count = L.mpx_gemm_variant_count(base)
        assert count > 3 and L.mpx_gemm_variant_count(p) == count
        for v in range(count):
            mine = L.mpx_gemm_variant_name(p, v).decode()
            theirs = L.mpx_gemm_variant_name(base, v).decode()
            assert mine.startswith(theirs[:2] + "_nobf") and mine.endswith(theirs[2:])
        # accepted: the first failure is the size check
        assert L.mpx_add(p, -1, FAKE, 10, FAKE, 10, FAKE, 10, None) == -1
        assert L.mpx_gemm(p, 0, 0, 4, 4, 4, FAKE, 3, 16, FAKE, 4, 16, FAKE, 4, 16, None) == -1
        assert L.mpx_polyval(p, -1, 3, FAKE, 4, FAKE, 1, FAKE, 1, None) == -1
        # rejected by the entry points without a conventional path
        assert L.mpx_gemv(p, 0, 4, 4, FAKE, 4, 16, FAKE, 4, FAKE, 4, None, 0, None) == -2
        assert L.mpx_polyval_estrin(p, 1, 3, FAKE, 4, FAKE, 1, FAKE, 1, None) == -2
    for p in (0x102 | NOBF, 3 | ACC, 4 | ACC, 2 | NOBF | ACC):
        assert L.mpx_gemm_variant_count(p) == 0
        assert L.mpx_add(p, 1, FAKE, 10, FAKE, 10, FAKE, 10, None) == -2
        assert L.mpx_dot(p, 1, FAKE, 1, FAKE, 1, FAKE, None, 0, None) == -2
    assert L.mpx_workspace_size(1, 4 | NOBF, 1 << 20, 0, 0, 0) == \
        L.mpx_workspace_size(1, 4, 1 << 20, 0, 0, 0) > 0


def test_batched_gemm_plan_argument_errors():
    """Plan creation validates before touching the device."""
    L = mpx.lib()
    m = (C.c_int64 * 2)(4, 5)
    h = C.c_void_p()
    assert L.mpx_gemm_batched_plan(None, 4, 2, m, m, m) == -1
    assert L.mpx_gemm_batched_plan(C.byref(h), 7, 2, m, m, m) == -2            # unknown precision
    assert L.mpx_gemm_batched_plan(C.byref(h), 4 | mpx.NOBF, 2, m, m, m) == -2  # no flags here
    assert L.mpx_gemm_batched_plan(C.byref(h), 4, -1, m, m, m) == -1
    assert L.mpx_gemm_batched_plan(C.byref(h), 4, 2, None, m, m) == -1
    bad = (C.c_int64 * 2)(4, -5)
    assert L.mpx_gemm_batched_plan(C.byref(h), 4, 2, m, bad, m) == -1
    assert L.mpx_gemm_batched(None, FAKE, 1, FAKE, 1, FAKE, 1, None) == -1
    assert L.mpx_gemm_batched_variant_count(None) == 0
    assert L.mpx_gemm_plan_destroy(None) == -1


def test_probe_rejects_bad_arguments():
    L = mpx.lib()
    assert L.mpx_probe_valu(7, 1, FAKE, 256, None) == -1       # unknown kind
    assert L.mpx_probe_valu(0, 0, FAKE, 256, None) == -1       # iters < 1
    assert L.mpx_probe_valu(0, 1, FAKE, 300, None) == -1       # not a multiple of 256
    assert L.mpx_probe_valu(0, 1, None, 256, None) == -1       # null output
    assert L.mpx_probe_chains_threads(0) == 0 and L.mpx_probe_chains_threads(5) == 0
    big = 1 << 40
    assert L.mpx_probe_chains(3, 1, 1, FAKE, big, None) == -1     # chains not a power of two <= 16
    assert L.mpx_probe_chains(4, 0, 1, FAKE, big, None) == -1     # waves per SIMD outside 1..4
    assert L.mpx_probe_chains(4, 1, 0, FAKE, big, None) == -1     # iters < 1
    assert L.mpx_probe_chains(4, 1, 1, None, big, None) == -1     # null output
    assert L.mpx_probe_chains(4, 1, 1, FAKE, 1, None) == -1       # output too short


def test_strides_whose_span_overflows_int64_rejected():
    """A leading dimension or degree so large that the needed span does not
    fit in int64 is an argument error (the check must not wrap around)."""
    L = mpx.lib()
    big = 1 << 62
    # (m - 1) * lda + k would be 2 * 2^62 + 4: beyond int64
    assert L.mpx_gemm(4, 0, 0, 3, 4, 4, FAKE, big, 16, FAKE, 4, 16, FAKE, 4, 16, None) == -1
    assert L.mpx_gemm(4, 0, 0, 4, 4, 3, FAKE, 4, 16, FAKE, big, 16, FAKE, 4, 16, None) == -1
    assert L.mpx_gemm(4, 0, 0, 3, 4, 4, FAKE, 4, 16, FAKE, 4, 16, FAKE, big, 16, None) == -1
    assert L.mpx_gemv(4, 0, 3, 4, FAKE, big, 16, FAKE, 4, FAKE, 4, None, 0, None) == -1
    assert L.mpx_gemm_strassen(4, 3, 4, 4, FAKE, big, 16, FAKE, 4, 16, FAKE, 4, 16, 2, FAKE, 1 << 20,
                               None) == -1
    assert L.mpx_cgemm_3m(4, 3, 4, 4, FAKE, FAKE, big, 16, FAKE, FAKE, 4, 16, FAKE, FAKE, 4, 16, FAKE,
                          1 << 20, None) == -1
    assert L.mpx_gemm_ozaki_dd(3, 4, 4, FAKE, big, 16, FAKE, 4, 16, FAKE, 4, 16, 4, 20, 64, FAKE,
                               1 << 20, None) == -1
    # batch * (deg + 1) would be 4 * 2^62: beyond int64
    assert L.mpx_polyval(4, 4, big, FAKE, 10, FAKE, 4, FAKE, 4, None) == -1
    assert L.mpx_polyval_estrin(4, 4, big, FAKE, 10, FAKE, 4, FAKE, 4, None) == -1
    assert L.mpx_polyval(4, 4, (1 << 63) - 1, FAKE, 10, FAKE, 4, FAKE, 4, None) == -1


def test_overlapping_outputs_rejected():
    """Outputs that overlap an input, and workspaces that overlap an operand,
    are argument errors for the dot / GEMV / GEMM family (checked before any
    launch, on the pointer ranges of all K planes)."""
    L = mpx.lib()
    base = 1 << 40                        # fake device addresses, never dereferenced
    A, B, Cp = C.c_void_p(base), C.c_void_p(base + (1 << 20)), C.c_void_p(base + (2 << 20))
    inside_A = C.c_void_p(base + 3 * 16 * 8)   # within plane 3 of a QD 4 x 4 matrix at A
    assert L.mpx_gemm(4, 0, 0, 4, 4, 4, A, 4, 16, B, 4, 16, A, 4, 16, None) == -1         # C == A
    assert L.mpx_gemm(4, 0, 0, 4, 4, 4, A, 4, 16, B, 4, 16, inside_A, 4, 16, None) == -1  # C in A
    assert L.mpx_gemm(4, 0, 0, 4, 4, 4, A, 4, 16, B, 4, 16, B, 4, 16, None) == -1         # C == B
    assert L.mpx_gemm_strassen(4, 4, 4, 4, A, 4, 16, B, 4, 16, A, 4, 16, 2, Cp, 1 << 20, None) == -1
    assert L.mpx_gemm_ozaki_dd(4, 4, 4, A, 4, 16, B, 4, 16, B, 4, 16, 4, 20, 64, Cp, 1 << 20,
                               None) == -1
    assert L.mpx_gemm_ozaki_dd(4, 4, 4, A, 4, 16, B, 4, 16, Cp, 4, 16, 4, 20, 64, A, 1 << 20,
                               None) == -1                                                  # ws == A
    assert L.mpx_cgemm_3m(4, 4, 4, 4, A, B, 4, 16, Cp, C.c_void_p(base + (3 << 20)), 4, 16,
                          A, C.c_void_p(base + (5 << 20)), 4, 16, C.c_void_p(base + (6 << 20)),
                          1 << 20, None) == -1                                              # Cre == Are
    assert L.mpx_gemv(4, 0, 4, 4, A, 4, 16, B, 4, inside_A, 4, None, 0, None) == -1         # y in A
    assert L.mpx_dot(4, 8, A, 8, B, 8, C.c_void_p(base + 8 * 8), None, 0, None) == -1      # result in x


def test_polynomial_outputs_overlapping_inputs_rejected():
    """Horner / Estrin / complex-point evaluation and the backward pass reject
    outputs that overlap the coefficients, the points, the weights or each
    other (checked on the pointer ranges of all K planes, before any launch)."""
    L = mpx.lib()
    base = 1 << 40
    coef = C.c_void_p(base)                              # QD, 8 polynomials of degree 3: 32 per plane
    x = C.c_void_p(base + (1 << 20))
    y = C.c_void_p(base + (2 << 20))
    in_coef = C.c_void_p(base + 2 * 32 * 8)              # plane 2 of the coefficients
    in_x = C.c_void_p(base + (1 << 20) + 3 * 8 * 8)      # plane 3 of x
    for fn in (L.mpx_polyval, L.mpx_polyval_estrin):
        assert fn(4, 8, 3, coef, 32, x, 8, in_coef, 8, None) == -1
        assert fn(4, 8, 3, coef, 32, x, 8, in_x, 8, None) == -1
        assert fn(4, 8, 3, coef, 32, x, 8, x, 8, None) == -1
    xi, yi = C.c_void_p(base + (3 << 20)), C.c_void_p(base + (4 << 20))
    assert L.mpx_polyval_cplx(4, 8, 3, coef, 32, x, xi, 8, y, y, 8, 0, None) == -1      # yre == yim
    assert L.mpx_polyval_cplx(4, 8, 3, coef, 32, x, xi, 8, y, xi, 8, 0, None) == -1     # yim == xim
    assert L.mpx_polyval_cplx(4, 8, 3, coef, 32, x, xi, 8, in_coef, yi, 8, 1, None) == -1
    gy = C.c_void_p(base + (5 << 20))
    gc = C.c_void_p(base + (6 << 20))
    assert L.mpx_polyval_backward(4, 8, 3, coef, 32, x, 8, gy, 8, None, 0, gy, 8, None) == -1   # gx == gy
    assert L.mpx_polyval_backward(4, 8, 3, coef, 32, x, 8, gy, 8, in_coef, 32, None, 0, None) == -1
    assert L.mpx_polyval_backward(4, 8, 3, coef, 32, x, 8, gy, 8, gc, 32, in_x, 8, None) == -1
    assert L.mpx_polyval_backward(4, 8, 3, coef, 32, x, 8, gy, 8, gc, 32,
                                  C.c_void_p(base + (6 << 20) + 8), 8, None) == -1           # gx in gcoef


def _plan_ok_or_no_device(r):
    """A valid plan is built (0) when a GPU is present; without one the
    schedule is still built on the host and the first device allocation fails
    (MPX_EDEVICE)."""
    return r in (0, -5)


def test_roots_plan_host_schedules():
    """The plan constructor's host work (validation, LPT order, packed and
    lane-packed schedules) on ragged batches, with packed and caller offsets;
    run under AddressSanitizer by test_asan_host.py."""
    L = mpx.lib()
    rng = np.random.default_rng(3)
    for degs in ([1], [64, 1, 65, 128, 3], rng.integers(1, 600, 500).tolist(), [512] * 40 + [16] * 300):
        d = np.ascontiguousarray(degs, np.int32)
        for offs in (False, True):
            co = ro = None
            if offs:
                co = np.concatenate([[5], 5 + np.cumsum(d.astype(np.int64) + 3)]).astype(np.int64)
                ro = np.concatenate([[0], np.cumsum(d.astype(np.int64) + 1)]).astype(np.int64)
            h = C.c_void_p()
            r = L.mpx_polyroots_plan(C.byref(h), 4, d.size, d.ctypes.data_as(C.c_void_p),
                                     None if co is None else co.ctypes.data_as(C.c_void_p),
                                     None if ro is None else ro.ctypes.data_as(C.c_void_p), 3, 0)
            assert _plan_ok_or_no_device(r), r
            if r == 0:
                assert L.mpx_plan_destroy(h) == 0
    d = np.array([3, 0], np.int32)
    h = C.c_void_p()
    assert L.mpx_polyroots_plan(C.byref(h), 4, 2, d.ctypes.data_as(C.c_void_p), None, None, 1, 0) == -1
    d = np.array([3, 3], np.int32)
    co = np.array([0, 3, 8], np.int64)        # polynomial 0 needs 4 coefficient columns
    ro = np.array([0, 3, 6], np.int64)
    assert L.mpx_polyroots_plan(C.byref(h), 4, 2, d.ctypes.data_as(C.c_void_p),
                                co.ctypes.data_as(C.c_void_p), ro.ctypes.data_as(C.c_void_p), 1, 0) == -1
    assert L.mpx_polyroots_plan(C.byref(h), 4, 2, d.ctypes.data_as(C.c_void_p),
                                co.ctypes.data_as(C.c_void_p), None, 1, 0) == -1      # only one given
    assert L.mpx_polyroots_plan(C.byref(h), 4, 2, d.ctypes.data_as(C.c_void_p), None, None, 1, 4) == -1


def test_batched_gemm_plan_host_schedule():
    L = mpx.lib()
    rng = np.random.default_rng(4)
    for cnt in (1, 7, 300):
        ms = np.ascontiguousarray(rng.integers(0, 130, cnt), np.int64)
        ns = np.ascontiguousarray(rng.integers(1, 130, cnt), np.int64)
        ks = np.ascontiguousarray(rng.integers(0, 130, cnt), np.int64)
        h = C.c_void_p()
        r = L.mpx_gemm_batched_plan(C.byref(h), 4, cnt, ms.ctypes.data_as(C.c_void_p),
                                    ns.ctypes.data_as(C.c_void_p), ks.ctypes.data_as(C.c_void_p))
        assert _plan_ok_or_no_device(r), r
        if r == 0:
            assert L.mpx_gemm_plan_destroy(h) == 0
