"""GPU parity of the vector and matrix kernels against the CPU oracle.

Elementwise add / mul, AXPY and GEMM must match the oracle bit for bit (the
GEMM keeps the per-entry sequential k order of the naive triple loop).  Dot
and GEMV use a fixed reduction tree and must be within
n * 2^-b * sum |x_i y_i| of the exact result (b = 104 / 155 / 208, FF 46),
checked with exact rational arithmetic."""
from fractions import Fraction

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from tests import paper_values
from oracle import exact
from paper_2603_14926_amd import mpx, synth
from tests.gpu_util import PREC_K, bits_equal, first_mismatch, to_gpu, to_np

pytestmark = pytest.mark.gpu

BITS = {"dd": 104, "td": 155, "qd": 208, "ff": 46}


def _vec(K, n, seed, dtype, dist="U"):
    return synth.mp_array(K, n, seed, dist, dtype=dtype)


def _orc(name, p):
    ff = p == "ff"
    return getattr(oracle, ("ff_" if ff else "") + name)


@pytest.mark.parametrize("p,K,dt", PREC_K)
@pytest.mark.parametrize("n", [0, 1, 63, 65, 4096, 100003])
def test_elementwise_bit_exact(p, K, dt, n):
    x = _vec(K, n, 1000 + n, dt, "W" if n % 2 else "U")
    y = _vec(K, n, 2000 + n, dt, "W" if n % 2 else "U")
    gx, gy = to_gpu(x), to_gpu(y)
    if p == "ff":
        want_add, want_mul = oracle.ff_add(x, y), oracle.ff_mul(x, y)
    else:
        want_add, want_mul = oracle.add(K, x, y), oracle.mul(K, x, y)
    got_add = to_np(mpx.add(p, gx, gy))
    got_mul = to_np(mpx.mul(p, gx, gy))
    assert bits_equal(got_add, want_add), first_mismatch(got_add, want_add)
    assert bits_equal(got_mul, want_mul), first_mismatch(got_mul, want_mul)
    # in-place (output aliases an input)
    mpx.add(p, gx, gy, out=gx)
    assert bits_equal(to_np(gx), want_add)


@pytest.mark.parametrize("p,K,dt", PREC_K)
@pytest.mark.parametrize("n", [1, 4096, 65537])
def test_axpy_bit_exact(p, K, dt, n):
    alpha = _vec(K, 1, 3, dt)[:, 0]
    x = _vec(K, n, 4, dt)
    y = _vec(K, n, 5, dt)
    want = oracle.ff_axpy(alpha, x, y) if p == "ff" else oracle.axpy(K, alpha, x, y)
    gy = to_gpu(y)
    mpx.axpy(p, alpha.tolist(), to_gpu(x), gy)
    got = to_np(gy)
    assert bits_equal(got, want), first_mismatch(got, want)


def _within_bound(p, got, x, y):
    n = x.shape[1]
    ex = exact.dot(x.astype(np.float64), y.astype(np.float64))
    err = abs(exact.value(got.astype(np.float64)) - ex)
    bound = Fraction(n * 2.0 ** -BITS[p] * exact.abs_dot(x, y))
    return err <= bound, float(err), float(bound)


@pytest.mark.parametrize("p,K,dt", PREC_K)
@pytest.mark.parametrize("n", [0, 1, 2, 256, 257, 4096, 4097, 65536, 65537, 100003, 1 << 20])
def test_dot_within_bound(p, K, dt, n):
    x = _vec(K, n, 10 + n % 97, dt, "W")
    y = _vec(K, n, 20 + n % 89, dt, "W")
    got = to_np(mpx.dot(p, to_gpu(x), to_gpu(y)))
    if n == 0:
        assert np.all(got == 0)
        return
    ok, err, bound = _within_bound(p, got, x, y)
    assert ok, (err, bound)
    # The GPU's fixed two-stage tree is no less accurate than the sequential
    # oracle: its error is at most twice the oracle's, plus a slack of four
    # units of 2^-b sum|x y| for the sizes where both errors are near zero.
    want = oracle.ff_dot(x, y) if p == "ff" else oracle.dot(K, x, y)
    ok2, err_oracle, _ = _within_bound(p, want, x, y)
    assert ok2
    slack = 4.0 * bound / n
    assert err <= 2.0 * err_oracle + slack, (err, err_oracle, slack)


def test_dot_deterministic():
    K = 4
    x = to_gpu(_vec(K, 300001, 7, np.float64))
    y = to_gpu(_vec(K, 300001, 8, np.float64))
    a = to_np(mpx.dot("qd", x, y))
    b = to_np(mpx.dot("qd", x, y))
    assert bits_equal(a, b)


@pytest.mark.parametrize("p,K,dt", PREC_K)
@pytest.mark.parametrize("shape", [(1, 1), (37, 53), (300, 1000), (2000, 130)])
@pytest.mark.parametrize("trans", [False, True])
def test_gemv_within_bound(p, K, dt, shape, trans):
    m, n = shape
    A = synth.mp_array(K, (m, n), 30, "W", dtype=dt)
    x = _vec(K, m if trans else n, 31, dt)
    got = to_np(mpx.gemv(p, to_gpu(A), to_gpu(x), trans=trans))
    rows = n if trans else m
    At = A.transpose(0, 2, 1) if trans else A
    for r in sorted(set(np.linspace(0, rows - 1, 7).astype(int).tolist())):
        ok, err, bound = _within_bound(p, got[:, r], np.ascontiguousarray(At[:, r, :]), x)
        assert ok, (r, err, bound)


def test_gemv_full_size_sampled():
    """GEMV at n = 8192 (QD), sampled rows checked exactly."""
    K, n = 4, 8192
    A = synth.mp_array(K, (n, n), 40, "U")
    x = _vec(K, n, 41, np.float64)
    gA, gx = to_gpu(A), to_gpu(x)
    for trans in (False, True):
        got = to_np(mpx.gemv("qd", gA, gx, trans=trans))
        At = A.transpose(0, 2, 1) if trans else A
        for r in (0, 1, 4095, 8191):
            ok, err, bound = _within_bound("qd", got[:, r], np.ascontiguousarray(At[:, r, :]), x)
            assert ok, (trans, r, err, bound)


def _oracle_gemm(p, K, A, B, tA, tB):
    if p == "ff":
        return oracle.ff_gemm(A, B, tA, tB)
    return oracle.gemm(K, A, B, tA, tB)


@pytest.mark.parametrize("p,K,dt", PREC_K)
# (5, 130, 12) and (67, 3, 7): odd and single panel counts of the row-wave
# tilings' 2-, 4- and 8-deep panels, ragged rows within a wave and a ragged
# third column group; (9, 64, 8): k exactly one 8-deep panel, n one full group;
# (3, 70, 3001): a long k (hundreds of panels and an odd tail)
@pytest.mark.parametrize("mnk", [(1, 1, 1), (33, 17, 65), (100, 70, 129), (64, 64, 0),
                                 (5, 130, 12), (67, 3, 7), (9, 64, 8), (3, 70, 3001)])
def test_gemm_bit_exact_all_variants(p, K, dt, mnk):
    m, n, k = mnk
    A = synth.mp_array(K, (m, k), 50 + m, "W", dtype=dt)
    B = synth.mp_array(K, (k, n), 60 + n, "W", dtype=dt)
    want = _oracle_gemm(p, K, A, B, False, False)
    gA, gB = to_gpu(A), to_gpu(B)
    for v in range(len(mpx.gemm_variants(p))):
        got = to_np(mpx.gemm(p, gA, gB, variant=v))
        assert bits_equal(got, want), (v, first_mismatch(got, want))
    got = to_np(mpx.gemm(p, gA, gB))
    assert bits_equal(got, want)


@pytest.mark.parametrize("p,K,dt", PREC_K)
def test_gemm_transposes_bit_exact(p, K, dt):
    m, n, k = 45, 38, 71
    A = synth.mp_array(K, (m, k), 70, "U", dtype=dt)
    B = synth.mp_array(K, (k, n), 71, "U", dtype=dt)
    want = _oracle_gemm(p, K, A, B, False, False)
    At = np.ascontiguousarray(A.transpose(0, 2, 1))
    Bt = np.ascontiguousarray(B.transpose(0, 2, 1))
    for tA, tB in ((True, False), (False, True), (True, True)):
        a = At if tA else A
        b = Bt if tB else B
        for v in range(len(mpx.gemm_variants(p))):
            got = to_np(mpx.gemm(p, to_gpu(a), to_gpu(b), transA=tA, transB=tB, variant=v))
            assert bits_equal(got, want), (tA, tB, v, first_mismatch(got, want))


@pytest.mark.parametrize("p,K,dt", PREC_K)
def test_gemm_512_full_bit_exact(p, K, dt):
    """n = 512 on the default tiling and on every row-wave tiling (the
    autotuner's choices at this size): 74 sampled entries spread over all
    rows and column groups."""
    n = 512
    A = synth.mp_array(K, (n, n), 80, "U", dtype=dt)
    B = synth.mp_array(K, (n, n), 81, "U", dtype=dt)
    rows = np.arange(0, n, 7); cols = (rows * 13 + 5) % n
    if p == "ff":
        want = oracle.ff_gemm_entries(A, B, rows, cols)
    else:
        want = oracle.gemm_entries(K, A, B, rows, cols)
    gA, gB = to_gpu(A), to_gpu(B)
    got = to_np(mpx.gemm(p, gA, gB))
    assert bits_equal(np.ascontiguousarray(got[:, rows, cols]), want)
    for v, name in enumerate(mpx.gemm_variants(p)):
        if "_rw" in name:
            got = to_np(mpx.gemm(p, gA, gB, variant=v))
            assert bits_equal(np.ascontiguousarray(got[:, rows, cols]), want), name


@pytest.mark.parametrize("p,K,dt", PREC_K)
def test_gemm_1024_row_wave_sampled_bit_exact(p, K, dt):
    """n = 1024, wide-exponent inputs, every row-wave tiling: 40 sampled
    entries (corners, the edges of column groups, interior)."""
    n = 1024
    A = synth.mp_array(K, (n, n), 84, "W", dtype=dt)
    B = synth.mp_array(K, (n, n), 85, "W", dtype=dt)
    rng = np.random.default_rng(5)
    rows = np.concatenate([[0, 0, n - 1, n - 1, 511, 3], rng.integers(0, n, 34)])
    cols = np.concatenate([[0, n - 1, 0, n - 1, 63, 64], rng.integers(0, n, 34)])
    if p == "ff":
        want = oracle.ff_gemm_entries(A, B, rows, cols)
    else:
        want = oracle.gemm_entries(K, A, B, rows, cols)
    gA, gB = to_gpu(A), to_gpu(B)
    for v, name in enumerate(mpx.gemm_variants(p)):
        if "_rw" in name:
            got = to_np(mpx.gemm(p, gA, gB, variant=v))
            assert bits_equal(np.ascontiguousarray(got[:, rows, cols]), want), name


@pytest.mark.parametrize("p,K,dt,dist", [("qd", 4, np.float64, "U"), ("qd", 4, np.float64, "W"),
                                         ("td", 3, np.float64, "W"), ("dd", 2, np.float64, "U"),
                                         ("ff", 2, np.float32, "U")])
def test_gemm_2048_sampled_bit_exact(p, K, dt, dist):
    """Full benchmark size: 48 sampled entries (corners, edges, interior)
    computed one by one by the oracle must match bit for bit."""
    n = 2048
    A = synth.mp_array(K, (n, n), 90, dist, dtype=dt)
    B = synth.mp_array(K, (n, n), 91, dist, dtype=dt)
    got = to_np(mpx.gemm(p, to_gpu(A), to_gpu(B)))
    rng = np.random.default_rng(3)
    rows = np.concatenate([[0, 0, n - 1, n - 1, 1023], rng.integers(0, n, 43)])
    cols = np.concatenate([[0, n - 1, 0, n - 1, 1024], rng.integers(0, n, 43)])
    if p == "ff":
        want = oracle.ff_gemm_entries(A, B, rows, cols)
    else:
        want = oracle.gemm_entries(K, A, B, rows, cols)
    assert bits_equal(np.ascontiguousarray(got[:, rows, cols]), want)
    assert np.all(np.isfinite(got))


@pytest.mark.parametrize("n", [512, 1024, 2048, 2049])
def test_gemm_paper_matrices_digits(n):
    """The real test matrices of Section 3.1 at the paper's sizes reach its
    digit ranges (DD >= 29.0, TD >= 45.5, QD >= 61.7) against the closed
    form, on sampled entries (corners, interior, the last row and column)."""
    import math
    s15 = synth.sqrt_fraction(15, bits=400)
    need_by_k = paper_values.gemm_digits("real")     # tests/golden/gemm_digits.txt
    entries = ((0, 0), (100, 7), (n - 1, n - 1), (n // 2 - 1, 400), (0, n - 1), (n - 1, 0))
    for p, K in (("dd", 2), ("td", 3), ("qd", 4)):
        need = need_by_k[K]
        A, B = synth.paper_real_gemm(K, n)
        got = to_np(mpx.gemm(p, to_gpu(A), to_gpu(B)))
        for (i, j) in entries:
            ex = s15 * synth.paper_real_gemm_exact(n, i, j)
            rel = abs(exact.value(got[:, i, j]) - ex) / ex
            digits = -math.log10(float(rel)) if rel else 99.0
            assert digits >= need, (p, i, j, digits)


def test_gemm_autotune_keeps_bits():
    K = 4
    A = to_gpu(synth.mp_array(K, (256, 256), 95, "U"))
    B = to_gpu(synth.mp_array(K, (256, 256), 96, "U"))
    ref = to_np(mpx.gemm("qd", A, B, variant=0))
    out = torch.empty_like(A)
    v, ms = mpx.gemm_autotune("qd", A, B, out, reps=1)
    assert 0 <= v < len(mpx.gemm_variants("qd")) and ms > 0
    assert bits_equal(to_np(mpx.gemm("qd", A, B)), ref)


def test_graph_captured_axpy_and_dot_replay():
    """Launch-bound n = 4096 calls captured in one HIP graph: every replay
    (with eager work and synchronisation between replays) matches the oracle
    applied the same number of times."""
    K, n, per = 4, 4096, 3
    x = _vec(K, n, 501, np.float64)
    y0 = _vec(K, n, 502, np.float64)
    alpha = [0.75, 2.0 ** -60, 0.0, 0.0]
    gx, gy = to_gpu(x), to_gpu(y0)
    r = torch.empty(K, dtype=torch.float64, device="cuda")
    ws = mpx.workspace(mpx.OP_DOT, "qd", n)
    mpx.axpy("qd", alpha, gx, gy)      # warm-up outside the capture
    torch.cuda.synchronize()
    gy.copy_(to_gpu(y0))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(per):
            mpx.axpy("qd", alpha, gx, gy)
        mpx.dot("qd", gx, gy, out=r, ws=ws)
    torch.cuda.synchronize()
    gy.copy_(to_gpu(y0))
    want_y = y0.copy()
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        _ = (torch.ones(1000, device="cuda") * 3).sum().item()   # eager work between replays
        for _ in range(per):
            want_y = oracle.axpy(K, np.array(alpha), x, want_y)
        assert bits_equal(to_np(gy), want_y), rep
        ok, err, bound = _within_bound("qd", to_np(r), x, want_y)
        assert ok, (rep, err, bound)
