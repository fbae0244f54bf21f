"""GPU parity at sizes whose element offsets pass 2^31 (DD, K = 2).

The kernels index with 64-bit integers; these cases put the checked elements
beyond the 32-bit range: vectors of 2^31 + 4099 elements (add, mul, AXPY, dot),
a GEMV whose matrix holds more than 2^31 entries, Horner / Estrin over a batch
whose coefficient array holds more than 2^31 values, and small GEMMs whose
leading dimensions put the last row past 2^31.  Inputs repeat a seeded block
with a prime period, so an offset taken modulo 2^32 (or truncated to 32 bits)
would read or write a different element than the one the oracle is given.
Every check is on sampled outputs computed one by one by the oracle; the large
operands need about 100 GiB of device memory at most."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle import exact
from paper_2603_14926_amd import mpx, synth
from tests.gpu_util import bits_equal, first_mismatch, to_gpu, to_np

pytestmark = pytest.mark.gpu

K = 2
P = 1_000_003                 # period of the repeated block (prime)
BITS = 104
TWO31 = 1 << 31


def _tiled(base: torch.Tensor, n: int) -> torch.Tensor:
    """(K, n) device tensor whose element i is base[:, i % P] (no temporaries)."""
    out = torch.empty((K, n), dtype=torch.float64, device="cuda")
    q, r = divmod(n, P)
    if q:
        out[:, :q * P].view(K, q, P).copy_(base[:, None, :].expand(K, q, P))
    if r:
        out[:, q * P:].copy_(base[:, :r])
    return out


@pytest.fixture(autouse=True)
def _release_memory():
    """Hand the large operands back to the device after each case."""
    yield
    import gc
    gc.collect()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _within(got, x, y):
    ex = exact.dot(x, y)
    err = abs(exact.value(got) - ex)
    bound = x.shape[1] * 2.0 ** -BITS * exact.abs_dot(x, y)
    return float(err) <= bound, float(err), bound


def test_vectors_beyond_2p31():
    n = TWO31 + 4099
    bx = synth.mp_array(K, P, 901, "U")
    by = synth.mp_array(K, P, 902, "U")
    x, y = _tiled(to_gpu(bx), n), _tiled(to_gpu(by), n)
    rng = np.random.default_rng(9)
    idx = np.unique(np.concatenate([
        [0, 1, P - 1, P, TWO31 - 1, TWO31, TWO31 + 1, n - 2, n - 1],
        TWO31 - 2048 + np.arange(64), rng.integers(TWO31, n, 200), rng.integers(0, n, 200)]))
    xs, ys = bx[:, idx % P], by[:, idx % P]
    gidx = torch.from_numpy(idx).cuda()

    z = mpx.add("dd", x, y)
    got = to_np(z[:, gidx])
    want = oracle.add(K, xs, ys)
    assert bits_equal(got, want), first_mismatch(got, want)
    mpx.mul("dd", x, y, out=z)
    got = to_np(z[:, gidx])
    want = oracle.mul(K, xs, ys)
    assert bits_equal(got, want), first_mismatch(got, want)
    del z

    alpha = synth.mp_array(K, 1, 903, "U")[:, 0]
    mpx.axpy("dd", alpha.tolist(), x, y)
    got = to_np(y[:, gidx])
    want = oracle.axpy(K, alpha, xs, ys)
    assert bits_equal(got, want), first_mismatch(got, want)

    # dot: y zero except at a few positions, most of them past 2^31, so the
    # exact value is a short sum the oracle can form
    sel = np.array([3, TWO31 - 1, TWO31, TWO31 + 77, n - 1000, n - 1])
    assert np.unique(sel).size == sel.size
    vals = synth.mp_array(K, sel.size, 904, "U")
    y.zero_()
    gv = to_gpu(vals)
    for j, i in enumerate(sel.tolist()):
        y[:, i:i + 1].copy_(gv[:, j:j + 1])
    # the input is what the oracle is given: nonzero exactly at `sel`
    assert int(torch.count_nonzero(y)) == int(np.count_nonzero(vals))
    assert bits_equal(np.stack([to_np(y[:, i]) for i in sel.tolist()], 1), vals)
    got = to_np(mpx.dot("dd", x, y))
    ok, err, bound = _within(got, bx[:, sel % P], vals)
    assert ok, (err, bound)
    want = oracle.dot(K, np.ascontiguousarray(bx[:, sel % P]), vals)
    assert _within(want, bx[:, sel % P], vals)[0]


def test_gemv_matrix_beyond_2p31_entries():
    m, n = 65539, 32771                  # m n = 2147811369 > 2^31
    assert m * n > TWO31
    ba = synth.mp_array(K, P, 911, "U")
    A = _tiled(to_gpu(ba), m * n).view(K, m, n)
    xn = synth.mp_array(K, n, 912, "U")
    xt = synth.mp_array(K, m, 913, "U")
    y = to_np(mpx.gemv("dd", A, to_gpu(xn)))
    for r in (0, 1, m // 2, m - 2, m - 1):
        row = ba[:, (r * n + np.arange(n)) % P]
        ok, err, bound = _within(y[:, r], row, xn)
        assert ok, ("n", r, err, bound)
    yt = to_np(mpx.gemv("dd", A, to_gpu(xt), trans=True))
    for c in (0, 1, n // 2, n - 1):
        col = ba[:, (np.arange(m) * n + c) % P]
        ok, err, bound = _within(yt[:, c], col, xt)
        assert ok, ("t", c, err, bound)


def test_polyval_coefficients_beyond_2p31():
    # degree 2047, the deepest list Estrin takes; batch (deg + 1) =
    # 2147493888 > 2^31
    batch, d1 = (1 << 20) + 5, 2048
    assert batch * d1 > TWO31
    bc = synth.mp_array(K, P, 921, "U")
    coef = _tiled(to_gpu(bc), batch * d1).view(K, batch, d1)
    # points in [-1, 1): the value stays below the sum of |coefficients|
    xs = synth.mp_array(K, batch, 922, "U")
    gx = to_gpu(xs)
    horner = to_np(mpx.polyval("dd", coef, gx))
    estrin = to_np(mpx.polyval("dd", coef, gx, method="estrin"))
    rng = np.random.default_rng(5)
    for b in [0, batch // 2, batch - 2, batch - 1, *rng.integers(batch // 2, batch, 8).tolist()]:
        cb = np.ascontiguousarray(bc[:, (b * d1 + np.arange(d1)) % P][:, None, :])
        xb = np.ascontiguousarray(xs[:, b:b + 1])
        want = oracle.polyval(K, cb, xb)[:, 0]
        assert bits_equal(horner[:, b], want), ("horner", b)
        want = oracle.polyval_estrin(K, cb, xb)[:, 0]
        assert bits_equal(estrin[:, b], want), ("estrin", b)


@pytest.mark.parametrize("which", ["A", "At", "B", "Bt", "C"])
def test_gemm_leading_dimension_beyond_2p31(which):
    """m = n = 40, k = 36; the operand named by `which` is stored with leading
    dimension 2^26 + 7, so its last row starts past element 2^31.  The
    default tiling and every row-wave tiling ("_rw": A through 64-bit scalar
    addresses, B through 32-bit byte offsets from each panel's first row, or
    the LDS tiling in their place where a transposed B's offsets would not
    fit) give the oracle's bits."""
    m, n, k = 40, 40, 36
    ld = (1 << 26) + 7
    A = synth.mp_array(K, (m, k), 931, "U")
    B = synth.mp_array(K, (k, n), 932, "U")
    want = oracle.gemm(K, A, B)

    def big(rows, cols):
        ps = (rows - 1) * ld + cols
        assert (rows - 1) * ld > TWO31
        return torch.empty(K * ps, dtype=torch.float64, device="cuda").as_strided(
            (K, rows, cols), (ps, ld, 1))

    tA, tB = which == "At", which == "Bt"
    if which in ("A", "At"):
        gA = big(k, m) if tA else big(m, k)
        gA.copy_(to_gpu(A.transpose(0, 2, 1) if tA else A))
    else:
        gA = to_gpu(A)
    if tB:
        gB = big(n, k)
        gB.copy_(to_gpu(B.transpose(0, 2, 1)))
    else:
        gB = to_gpu(B)
    if which == "B":
        gB = big(k, n)
        gB.copy_(to_gpu(B))
    out = big(m, n) if which == "C" else None
    C = mpx.gemm("dd", gA, gB, transA=tA, transB=tB, out=out)
    got = to_np(C)
    assert bits_equal(got, want), first_mismatch(got, want)
    for v, name in enumerate(mpx.gemm_variants("dd")):
        if "_rw" in name:
            if out is not None:
                out.fill_(float("nan"))
            got = to_np(mpx.gemm("dd", gA, gB, transA=tA, transB=tB, out=out, variant=v))
            assert bits_equal(got, want), (name, first_mismatch(got, want))
