"""GPU parity of the polynomial kernels against the CPU oracle: real Horner
and its backward (bit-exact), and the batched Durand-Kerner solver
(bit-exact per iteration from identical start values; Aberth start values
within binary64 rounding, since they use device libm)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2603_14926_amd import mpx, synth
from tests.gpu_util import bits_equal, first_mismatch, to_gpu, to_np

pytestmark = pytest.mark.gpu

PRECS = [("dd", 2), ("td", 3), ("qd", 4)]


@pytest.mark.parametrize("p,K", PRECS)
@pytest.mark.parametrize("batch,deg", [(1, 0), (5, 1), (70, 33), (130, 257), (1024, 1024)])
def test_polyval_and_backward_bit_exact(p, K, batch, deg):
    coef = synth.mp_array(K, (batch, deg + 1), 1 + deg, "U")
    x = synth.mp_array(K, batch, 2 + deg, "U")
    g = synth.mp_array(K, batch, 3 + deg, "U")
    gcoef, gx, gg = to_gpu(coef), to_gpu(x), to_gpu(g)
    y = to_np(mpx.polyval(p, gcoef, gx))
    want = oracle.polyval(K, coef, x)
    assert bits_equal(y, want), first_mismatch(y, want)
    dc, dx = mpx.polyval_backward(p, gcoef, gx, gg)
    wc, wx = oracle.polyval_backward(K, coef, x, g)
    assert bits_equal(to_np(dc), wc), first_mismatch(to_np(dc), wc)
    assert bits_equal(to_np(dx), wx)


def _dk_inputs(K, degrees, seed):
    degrees = np.asarray(degrees, np.int32)
    total = int((degrees + 1).sum())
    cre = synth.mp_array(K, total, seed, "N")
    cim = synth.mp_array(K, total, seed + 1, "N")
    return degrees, cre, cim


RAGGED = [1, 2, 3, 17, 64, 65, 130, 5, 40]


@pytest.mark.parametrize("p,K", PRECS)
def test_dk_iterations_bit_exact_from_same_start(p, K):
    deg, cre, cim = _dk_inputs(K, RAGGED, 10 + K)
    z0r, z0i, _ = oracle.polyroots(K, deg, cre, cim, iters=0, init=True)
    wr, wi, wst = oracle.polyroots(K, deg, cre, cim, z0r, z0i, iters=6, init=False)
    for v in range(mpx.polyroots_variant_count()):
        plan = mpx.RootsPlan(p, deg, iters=6, init=False, graph=False)
        plan.set_variant(v)
        zr, zi = to_gpu(z0r), to_gpu(z0i)
        st = plan.run(to_gpu(cre), to_gpu(cim), zr, zi)
        assert bits_equal(to_np(zr), wr), (v, first_mismatch(to_np(zr), wr))
        assert bits_equal(to_np(zi), wi), v
        assert np.array_equal(to_np(st), wst)


# High degrees of the benchmark mix (16..512) beside small ones.  The packed
# schedule caps a job at the largest polynomial spread over four waves, so the
# degree-512 and degree-384 polynomials each put two 64-root chunks on one
# wave, and the small ones are packed around them.
HIGH = [512, 16, 384, 20, 257, 33, 511, 64, 300, 65, 17, 129, 448, 5]


def _max_horner_exponent(deg, z0r, z0i):
    """Largest n log2|z| over the start values: the exponent E that Horner's
    power-of-two rescaling reaches on the first sweep."""
    _, roff = synth.offsets(deg)
    e = 0.0
    for b, n in enumerate(deg):
        z = np.abs(z0r[0, roff[b]:roff[b + 1]] + 1j * z0i[0, roff[b]:roff[b + 1]])
        e = max(e, float(n) * float(np.log2(z.max())))
    return e


@pytest.mark.parametrize("p,K", PRECS)
def test_dk_high_degree_bit_exact_every_variant(p, K):
    """Degrees up to 512 from the oracle's Aberth start values, 3 sweeps, on
    every launch variant.  The start radius is ~n |c_{n-1}|, so E reaches
    thousands of bits on the first sweep and the scaled coefficients
    c_k 2^-E pass through the subnormal range to zero: those ldexp results
    must round as the oracle's do."""
    deg, cre, cim = _dk_inputs(K, HIGH, 70 + K)
    z0r, z0i, _ = oracle.polyroots(K, deg, cre, cim, iters=0, init=True)
    assert _max_horner_exponent(deg, z0r, z0i) > 1100   # c_k 2^-E underflows on the way
    wr, wi, wst = oracle.polyroots(K, deg, cre, cim, z0r, z0i, iters=3, init=False)
    gc_r, gc_i = to_gpu(cre), to_gpu(cim)
    for v in range(mpx.polyroots_variant_count()):
        plan = mpx.RootsPlan(p, deg, iters=3, init=False, graph=False)
        plan.set_variant(v)
        zr, zi = to_gpu(z0r), to_gpu(z0i)
        st = plan.run(gc_r, gc_i, zr, zi)
        assert bits_equal(to_np(zr), wr), (v, first_mismatch(to_np(zr), wr))
        assert bits_equal(to_np(zi), wi), v
        assert np.array_equal(to_np(st), wst), v


def test_dk_degree_512_200_sweeps_bit_exact():
    """One degree-512 QD polynomial (with two small ones) over the benchmark's
    200 sweeps in a graph-replayed packed launch, bit for bit."""
    K = 4
    deg, cre, cim = _dk_inputs(K, [512, 24, 61], 90)
    z0r, z0i, _ = oracle.polyroots(K, deg, cre, cim, iters=0, init=True)
    wr, wi, wst = oracle.polyroots(K, deg, cre, cim, z0r, z0i, iters=200, init=False)
    plan = mpx.RootsPlan("qd", deg, iters=200, init=False, graph=True)
    zr, zi = to_gpu(z0r), to_gpu(z0i)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        st = plan.run(to_gpu(cre), to_gpu(cim), zr, zi)
    stream.synchronize()
    assert bits_equal(to_np(zr), wr), first_mismatch(to_np(zr), wr)
    assert bits_equal(to_np(zi), wi)
    assert np.array_equal(to_np(st), wst)


def _spread(planes, off_packed, off_new, deg, extra):
    """Copy packed columns of each polynomial to new offsets; gaps hold NaN."""
    K = planes.shape[0]
    out = np.full((K, int(off_new[-1])), np.nan)
    for b, n in enumerate(deg):
        w = int(n) + extra
        out[:, off_new[b]:off_new[b] + w] = planes[:, off_packed[b]:off_packed[b] + w]
    return out


def test_dk_caller_offsets_with_gaps_every_variant():
    """Polynomials placed at caller-given offsets with NaN-filled gaps between
    them: every variant reproduces the oracle's sweeps on the packed layout,
    never reads a gap (a NaN would spread) and never writes one; with the
    Aberth start the result equals the packed-layout plan's bit for bit."""
    K = 4
    deg, cre, cim = _dk_inputs(K, [17, 64, 5, 130, 40, 65, 1], 95)
    z0r, z0i, _ = oracle.polyroots(K, deg, cre, cim, iters=0, init=True)
    wr, wi, wst = oracle.polyroots(K, deg, cre, cim, z0r, z0i, iters=4, init=False)
    cp, rp = synth.offsets(deg)
    idx = np.arange(deg.size + 1)
    co, ro = cp + 7 * idx + 2, rp + 3 * idx + 1
    Cr, Ci = _spread(cre, cp, co, deg, 1), _spread(cim, cp, co, deg, 1)
    Zr, Zi = _spread(z0r, rp, ro, deg, 0), _spread(z0i, rp, ro, deg, 0)
    gC_r, gC_i = to_gpu(Cr), to_gpu(Ci)
    for v in range(mpx.polyroots_variant_count()):
        plan = mpx.RootsPlan("qd", deg, iters=4, init=False, graph=False, coef_off=co, root_off=ro)
        plan.set_variant(v)
        zr, zi = to_gpu(Zr), to_gpu(Zi)
        st = plan.run(gC_r, gC_i, zr, zi)
        gr, gi = to_np(zr), to_np(zi)
        assert bits_equal(gr, _spread(wr, rp, ro, deg, 0)), v   # gaps still NaN
        assert bits_equal(gi, _spread(wi, rp, ro, deg, 0)), v
        assert np.array_equal(to_np(st), wst), v
    # Aberth start values computed on the GPU: same bits in either layout
    packed = mpx.RootsPlan("qd", deg, iters=3, init=True, graph=False)
    zr, zi = torch.zeros((K, int(rp[-1])), dtype=torch.float64, device="cuda"), None
    zi = torch.zeros_like(zr)
    packed.run(to_gpu(cre), to_gpu(cim), zr, zi)
    spread = mpx.RootsPlan("qd", deg, iters=3, init=True, graph=False, coef_off=co, root_off=ro)
    zr2, zi2 = to_gpu(np.full((K, int(ro[-1])), np.nan)), to_gpu(np.full((K, int(ro[-1])), np.nan))
    spread.run(gC_r, gC_i, zr2, zi2)
    assert bits_equal(to_np(zr2), _spread(to_np(zr), rp, ro, deg, 0))
    assert bits_equal(to_np(zi2), _spread(to_np(zi), rp, ro, deg, 0))


def test_dk_offsets_rejected():
    bad = [([0, 3, 6], [0, 3, 6]),      # polynomial 0 of degree 3 needs 4 coefficient columns
           ([0, 4, 8], [0, 2, 5]),      # and 3 root columns
           ([-1, 4, 8], [0, 3, 6])]     # negative first offset
    for co, ro in bad:
        with pytest.raises(mpx.MpxError):
            mpx.RootsPlan("qd", [3, 3], iters=1, init=False, graph=False, coef_off=co, root_off=ro)
    with pytest.raises(ValueError):
        mpx.RootsPlan("qd", [3, 3], iters=1, coef_off=[0, 4, 8])


def test_dk_odd_and_even_iteration_counts_and_resume():
    K = 4
    deg, cre, cim = _dk_inputs(K, [7, 33, 2, 64], 20)
    z0r, z0i, _ = oracle.polyroots(K, deg, cre, cim, iters=0, init=True)
    gc_r, gc_i = to_gpu(cre), to_gpu(cim)
    for iters in (0, 1, 2, 5):
        wr, wi, _ = oracle.polyroots(K, deg, cre, cim, z0r, z0i, iters=iters, init=False)
        zr, zi = to_gpu(z0r), to_gpu(z0i)
        mpx.RootsPlan("qd", deg, iters=iters, init=False, graph=False).run(gc_r, gc_i, zr, zi)
        assert bits_equal(to_np(zr), wr) and bits_equal(to_np(zi), wi), iters
    # 3 + 2 iterations == 5 iterations (resume from the current roots)
    zr, zi = to_gpu(z0r), to_gpu(z0i)
    mpx.RootsPlan("qd", deg, iters=3, init=False, graph=False).run(gc_r, gc_i, zr, zi)
    mpx.RootsPlan("qd", deg, iters=2, init=False, graph=False).run(gc_r, gc_i, zr, zi)
    wr, wi, _ = oracle.polyroots(K, deg, cre, cim, z0r, z0i, iters=5, init=False)
    assert bits_equal(to_np(zr), wr) and bits_equal(to_np(zi), wi)


@pytest.mark.parametrize("p,K", PRECS)
def test_dk_aberth_start_close_to_oracle(p, K):
    deg, cre, cim = _dk_inputs(K, RAGGED, 30 + K)
    wr, wi, _ = oracle.polyroots(K, deg, cre, cim, iters=0, init=True)
    zr = torch.zeros((K, int(deg.sum())), dtype=torch.float64, device="cuda")
    zi = torch.zeros_like(zr)
    mpx.RootsPlan(p, deg, iters=0, init=True, graph=False).run(to_gpu(cre), to_gpu(cim), zr, zi)
    gr, gi = to_np(zr), to_np(zi)
    scale = np.maximum(np.abs(wr[0]) + np.abs(wi[0]), 1e-300)
    assert np.max((np.abs(gr[0] - wr[0]) + np.abs(gi[0] - wi[0])) / scale) < 1e-13
    assert np.all(gr[1:] == 0) and np.all(gi[1:] == 0)


def test_dk_autotune_leaves_roots_and_results_unchanged():
    """The autotuner probes every variant on a private copy of the start
    roots, keeps a valid variant in the plan (the default unless another is
    clearly faster), and the tuned plan gives the oracle's bits."""
    K = 4
    deg, cre, cim = _dk_inputs(K, RAGGED * 8, 60)
    z0r, z0i, _ = oracle.polyroots(K, deg, cre, cim, iters=0, init=True)
    wr, wi, _ = oracle.polyroots(K, deg, cre, cim, z0r, z0i, iters=5, init=False)
    plan = mpx.RootsPlan("qd", deg, iters=5, init=False, graph=False)
    gc_r, gc_i = to_gpu(cre), to_gpu(cim)
    zr, zi = to_gpu(z0r), to_gpu(z0i)
    v, ms = plan.autotune(gc_r, gc_i, zr, zi, iters_probe=2)
    assert 0 <= v < mpx.polyroots_variant_count() and ms > 0
    assert bits_equal(to_np(zr), z0r) and bits_equal(to_np(zi), z0i)   # start roots untouched
    plan.run(gc_r, gc_i, zr, zi)
    assert bits_equal(to_np(zr), wr) and bits_equal(to_np(zi), wi), v


def test_dk_graph_replay_matches_eager():
    K = 4
    deg, cre, cim = _dk_inputs(K, [16, 31, 48, 3, 9], 40)
    z0r, z0i, _ = oracle.polyroots(K, deg, cre, cim, iters=0, init=True)
    wr, wi, _ = oracle.polyroots(K, deg, cre, cim, z0r, z0i, iters=4, init=False)
    stream = torch.cuda.Stream()
    plan = mpx.RootsPlan("qd", deg, iters=4, init=False, graph=True)
    gc_r, gc_i = to_gpu(cre), to_gpu(cim)
    zr, zi = to_gpu(z0r), to_gpu(z0i)
    st = torch.zeros(deg.size, dtype=torch.int32, device="cuda")
    for rep in range(3):
        with torch.no_grad():
            zr.copy_(to_gpu(z0r)); zi.copy_(to_gpu(z0i))
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            plan.run(gc_r, gc_i, zr, zi, status=st)
        stream.synchronize()
        _ = (torch.ones(1000, device="cuda") * 2).sum().item()   # eager work between replays
        assert bits_equal(to_np(zr), wr) and bits_equal(to_np(zi), wi), rep
        assert int(to_np(st).sum()) == 0


def test_dk_plan_with_graph_flag_inside_an_outer_capture():
    """A plan created with the graph flag, called while the caller captures
    the stream, launches directly into the caller's graph; replays of that
    graph reproduce the oracle's iterates."""
    K = 4
    deg, cre, cim = _dk_inputs(K, [16, 31, 48, 3, 9], 41)
    z0r, z0i, _ = oracle.polyroots(K, deg, cre, cim, iters=0, init=True)
    wr, wi, _ = oracle.polyroots(K, deg, cre, cim, z0r, z0i, iters=3, init=False)
    plan = mpx.RootsPlan("qd", deg, iters=3, init=False, graph=True)
    gc_r, gc_i = to_gpu(cre), to_gpu(cim)
    zr, zi = to_gpu(z0r), to_gpu(z0i)
    st = torch.zeros(deg.size, dtype=torch.int32, device="cuda")
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=s):
        plan.run(gc_r, gc_i, zr, zi, status=st)
    torch.cuda.synchronize()
    for rep in range(3):
        zr.copy_(to_gpu(z0r)); zi.copy_(to_gpu(z0i))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        _ = (torch.ones(1000, device="cuda") * 2).sum().item()
        assert bits_equal(to_np(zr), wr) and bits_equal(to_np(zi), wi), rep


def test_dk_known_roots_and_status():
    K = 4
    deg, cre, cim, known = synth.dk_batch(K, 6, 16, 40, seed=50, n_known=4, known_degree=16)
    zr = torch.zeros((K, int(deg.sum())), dtype=torch.float64, device="cuda")
    zi = torch.zeros_like(zr)
    plan = mpx.RootsPlan("qd", deg, iters=200, init=True, graph=False)
    st = plan.run(to_gpu(cre), to_gpu(cim), zr, zi)
    assert int(to_np(st).sum()) == 0
    r, i = to_np(zr), to_np(zi)
    _, roff = synth.offsets(deg)
    for b in range(4):
        z = r[0, roff[b]:roff[b + 1]] + 1j * i[0, roff[b]:roff[b + 1]]
        for w in known[b]:
            assert np.min(np.abs(z - w)) < 1e-13
    # coincident start values -> non-finite -> status 1
    dz = np.array([3], np.int32)
    _, c2r, c2i = _dk_inputs(K, dz, 60)
    sr = np.zeros((K, 3)); si = np.zeros((K, 3))
    sr[0] = [0.5, 0.5, -0.3]
    zr2, zi2 = to_gpu(sr), to_gpu(si)
    st2 = mpx.RootsPlan("qd", dz, iters=2, init=False, graph=False).run(to_gpu(c2r), to_gpu(c2i), zr2, zi2)
    assert int(to_np(st2)[0]) == 1


def test_dk_full_batch_sampled_bit_exact():
    """Full-size batch (4096 QD polynomials, degrees 16..512, 200 sweeps, one
    persistent launch): polynomials of degree <= 40 sampled and re-run one by
    one in the oracle from the same start values must match bit for bit."""
    K = 4
    deg, cre, cim, known = synth.dk_batch(K, 4096, 16, 512, seed=synth.seed_for(2, 0), n_known=16)
    z0r, z0i, _ = oracle.polyroots(K, deg, cre, cim, iters=0, init=True)
    plan = mpx.RootsPlan("qd", deg, iters=200, init=False, graph=True)
    zr, zi = to_gpu(z0r), to_gpu(z0i)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        st = plan.run(to_gpu(cre), to_gpu(cim), zr, zi)
    stream.synchronize()
    r, i, s = to_np(zr), to_np(zi), to_np(st)
    coff, roff = synth.offsets(deg)
    small = [b for b in range(16, 4096) if deg[b] <= 40][:4] + [0, 1]
    for b in small:
        cs = slice(coff[b], coff[b + 1]); rs = slice(roff[b], roff[b + 1])
        wr, wi, ws = oracle.polyroots(K, deg[b:b + 1], cre[:, cs], cim[:, cs],
                                      z0r[:, rs], z0i[:, rs], iters=200, init=False)
        assert bits_equal(np.ascontiguousarray(r[:, rs]), wr), b
        assert bits_equal(np.ascontiguousarray(i[:, rs]), wi), b
        assert s[b] == ws[0]
    for b in range(16):
        z = r[0, roff[b]:roff[b + 1]] + 1j * i[0, roff[b]:roff[b + 1]]
        for w in known[b]:
            assert np.min(np.abs(z - w)) < 1e-12, b


@pytest.mark.parametrize("p,K", PRECS)
@pytest.mark.parametrize("batch,deg", [(1, 0), (3, 1), (5, 2), (70, 63), (9, 64), (33, 100), (64, 1023), (8, 2047),
                                       (1024, 2047), (5, 2048), (3, 3000), (4, 4095), (3, 4096), (2, 8191),
                                       (1024, 4095)])
def test_estrin_bit_exact(p, K, batch, deg):
    coef = synth.mp_array(K, (batch, deg + 1), 80 + deg, "U")
    x = synth.mp_array(K, batch, 81 + deg, "U")
    got = to_np(mpx.polyval(p, to_gpu(coef), to_gpu(x), method="estrin"))
    want = oracle.polyval_estrin(K, coef, x)
    assert bits_equal(got, want), first_mismatch(got, want)


def test_estrin_rejects_degree_beyond_8191():
    coef = torch.zeros((4, 2, 8193), dtype=torch.float64, device="cuda")
    x = torch.zeros((4, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(mpx.MpxError):
        mpx.polyval("qd", coef, x, method="estrin")


@pytest.mark.parametrize("p,K", PRECS)
@pytest.mark.parametrize("batch,deg", [(1, 0), (3, 1), (5, 2), (70, 63), (9, 64), (33, 100), (64, 1023),
                                       (1024, 1023), (3, 1024), (4, 2047), (2, 3001), (3, 4095)])
def test_polyval_cplx_bit_exact(p, K, batch, deg):
    """Real-coefficient polynomials at complex points, Horner and Estrin."""
    coef = synth.mp_array(K, (batch, deg + 1), 90 + deg, "U")
    xr = synth.mp_array(K, batch, 91 + deg, "U")
    xi = synth.mp_array(K, batch, 92 + deg, "U")
    for method in ("horner", "estrin"):
        gr, gi = mpx.polyval_cplx(p, to_gpu(coef), to_gpu(xr), to_gpu(xi), method=method)
        wr, wi = oracle.polyval_cplx(K, coef, xr, xi, method)
        assert bits_equal(to_np(gr), wr), (method, first_mismatch(to_np(gr), wr))
        assert bits_equal(to_np(gi), wi), method


@pytest.mark.parametrize("p,K,mode", [("qd_nobf", 4, "nobf"), ("td_nobf", 3, "nobf"),
                                      ("dd_nobf_acc", 2, "nobf_acc")])
def test_polyval_cplx_conventional_bit_exact(p, K, mode):
    coef = synth.mp_array(K, (130, 258), 95, "U")
    xr = synth.mp_array(K, 130, 96, "U")
    xi = synth.mp_array(K, 130, 97, "U")
    with oracle.arith(mode):
        wr, wi = oracle.polyval_cplx(K, coef, xr, xi)
    gr, gi = mpx.polyval_cplx(p, to_gpu(coef), to_gpu(xr), to_gpu(xi))
    assert bits_equal(to_np(gr), wr) and bits_equal(to_np(gi), wi)


def test_polyval_cplx_estrin_limits():
    coef = torch.zeros((4, 2, 4097), dtype=torch.float64, device="cuda")
    x = torch.zeros((4, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(mpx.MpxError):
        mpx.polyval_cplx("qd", coef, x, x.clone(), method="estrin")          # degree 4096
    with pytest.raises(mpx.MpxError):
        mpx.polyval_cplx("qd_nobf", coef[:, :, :4].contiguous(), x, x.clone(), method="estrin")
