"""The Python binding rejects outputs and operands whose shape or layout
differs from what the call computes (before any launch): the library writes
the whole extent given by the plane stride and leading dimension, so a
smaller view, or an imaginary part laid out differently from the real part,
would be written past its end."""
import pytest

torch = pytest.importorskip("torch")

from paper_2603_14926_amd import mpx

pytestmark = pytest.mark.gpu


def _z(*shape, dtype=torch.float64):
    return torch.zeros(shape, dtype=dtype, device="cuda")


def test_wrong_output_shapes_rejected():
    K = 4
    x, y = _z(K, 10), _z(K, 10)
    A, B = _z(K, 6, 5), _z(K, 5, 7)
    with pytest.raises(ValueError):
        mpx.add("qd", x, y, out=_z(K, 9))
    with pytest.raises(ValueError):
        mpx.dot("qd", x, y, out=_z(K + 1))
    with pytest.raises(ValueError):
        mpx.gemv("qd", A, _z(K, 5), out=_z(K, 5))            # 6 rows
    with pytest.raises(ValueError):
        mpx.gemm("qd", A, B, out=_z(K, 12, 5)[:, :6, :5])     # a 6 x 5 view, 7 columns needed
    with pytest.raises(ValueError):
        mpx.gemm("qd", A, B, out=_z(K, 7, 7))
    with pytest.raises(ValueError):
        mpx.gemm_strassen("qd", A, B, 2, out=_z(K, 6, 6))
    with pytest.raises(ValueError):
        mpx.gemm_ozaki_dd(_z(2, 6, 5), _z(2, 5, 7), 3, out=_z(2, 6, 6))
    with pytest.raises(ValueError):
        mpx.polyval("qd", _z(K, 10, 4), _z(K, 10), out=_z(K, 9))
    with pytest.raises(ValueError):
        mpx.polyval_backward("qd", _z(K, 10, 4), _z(K, 9), _z(K, 10))


def test_complex_parts_must_share_a_layout():
    K = 2
    A, B = _z(K, 6, 5), _z(K, 5, 7)
    Cre = _z(K, 6, 7)
    with pytest.raises(ValueError):
        mpx.cgemm_3m("dd", A, A, B, B, out=(Cre, _z(K, 6, 6)))
    with pytest.raises(ValueError):
        mpx.cgemm_3m("dd", A, A, B, B, out=(Cre, _z(K, 6, 8)[:, :, :7]))   # same shape, ld 8
    with pytest.raises(ValueError):
        mpx.cgemm_3m("dd", A, _z(K, 6, 6)[:, :, :5], B, B)
    coef = _z(K, 10, 4)
    with pytest.raises(ValueError):
        mpx.polyval_cplx("dd", coef, _z(K, 10), _z(K, 12)[:, :10])           # plane strides differ
    with pytest.raises(ValueError):
        mpx.polyval_cplx("dd", coef, _z(K, 10), _z(K, 10), out=(_z(K, 10), _z(K, 9)))


def test_plan_operands_checked():
    plan = mpx.GemmBatchPlan("dd", [4, 3], [4, 2], [4, 5])
    _, _, _, (ta, tb, tc) = plan.offsets()
    A, B, C = _z(2, ta), _z(2, tb), _z(2, tc)
    with pytest.raises(ValueError):
        plan.run(A, B, _z(2, tc - 1))
    with pytest.raises(ValueError):
        plan.run(_z(2, ta + 1)[:, :ta - 1], B, C)
    rp = mpx.RootsPlan("dd", [3, 5], iters=1, init=True, graph=False)
    cre, cim = _z(2, rp.total_coef), _z(2, rp.total_coef)
    zr, zi = _z(2, rp.total_roots), _z(2, rp.total_roots)
    with pytest.raises(ValueError):
        rp.run(cre, cim, zr, zi, status=torch.zeros(1, dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError):
        rp.run(cre, cim, zr, zi, status=torch.zeros(2, dtype=torch.int64, device="cuda"))


def test_root_solver_rejects_overlapping_buffers():
    """The library (called directly): roots overlapping the coefficients or
    each other, and a status array overlapping any of them, are argument
    errors returned before any launch (ranges cover all K planes)."""
    import ctypes as C
    L = mpx.lib()
    rp = mpx.RootsPlan("dd", [3, 5], iters=1, init=True, graph=False)
    cre, cim = _z(2, rp.total_coef), _z(2, rp.total_coef)
    zr, zi = _z(2, rp.total_roots), _z(2, rp.total_roots)
    pc, pr = cre.stride(0), zr.stride(0)
    ptr = lambda t, off=0: C.c_void_p(t.data_ptr() + 8 * off)
    h = rp._h
    assert L.mpx_polyroots(h, ptr(cre), ptr(cim), pc, ptr(cre), ptr(zi), pr, None, None) == -1
    assert L.mpx_polyroots(h, ptr(cre), ptr(cim), pc, ptr(zr), ptr(cim, 3), pr, None, None) == -1
    assert L.mpx_polyroots(h, ptr(cre), ptr(cim), pc, ptr(zr), ptr(zr, 2), pr, None, None) == -1
    assert L.mpx_polyroots(h, ptr(cre), ptr(cim), pc, ptr(zr), ptr(zi), pr, ptr(zi, 1), None) == -1
    # the same buffers without overlap are accepted (and solved)
    st = torch.zeros(2, dtype=torch.int32, device="cuda")
    cre[0, 0] = -1.0; cre[0, 3] = 1.0                # x^3 - 1
    cre[0, 4] = -1.0; cre[0, 9] = 1.0                # x^5 - 1
    mpx.RootsPlan("dd", [3, 5], iters=0, init=True, graph=False).run(cre, cim, zr, zi)
    assert L.mpx_polyroots(h, ptr(cre), ptr(cim), pc, ptr(zr), ptr(zi), pr, ptr(st), None) == 0
    torch.cuda.synchronize()
