"""The allocation-free dot (mpx_dot_noalloc, a static device scratch instead
of a caller workspace), called through the C ABI, gives the same bits as
mpx_dot with a workspace: two calls in a row, the second with a smaller
input, for every precision, plus single-block sizes that need no scratch."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2603_14926_amd import mpx, synth
from tests.gpu_util import bits_equal, to_gpu, to_np

pytestmark = pytest.mark.gpu

PRECS = [("qd", 4, np.float64), ("td", 3, np.float64), ("dd", 2, np.float64), ("ff", 2, np.float32)]


def _noalloc(p, x, y):
    """mpx_dot_noalloc through ctypes on the current stream."""
    L = mpx.lib()
    K, n = x.shape
    out = torch.full((K,), float("nan"), dtype=x.dtype, device="cuda")
    st = L.mpx_dot_noalloc(mpx.prec_of(p), n, C.c_void_p(x.data_ptr()), x.stride(0),
                           C.c_void_p(y.data_ptr()), y.stride(0), C.c_void_p(out.data_ptr()),
                           C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, st
    return out


@pytest.mark.parametrize("p,K,dt", PRECS)
@pytest.mark.parametrize("sizes", [(100003, 4097), (1 << 20, 300), (65536, 257), (256, 17)])
def test_noalloc_dot_matches_workspace_dot(p, K, dt, sizes):
    for i, n in enumerate(sizes):          # the second call is smaller
        x = to_gpu(synth.mp_array(K, n, 500 + n % 1000 + i, "W", dtype=dt))
        y = to_gpu(synth.mp_array(K, n, 600 + n % 1000 + i, "W", dtype=dt))
        want = to_np(mpx.dot(p, x, y))
        got = to_np(_noalloc(p, x, y))
        torch.cuda.synchronize()
        assert bits_equal(got, want), (p, n, got, want)


def test_noalloc_dot_rejects_bad_arguments():
    L = mpx.lib()
    fake = C.c_void_p(1 << 20)
    assert L.mpx_dot_noalloc(4, 10, fake, 10, fake, 10, None, None) == -1      # no result
    assert L.mpx_dot_noalloc(7, 10, fake, 10, fake, 10, fake, None) == -2      # unknown precision
    assert L.mpx_dot_noalloc(4, 10, fake, 9, fake, 10, fake, None) == -1       # plane stride < n
