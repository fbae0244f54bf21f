"""GPU parity of the vector kernels at the size the benchmark times them for
bandwidth (n = 2^24, grid-stride launches with the full block counts):
elementwise add / mul and AXPY bit-exact on sampled indices, dot within
twice the reduction bound of the oracle's sequential dot (both are within
n 2^-b sum |x_i y_i| of the exact value, so they are within twice that of
each other)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2603_14926_amd import mpx, synth
from tests.gpu_util import bits_equal, first_mismatch, to_gpu, to_np

pytestmark = pytest.mark.gpu

N = 1 << 24
BITS = {2: 104, 3: 155, 4: 208}
NAMES = {2: "dd", 3: "td", 4: "qd"}


@pytest.fixture(scope="module")
def vectors():
    # the leading K components of a renormalised QD expansion are a valid
    # non-overlapping K-component value, so one pair serves DD, TD and QD
    x = synth.mp_array(4, N, 77, "U")
    y = synth.mp_array(4, N, 78, "U")
    rng = np.random.default_rng(3)
    idx = np.unique(np.concatenate([np.arange(64), N - 64 + np.arange(64),
                                    rng.integers(0, N, 4000)]))
    return x, y, idx


@pytest.mark.parametrize("K", [2, 3, 4])
def test_elementwise_and_axpy_2p24_sampled(vectors, K):
    x, y, idx = vectors
    xs, ys = np.ascontiguousarray(x[:K]), np.ascontiguousarray(y[:K])
    gx, gy = to_gpu(xs), to_gpu(ys)
    p = NAMES[K]
    xi, yi = np.ascontiguousarray(xs[:, idx]), np.ascontiguousarray(ys[:, idx])
    got = to_np(mpx.add(p, gx, gy)[:, idx])
    want = oracle.add(K, xi, yi)
    assert bits_equal(got, want), first_mismatch(got, want)
    got = to_np(mpx.mul(p, gx, gy)[:, idx])
    want = oracle.mul(K, xi, yi)
    assert bits_equal(got, want), first_mismatch(got, want)
    alpha = synth.mp_array(K, 1, 5, "U")[:, 0]
    mpx.axpy(p, alpha.tolist(), gx, gy)
    got = to_np(gy[:, idx])
    want = oracle.axpy(K, alpha, xi, yi)
    assert bits_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_dot_2p24_against_oracle(vectors, K):
    x, y, _ = vectors
    xs, ys = np.ascontiguousarray(x[:K]), np.ascontiguousarray(y[:K])
    got = to_np(mpx.dot(NAMES[K], to_gpu(xs), to_gpu(ys)))
    want = oracle.dot(K, xs, ys)
    diff = oracle.op1(K, "add", got, -want)
    scale = float(np.sum(np.abs(xs[0] * ys[0]))) * (1 + 1e-10)
    assert abs(diff[0]) <= 2 * N * 2.0 ** -BITS[K] * scale, (diff[0], scale)
