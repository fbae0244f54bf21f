"""GPU parity of the Ozaki-split DD GEMM on FP64 MFMA against the CPU oracle's
implementation of the same definition (bit-exact: slices and level sums are
exact integers, the DD fold runs in a fixed order), plus its error against
exact arithmetic."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from oracle import exact
from paper_2603_14926_amd import mpx, synth
from tests.gpu_util import bits_equal, first_mismatch, to_gpu, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("s", [1, 3, 6, 7, 9, 12])
@pytest.mark.parametrize("mnk", [(16, 16, 8), (70, 45, 130), (129, 64, 300)])
def test_ozaki_bit_exact_vs_oracle(s, mnk):
    m, n, k = mnk
    A = synth.mp_array(2, (m, k), 1 + s, "W", phi=4.0)
    B = synth.mp_array(2, (k, n), 2 + s, "W", phi=4.0)
    got = to_np(mpx.gemm_ozaki_dd(to_gpu(A), to_gpu(B), s, beta=20, kblk=64))
    rows = np.repeat(np.arange(m), n); cols = np.tile(np.arange(n), m)
    want = oracle.ozaki_entries(A, B, rows, cols, s=s, beta=20, kblk=64).reshape(2, m, n)
    assert bits_equal(got, want), first_mismatch(got, want)


def test_ozaki_zero_k_and_zero_rows():
    A = np.zeros((2, 20, 0)); B = np.zeros((2, 0, 9))
    got = to_np(mpx.gemm_ozaki_dd(to_gpu(A), to_gpu(B), 4))
    assert np.all(got == 0)
    A = synth.mp_array(2, (20, 40), 5, "U"); A[:, 3, :] = 0.0
    B = synth.mp_array(2, (40, 9), 6, "U")
    got = to_np(mpx.gemm_ozaki_dd(to_gpu(A), to_gpu(B), 7))
    assert np.all(got[:, 3, :] == 0)


@pytest.mark.parametrize("phi", [1.0, 4.0, 8.0])
def test_ozaki_4096_sampled_error_and_parity(phi):
    """n = 4096: sampled entries bit-exact vs the oracle's Ozaki, and the
    error of enough slices within n 2^-104 sum |a b| of the exact product."""
    n = 4096
    s = {1.0: 7, 4.0: 8, 8.0: 10}[phi]
    A = synth.mp_array(2, (n, n), synth.seed_for(4, int(phi)), "W", phi=phi)
    B = synth.mp_array(2, (n, n), synth.seed_for(4, 10 + int(phi)), "W", phi=phi)
    got = to_np(mpx.gemm_ozaki_dd(to_gpu(A), to_gpu(B), s, beta=20, kblk=256))
    # rows cover every position inside a 16-row MFMA tile and the tile edges
    rows = np.array([0, 1, 2, 3, 4, 7, 9, 14, 15, 2049, 4094, 4095]); cols = np.array([4095, 77, 2048, 0, 31, 16, 1, 2, 3, 4094, 5, 17])
    want = oracle.ozaki_entries(A, B, rows, cols, s=s, beta=20, kblk=256)
    assert bits_equal(np.ascontiguousarray(got[:, rows, cols]), want)
    for t in range(rows.size):
        ex = exact.dot(np.ascontiguousarray(A[:, rows[t], :]), np.ascontiguousarray(B[:, :, cols[t]]))
        sc = exact.abs_dot(A[:, rows[t], :], B[:, :, cols[t]])
        err = float(abs(exact.value(got[:, rows[t], cols[t]]) - ex)) / sc
        assert err <= n * 2.0 ** -104, (phi, t, err)


@pytest.mark.parametrize("s,beta,kblk", [(6, 23, 64), (7, 22, 128), (9, 22, 128)])
def test_ozaki_wider_slices_smaller_blocks_bit_exact(s, beta, kblk):
    """The benchmark's other exact (slices, beta, k-block) choices."""
    m, n, k = 70, 45, 300
    A = synth.mp_array(2, (m, k), 600 + s, "W", phi=8.0)
    B = synth.mp_array(2, (k, n), 700 + s, "W", phi=8.0)
    got = to_np(mpx.gemm_ozaki_dd(to_gpu(A), to_gpu(B), s, beta=beta, kblk=kblk))
    rows, cols = np.divmod(np.arange(m * n), n)
    want = oracle.ozaki_entries(A, B, rows, cols, s=s, beta=beta, kblk=kblk).reshape(2, m, n)
    assert bits_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("kblk,k", [(16, 200), (48, 130), (32, 32)])
def test_ozaki_block_exponents_bit_exact(kblk, k):
    """k-blocks of very different magnitude (each gets its own exponents), a
    zero block, and a ragged last block: bit-exact against the oracle."""
    m, n = 37, 70
    A = synth.mp_array(2, (m, k), 900 + k, "W", phi=2.0)
    B = synth.mp_array(2, (k, n), 901 + k, "W", phi=2.0)
    blk = np.arange(k) // kblk
    A *= (2.0 ** (-7 * blk))[None, None, :]      # exact power-of-two scalings
    B *= (2.0 ** (-3 * blk))[None, :, None]
    A[:, 5, :kblk] = 0.0
    got = to_np(mpx.gemm_ozaki_dd(to_gpu(A), to_gpu(B), 5, beta=21, kblk=kblk))
    rows, cols = np.divmod(np.arange(m * n), n)
    want = oracle.ozaki_entries(A, B, rows, cols, s=5, beta=21, kblk=kblk).reshape(2, m, n)
    assert bits_equal(got, want), first_mismatch(got, want)


@pytest.fixture
def oz_variant():
    """Stage-depth variant of the slice GEMM, restored to the default after."""
    yield mpx.gemm_ozaki_set_variant
    mpx.gemm_ozaki_set_variant(0)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("s,beta,kblk", [(s, 20, 64) for s in range(1, 13)] +
                         [(4, 22, 256), (5, 22, 256), (6, 22, 256)])
@pytest.mark.parametrize("mnk", [(70, 45, 300), (129, 97, 530)])
def test_ozaki_every_slice_count_and_stage_variant(oz_variant, variant, s, beta, kblk, mnk):
    """Every slice count 1..12, the benchmark's exact (slices, 22, 256)
    choices, and both LDS stage depths (8 and 16 k per stage), at shapes
    ragged against the 32-row / 32-column MFMA tiles and the k-blocks."""
    m, n, k = mnk
    oz_variant(variant)
    A = synth.mp_array(2, (m, k), 1100 + 13 * s + kblk, "W", phi=4.0)
    B = synth.mp_array(2, (k, n), 1200 + 13 * s + kblk, "W", phi=4.0)
    got = to_np(mpx.gemm_ozaki_dd(to_gpu(A), to_gpu(B), s, beta=beta, kblk=kblk))
    rows, cols = np.divmod(np.arange(m * n), n)
    want = oracle.ozaki_entries(A, B, rows, cols, s=s, beta=beta, kblk=kblk).reshape(2, m, n)
    assert bits_equal(got, want), (variant, first_mismatch(got, want))
