// mpx_ozaki.hip -- Ozaki-style split DD GEMM on the FP64 matrix cores of gfx950.
//
// Section 3.1 lists the Ozaki scheme among the GEMM schemes of the paper's
// library without giving it; this is the reading implemented (the CPU
// reference implements the same definition independently):
//
//  1. exponents per k-block b of kblk consecutive k: e_ib with
//     max_{l in b} |A_il.hi| < 2^{e_ib} (frexp of the block maximum; 0 for a
//     zero block), f_jb likewise for the columns of B; a block of small
//     entries is so split relative to its own size, not to the row's;
//  2. error-free split of each DD element (hi, lo) into s integer slices:
//     m_p = rint(r1 * 2^{p beta - e}), then (r1, r2) := TwoSum(r1 - m_p
//     2^{e - p beta}, r2), p = 1..s, starting from (r1, r2) = (hi, lo), e
//     the exponent of the element's block;
//  3. for each k-block of kblk columns and each level g = p + q
//     (2 <= g <= s + 1) the level sum S_g = sum_{p+q=g} sum_l mA_p mB_q is
//     an integer below 2^53 (kblk (g-1) 2^{2 beta} < 2^53), so binary64
//     accumulation is exact in any order -- here the MFMA units compute it;
//  4. C_ij = DWBFAdd-accumulation, k-blocks ascending and g ascending, of
//     (S_g 2^{e_ib + f_jb - g beta}, 0).
//
// Kernels: row / column maxima, the split (VALU, HBM-bound, writes the s
// integer slice planes of A and B zero-padded to the tile grid), and the
// slice GEMM: a 256-thread workgroup owns a 64 x 64 tile of C, each wave a
// 32 x 32 sub-tile = 2 x 2 tiles of v_mfma_f64_16x16x4_f64, holding s level
// accumulators per tile (they live in AGPRs / VGPRs); the s slice planes of
// an A panel (64 x 8) and a B panel (8 x 64) are staged in LDS per step.
// After each k-block the levels are folded into per-element DD accumulators
// with the branch-free DD addition.
#include "mp_arith.hpp"
#include "mpx_internal.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>

namespace mpx {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef double d2_t __attribute__((ext_vector_type(2)));

constexpr int OZ_BM = 64, OZ_BN = 64, OZ_KPAD = 16, OZ_THREADS = 256;
constexpr int OZ_MAX_S = 12;

__device__ __forceinline__ int exp_of(double m) {
    return m == 0.0 ? 0 : __builtin_amdgcn_frexp_exp(m);  // m = f 2^e, 0.5 <= f < 1
}

// Block exponents are stored block-major: e[b * mp + i], f[b * np + j], so
// the fold of block b reads one contiguous run of each.

// e_ib for row i of A (hi plane): one wave per row, blocks in turn.
__global__ void __launch_bounds__(256)
k_oz_row_exp(long long m, long long k, const double* __restrict__ A, long long lda,
             long long kblk, int* __restrict__ e, long long mp) {
    const long long row = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= m) return;
    for (long long l0 = 0, b = 0; l0 < k; l0 += kblk, ++b) {
        const long long l1 = l0 + kblk < k ? l0 + kblk : k;
        double mx = 0.0;
        for (long long l = l0 + lane; l < l1; l += 64) mx = fmax(mx, fabs(A[row * lda + l]));
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
        if (lane == 0) e[b * mp + row] = exp_of(mx);
    }
}

// f_jb for column j of B (hi plane): one thread per (column, block), the
// block's rows in turn; grid.y strides over the nb blocks.
__global__ void __launch_bounds__(256)
k_oz_col_exp(long long k, long long n, const double* __restrict__ B, long long ldb,
             long long kblk, long long nb, int* __restrict__ f, long long np) {
    const long long j = (long long)blockIdx.x * 256 + threadIdx.x;
    if (j >= n) return;
    for (long long b = blockIdx.y; b < nb; b += gridDim.y) {
        const long long l0 = b * kblk, l1 = l0 + kblk < k ? l0 + kblk : k;
        double mx = 0.0;
        for (long long l = l0; l < l1; ++l) mx = fmax(mx, fabs(B[l * ldb + j]));
        f[b * np + j] = exp_of(mx);
    }
}

// Split one DD value into s integer slices (step 2 above).
template <int S>
__device__ __forceinline__ void split_dd(double hi, double lo, int e, int beta, double* out) {
    double r1 = hi, r2 = lo;
#pragma unroll
    for (int p = 1; p <= S; ++p) {
        const double q = rint(__builtin_amdgcn_ldexp(r1, p * beta - e));
        const double d = r1 - __builtin_amdgcn_ldexp(q, e - p * beta);
        ts(d, r2, r1, r2);
        out[p - 1] = q;
    }
}

// Slices of A into SA[p][l][i] (planes of kp x mp: k-major, so a 64-row A
// panel of one k is contiguous), of B into SB[p][l][j] (planes of kp x np);
// padding rows / columns are zero.
template <int S>
__global__ void __launch_bounds__(256)
k_oz_split_a(long long m, long long k, const double* __restrict__ A, long long lda,
             long long psA, const int* __restrict__ e, long long kblk, int beta,
             double* __restrict__ SA, long long mp, long long kp) {
    const long long total = mp * kp;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (long long)gridDim.x * 256) {
        const long long l = t / mp, i = t % mp;
        double sl[S];
        if (i < m && l < k) {
            split_dd<S>(A[i * lda + l], A[psA + i * lda + l], e[(l / kblk) * mp + i], beta, sl);
        } else {
#pragma unroll
            for (int p = 0; p < S; ++p) sl[p] = 0.0;
        }
#pragma unroll
        for (int p = 0; p < S; ++p) SA[p * total + t] = sl[p];
    }
}

template <int S>
__global__ void __launch_bounds__(256)
k_oz_split_b(long long k, long long n, const double* __restrict__ B, long long ldb,
             long long psB, const int* __restrict__ f, long long kblk, int beta,
             double* __restrict__ SB, long long kp, long long np) {
    const long long total = kp * np;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (long long)gridDim.x * 256) {
        const long long l = t / np, j = t % np;
        double sl[S];
        if (l < k && j < n) {
            split_dd<S>(B[l * ldb + j], B[psB + l * ldb + j], f[(l / kblk) * np + j], beta, sl);
        } else {
#pragma unroll
            for (int p = 0; p < S; ++p) sl[p] = 0.0;
        }
#pragma unroll
        for (int p = 0; p < S; ++p) SB[p * total + t] = sl[p];
    }
}

// Slice GEMM with level accumulation on MFMA and the DD fold.
//
// v_mfma_f64_16x16x4_f64 operand layout (wave64): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] of the 16x4 and 4x16 operands and
// holds D[l / 16 + 4 v][l % 16], v = 0..3, of the 16x16 result.
//
// Workgroup = 2 x 2 waves, each wave TA x TB MFMA tiles (16 x 16 each).  Per
// stage of OZ_KT = 8 k values the S slice panels of A (k-major, 8 x BM) and B
// (8 x BN) are copied into LDS with 16-byte loads that were issued one stage
// ahead (register prefetch).  LDS rows are padded by 16 doubles so the four
// k rows a wave reads at once fall in different bank halves.
template <int S, int TA, int TB, int OZ_KT>
__global__ void __launch_bounds__(OZ_THREADS)
k_oz_gemm(long long m, long long n, long long mp, long long np, long long kp,
          const double* __restrict__ SA, const double* __restrict__ SB,
          const int* __restrict__ e, const int* __restrict__ f, int beta, long long kblk,
          double* __restrict__ C, long long ldc, long long psC, int tiles_n) {
    constexpr int BM = 32 * TA, BN = 32 * TB;
    constexpr int LDA = BM + 16, LDB = BN + 16;
    constexpr int A_V2 = (S * OZ_KT * BM / 2 + OZ_THREADS - 1) / OZ_THREADS;
    constexpr int B_V2 = (S * OZ_KT * BN / 2 + OZ_THREADS - 1) / OZ_THREADS;
    __shared__ __attribute__((aligned(16))) double sA[S][OZ_KT][LDA];
    __shared__ __attribute__((aligned(16))) double sB[S][OZ_KT][LDB];

    const int tile = blockIdx.x;
    const long long m0 = (long long)(tile / tiles_n) * BM;
    const long long n0 = (long long)(tile % tiles_n) * BN;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wr = (w >> 1) * 16 * TA, wc = (w & 1) * 16 * TB;  // wave sub-tile origin
    const int lr = lane & 15, lk = lane >> 4;

    d4_t acc[S][TA][TB];
#pragma unroll
    for (int g = 0; g < S; ++g)
#pragma unroll
        for (int a = 0; a < TA; ++a)
#pragma unroll
            for (int b = 0; b < TB; ++b) acc[g][a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
    mpn<double, 2> dd[TA][TB][4];
#pragma unroll
    for (int a = 0; a < TA; ++a)
#pragma unroll
        for (int b = 0; b < TB; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) dd[a][b][v] = mp_zero<double, 2>();

    // Staging: thread tid moves 16-byte pairs v = tid + it*256 of the A panel
    // (S slices x 8 k x BM rows) and the B panel (S x 8 x BN).  When the count
    // is not a multiple of 256 the last pairs are clamped: two threads then copy
    // the same pair to the same place (no condition, so the prefetch registers
    // stay in VGPRs).
    const long long plA = mp * kp, plB = kp * np;
    constexpr int NA = S * OZ_KT * BM / 2, NB = S * OZ_KT * BN / 2;
    d2_t ra[A_V2], rb[B_V2];
    int oa[A_V2], ob[B_V2];          // LDS double offsets
    long long ga[A_V2], gb[B_V2];    // global offsets for k = 0
#pragma unroll
    for (int it = 0; it < A_V2; ++it) {
        int v = tid + it * OZ_THREADS;
        v = v < NA ? v : NA - 1;
        const int p = v / (OZ_KT * BM / 2), rem = v % (OZ_KT * BM / 2);
        const int kk = rem / (BM / 2), i2 = rem % (BM / 2);
        oa[it] = (p * OZ_KT + kk) * LDA + 2 * i2;
        ga[it] = p * plA + (long long)kk * mp + m0 + 2 * i2;
    }
#pragma unroll
    for (int it = 0; it < B_V2; ++it) {
        int v = tid + it * OZ_THREADS;
        v = v < NB ? v : NB - 1;
        const int p = v / (OZ_KT * BN / 2), rem = v % (OZ_KT * BN / 2);
        const int kk = rem / (BN / 2), j2 = rem % (BN / 2);
        ob[it] = (p * OZ_KT + kk) * LDB + 2 * j2;
        gb[it] = p * plB + (long long)kk * np + n0 + 2 * j2;
    }
    auto fetch = [&](long long kc) __attribute__((always_inline)) {
#pragma unroll
        for (int it = 0; it < A_V2; ++it)
            ra[it] = *reinterpret_cast<const d2_t*>(SA + ga[it] + kc * mp);
#pragma unroll
        for (int it = 0; it < B_V2; ++it)
            rb[it] = *reinterpret_cast<const d2_t*>(SB + gb[it] + kc * np);
    };
    auto stash = [&]() __attribute__((always_inline)) {
#pragma unroll
        for (int it = 0; it < A_V2; ++it)
            *reinterpret_cast<d2_t*>(&sA[0][0][0] + oa[it]) = ra[it];
#pragma unroll
        for (int it = 0; it < B_V2; ++it)
            *reinterpret_cast<d2_t*>(&sB[0][0][0] + ob[it]) = rb[it];
    };
    // fold of k-block blk: its level sums scaled by that block's exponents
    auto fold = [&](long long blk) __attribute__((always_inline)) {
        const int* __restrict__ eb = e + blk * mp;
        const int* __restrict__ fb = f + blk * np;
#pragma unroll
        for (int a = 0; a < TA; ++a)
#pragma unroll
            for (int b = 0; b < TB; ++b) {
                const long long j = n0 + wc + 16 * b + lr;
                const int fj = j < n ? fb[j] : 0;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const long long i = m0 + wr + 16 * a + lk + 4 * v;
                    const int ei = i < m ? eb[i] : 0;
#pragma unroll
                    for (int g = 0; g < S; ++g) {
                        mpn<double, 2> t;
                        t.c[0] = __builtin_amdgcn_ldexp(acc[g][a][b][v], ei + fj - (g + 2) * beta);
                        t.c[1] = 0.0;
                        dd[a][b][v] = bf_add(dd[a][b][v], t);
                    }
                }
#pragma unroll
                for (int g = 0; g < S; ++g) acc[g][a][b] = d4_t{0.0, 0.0, 0.0, 0.0};
            }
    };

    if (kp > 0) fetch(0);
    // k-blocks [0, kblk), [kblk, 2 kblk), ... (the padded tail beyond k holds
    // zero slices); the level sums are folded once per block.
    for (long long kb = 0, blk = 0; kb < kp; kb += kblk, ++blk) {
        const long long kend = kb + kblk < kp ? kb + kblk : kp;
        for (long long kc = kb; kc < kend; kc += OZ_KT) {
            __syncthreads();  // previous stage consumed
            stash();
            __syncthreads();
            if (kc + OZ_KT < kp) fetch(kc + OZ_KT);  // in flight during the MFMAs below
#pragma unroll
            for (int ks = 0; ks < OZ_KT; ks += 4) {
                double fb[S][TB];
#pragma unroll
                for (int q = 0; q < S; ++q)
#pragma unroll
                    for (int b = 0; b < TB; ++b) fb[q][b] = sB[q][ks + lk][wc + 16 * b + lr];
#pragma unroll
                for (int p = 0; p < S; ++p) {
                    double fa[TA];
#pragma unroll
                    for (int a = 0; a < TA; ++a) fa[a] = sA[p][ks + lk][wr + 16 * a + lr];
                    // slice pairs (p+1, q+1) with p + q + 2 <= S + 1 feed level p + q
#pragma unroll
                    for (int q = 0; q < S; ++q) {
                        if (p + q < S) {
#pragma unroll
                            for (int a = 0; a < TA; ++a)
#pragma unroll
                                for (int b = 0; b < TB; ++b)
                                    acc[p + q][a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                        fa[a], fb[q][b], acc[p + q][a][b], 0, 0, 0);
                        }
                    }
                }
            }
        }
        fold(blk);
    }
#pragma unroll
    for (int a = 0; a < TA; ++a)
#pragma unroll
        for (int b = 0; b < TB; ++b) {
            const long long j = n0 + wc + 16 * b + lr;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const long long i = m0 + wr + 16 * a + lk + 4 * v;
                if (i < m && j < n) mp_store<double, 2>(C, psC, i * ldc + j, dd[a][b][v]);
            }
        }
}

// Wave tile in 16x16 MFMA tiles: 2 x 1 up to 6 slices, 1 x 1 beyond (the
// level accumulators, 4 doubles per tile and level, must fit the registers).
constexpr int oz_ta(int S) { return S <= 6 ? 2 : 1; }

// Stage depth of the slice GEMM: 0 = 8 k per LDS stage, 1 = 16 k per stage.
static std::atomic<int> g_oz_variant{0};  // read by every call, set by mpx_gemm_ozaki_set_variant

static bool oz_exact(int slices, int beta, long long kblk) {
    if (beta > 26) return false;
    const long double per_k = ldexpl(1.0L, 2 * beta) * (1.0L + (slices > 2 ? (slices - 2) / 4.0L : 0.0L));
    return (long double)kblk * per_k <= ldexpl(1.0L, 53);
}

struct OzDims {
    long long mp, np, kp;
};
static OzDims oz_dims(long long m, long long n, long long k) {
    // padded to the largest tile (64 x 64) so one layout serves every s
    return {ceil_div(m, OZ_BM) * OZ_BM, ceil_div(n, OZ_BN) * OZ_BN, ceil_div(k, OZ_KPAD) * OZ_KPAD};
}

// Block exponents are sized for the smallest block (kblk = 16), so the size
// does not depend on kblk: at most kp / 16 blocks.
size_t ozaki_workspace(long long m, long long n, long long k, int slices) {
    if (slices < 1 || slices > OZ_MAX_S) return 0;
    const OzDims d = oz_dims(m, n, k);
    const size_t sl = (size_t)slices * (size_t)(d.mp * d.kp + d.kp * d.np) * sizeof(double);
    const size_t nb_max = (size_t)(d.kp / OZ_KPAD);
    return sl + nb_max * (size_t)(d.mp + d.np) * sizeof(int) + 512;
}

template <int S>
static int oz_run(long long m, long long n, long long k, const double* A, long long lda,
                  long long psA, const double* B, long long ldb, long long psB, double* C,
                  long long ldc, long long psC, int beta, long long kblk, void* ws,
                  hipStream_t s) {
    const OzDims d = oz_dims(m, n, k);
    char* p = (char*)ws;
    double* SA = (double*)p;
    p += (size_t)S * d.mp * d.kp * sizeof(double);
    double* SB = (double*)p;
    p += (size_t)S * d.kp * d.np * sizeof(double);
    const long long nb = ceil_div(k, kblk);  // == ceil(kp / kblk): kblk is a multiple of 16
    int* e = (int*)p;                         // nb x mp, block-major
    int* f = e + nb * d.mp;                   // nb x np
    int st;
    if (k > 0) {
        k_oz_row_exp<<<(unsigned)ceil_div(m, 4), 256, 0, s>>>(m, k, A, lda, kblk, e, d.mp);
        if ((st = launch_status())) return st;
        const unsigned gy = (unsigned)std::min<long long>(nb, 65535);
        k_oz_col_exp<<<dim3((unsigned)ceil_div(n, 256), gy), 256, 0, s>>>(k, n, B, ldb, kblk, nb, f,
                                                                          d.np);
        if ((st = launch_status())) return st;
    }
    const long long ta = d.mp * d.kp, tb = d.kp * d.np;
    if (ta > 0)
    k_oz_split_a<S><<<(unsigned)std::min<long long>(ceil_div(ta, 256), 65536), 256, 0, s>>>(
        m, k, A, lda, psA, e, kblk, beta, SA, d.mp, d.kp);
    if ((st = launch_status())) return st;
    if (tb > 0)
    k_oz_split_b<S><<<(unsigned)std::min<long long>(ceil_div(tb, 256), 65536), 256, 0, s>>>(
        k, n, B, ldb, psB, f, kblk, beta, SB, d.kp, d.np);
    if ((st = launch_status())) return st;
    constexpr int TA = oz_ta(S);
    const int tn = (int)(d.np / 32), tm = (int)(d.mp / (32 * TA));
    if (g_oz_variant.load(std::memory_order_relaxed) == 1)
        k_oz_gemm<S, TA, 1, 16><<<(unsigned)(tn * tm), OZ_THREADS, 0, s>>>(
            m, n, d.mp, d.np, d.kp, SA, SB, e, f, beta, kblk, C, ldc, psC, tn);
    else
        k_oz_gemm<S, TA, 1, 8><<<(unsigned)(tn * tm), OZ_THREADS, 0, s>>>(
            m, n, d.mp, d.np, d.kp, SA, SB, e, f, beta, kblk, C, ldc, psC, tn);
    return launch_status();
}

}  // namespace mpx

using namespace mpx;

extern "C" int mpx_gemm_ozaki_dd(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                                 int64_t psA, const double* B, int64_t ldb, int64_t psB,
                                 double* C, int64_t ldc, int64_t psC, int slices, int beta,
                                 int64_t kblk, void* ws, size_t ws_bytes, void* stream) {
    if (m < 0 || n < 0 || k < 0) return MPX_EINVAL;
    if (slices < 1 || slices > OZ_MAX_S || beta < 1 || kblk < OZ_KPAD || kblk % OZ_KPAD) return MPX_EINVAL;
    // Exactness of the level sums: |m_1| <= 2^beta and |m_p| <= 2^(beta-1)
    // for p >= 2, so a level g <= s+1 sums at most
    // 2^(2 beta) (1 + max(0, s-2)/4) per k; over kblk terms this must stay
    // <= 2^53 (every partial sum is then an exactly representable integer).
    if (!oz_exact(slices, beta, kblk)) return MPX_EINVAL;
    if (m > 0 && k > 0 && (A == nullptr || !span_fits(m, k, lda, psA))) return MPX_EINVAL;
    if (k > 0 && n > 0 && (B == nullptr || !span_fits(k, n, ldb, psB))) return MPX_EINVAL;
    if (m > 0 && n > 0 && (C == nullptr || !span_fits(m, n, ldc, psC))) return MPX_EINVAL;
    // C must not overlap A or B, nor the workspace any of them
    const uint64_t cb = planes_bytes(2, m, n, ldc, psC, sizeof(double));
    const uint64_t ab = planes_bytes(2, m, k, lda, psA, sizeof(double));
    const uint64_t bb = planes_bytes(2, k, n, ldb, psB, sizeof(double));
    if (overlaps(C, cb, A, ab) || overlaps(C, cb, B, bb)) return MPX_EINVAL;
    if (m == 0 || n == 0) return MPX_OK;
    if (m > INT32_MAX / 2 || n > INT32_MAX / 2) return MPX_ENOTSUP;
    const size_t need = ozaki_workspace(m, n, k, slices);
    if (ws == nullptr || ws_bytes < need) return MPX_EWORKSPACE;
    if (overlaps(ws, need, A, ab) || overlaps(ws, need, B, bb) || overlaps(ws, need, C, cb))
        return MPX_EINVAL;
    hipStream_t s = as_stream(stream);
#define MPX_OZ(SS)                                                                     \
    case SS:                                                                           \
        return oz_run<SS>(m, n, k, A, lda, psA, B, ldb, psB, C, ldc, psC, beta, kblk,  \
                          ws, s);
    switch (slices) {
        MPX_OZ(1) MPX_OZ(2) MPX_OZ(3) MPX_OZ(4) MPX_OZ(5) MPX_OZ(6)
        MPX_OZ(7) MPX_OZ(8) MPX_OZ(9) MPX_OZ(10) MPX_OZ(11) MPX_OZ(12)
        default: return MPX_EINVAL;
    }
#undef MPX_OZ
}

// Select the stage depth of the slice GEMM for subsequent calls (0: 8, 1: 16
// k per LDS stage).  Results do not depend on it.
extern "C" int mpx_gemm_ozaki_set_variant(int variant) {
    if (variant < 0 || variant > 1) return MPX_EINVAL;
    g_oz_variant.store(variant, std::memory_order_relaxed);
    return MPX_OK;
}
