// mpx_gemm.hip -- C := op(A) op(B) in DD / TD / QD / FF on gfx950.
//
// The product of Section 3.1 (benchmarked there with the branch-free TD and
// QD operations) is the dominant kernel.  Its multiply-add is 29 / 96 / 209
// FP64 VALU instructions (DD / TD / QD, Tables 1-2 plus the DW algorithms)
// against 2K operand doubles, so it is bound by FP64 VALU issue, not by
// memory, and the MFMA units cannot help (the BF operations are not dot
// products).  The design therefore maximises VALU issue:
//
//  * a 256-thread workgroup (four wave64s) owns a BM x BN tile of C, each
//    thread a TM x TN register micro-tile of K-component accumulators; the
//    independent accumulators give the scheduler TM*TN interleavable MAC
//    chains per thread;
//  * per k-panel of depth BK the workgroup stages the K component planes of
//    the A and B panels in LDS (sA[c][kk][row], sB[c][kk][col], the rows of
//    sB padded by one element when B is transposed); a thread
//    reads its rows ty + 16 i (wave-uniform broadcasts) and columns
//    tx + 16 j (16 consecutive doubles per wave: conflict-free);
//  * the next panel is fetched from global memory into registers while the
//    current one is consumed (one-deep software pipeline);
//  * every C_ij is accumulated in ascending l from zero, exactly the naive
//    triple loop's sequence, so results are bit-identical for every tiling.
//
// The template argument AR selects the branch-free operations (0) or the
// conventional ones the paper compares them with (1: sloppy DD addition,
// 2: accurate DD addition; TD / QD with renormalisation).
//
// Workgroups are numbered so that each of the eight XCDs (which receive
// workgroups round-robin) works on compact blocks of tiles whose A and B
// panels stay in its L2.
//
// For small products a second kernel, k_gemm_rw, gives each wave whole rows
// of C (A through scalar loads, B straight from global memory, no LDS and no
// barriers); it is described where it is defined.
#include "mp_arith.hpp"
#include "mp_conv.hpp"
#include "mpx_internal.hpp"

#include <algorithm>
#include <string>
#include <cstdlib>
#include <cstdio>
#include <mutex>
#include <new>
#include <map>
#include <memory>
#include <tuple>
#include <vector>

namespace mpx {

constexpr int kGemmThreads = 256;
// With B transposed, a thread stashes consecutive k of one column of B, so
// a wave's LDS stores stride by a whole panel row and land on one bank pair;
// one element of padding per row of sB spreads them over all banks (DD with
// B transposed at 2048: 9 % faster).  Padding sA likewise for the
// untransposed A, whose stash has the same pattern, measured slower on
// balance (QD 2048 -1.8 %, DD 512 -7.8 %), so sA is not padded.
template <bool TB>
constexpr int lds_pad_b() { return TB ? 1 : 0; }

// One BM x BN tile of C = op(A) op(B) at (m0, n0), computed by the 256
// threads of a workgroup with the LDS panels sA, sB (shared by k_gemm and the
// batched kernel, so both give the same bits).
template <typename T, int K, int TM, int TN, int BK, bool TA, bool TB, int AR, bool PF = false>
__device__ __forceinline__ void gemm_tile(int m, int n, int k, const T* __restrict__ A,
                                          long long lda, long long psA, const T* __restrict__ B,
                                          long long ldb, long long psB, T* __restrict__ C,
                                          long long ldc, long long psC, int m0, int n0,
                                          T (&sA)[K][BK][16 * TM],
                                          T (&sB)[K][BK][16 * TN + lds_pad_b<TB>()]) {
    constexpr int BM = 16 * TM, BN = 16 * TN;
    constexpr int A_PER = (BM * BK + kGemmThreads - 1) / kGemmThreads;
    constexpr int B_PER = (BN * BK + kGemmThreads - 1) / kGemmThreads;
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;

    mpn<T, K> acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = mp_zero<T, K>();

    T ra[A_PER][K], rb[B_PER][K];

    // Fetch the panel starting at k0 into registers (zero outside the matrix).
    auto fetch = [&](int k0) {
#pragma unroll
        for (int t = 0; t < A_PER; ++t) {
            const int e = tid + t * kGemmThreads;
            int r, kk;
            if (TA) { kk = e / BM; r = e % BM; } else { r = e / BK; kk = e % BK; }
            const int gr = m0 + r, gk = k0 + kk;
            const bool ok = e < BM * BK && gr < m && gk < k;
            const long long idx = TA ? (long long)gk * lda + gr : (long long)gr * lda + gk;
#pragma unroll
            for (int c = 0; c < K; ++c) ra[t][c] = ok ? A[c * psA + idx] : T(0);
        }
#pragma unroll
        for (int t = 0; t < B_PER; ++t) {
            const int e = tid + t * kGemmThreads;
            int cc, kk;
            if (TB) { cc = e / BK; kk = e % BK; } else { kk = e / BN; cc = e % BN; }
            const int gc = n0 + cc, gk = k0 + kk;
            const bool ok = e < BN * BK && gc < n && gk < k;
            const long long idx = TB ? (long long)gc * ldb + gk : (long long)gk * ldb + gc;
#pragma unroll
            for (int c = 0; c < K; ++c) rb[t][c] = ok ? B[c * psB + idx] : T(0);
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int t = 0; t < A_PER; ++t) {
            const int e = tid + t * kGemmThreads;
            if (e < BM * BK) {
                int r, kk;
                if (TA) { kk = e / BM; r = e % BM; } else { r = e / BK; kk = e % BK; }
#pragma unroll
                for (int c = 0; c < K; ++c) sA[c][kk][r] = ra[t][c];
            }
        }
#pragma unroll
        for (int t = 0; t < B_PER; ++t) {
            const int e = tid + t * kGemmThreads;
            if (e < BN * BK) {
                int cc, kk;
                if (TB) { cc = e / BK; kk = e % BK; } else { kk = e / BN; cc = e % BN; }
#pragma unroll
                for (int c = 0; c < K; ++c) sB[c][kk][cc] = rb[t][c];
            }
        }
    };
    auto load_ab = [&](int kk, mpn<T, K> (&a)[TM], mpn<T, K> (&b)[TN]) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int c = 0; c < K; ++c) a[i].c[c] = sA[c][kk][ty + 16 * i];
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int c = 0; c < K; ++c) b[j].c[c] = sB[c][kk][tx + 16 * j];
    };
    auto mac_ab = [&](const mpn<T, K> (&a)[TM], const mpn<T, K> (&b)[TN]) {
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) acc[i][j] = ar_add<AR>(acc[i][j], ar_mul<AR>(a[i], b[j]));
    };
    auto mac_step = [&](int kk) {
        mpn<T, K> a[TM], b[TN];
        load_ab(kk, a, b);
        mac_ab(a, b);
    };
    // PF: a full panel with the LDS operands of step kk + 1 read before the
    // arithmetic of step kk (the scheduling barrier keeps them there), so the
    // LDS latency overlaps a whole multiply-add; for short multiply-adds on
    // small tiles.  Same operations in the same order.
    auto panel_pf = [&]() {
        mpn<T, K> a[TM], b[TN];
        load_ab(0, a, b);
#pragma unroll
        for (int kk = 0; kk < BK; ++kk) {
            mpn<T, K> an[TM], bn[TN];
            if (kk + 1 < BK) load_ab(kk + 1, an, bn);
            __builtin_amdgcn_sched_barrier(0);
            mac_ab(a, b);
            if (kk + 1 < BK) {
#pragma unroll
                for (int i = 0; i < TM; ++i) a[i] = an[i];
#pragma unroll
                for (int j = 0; j < TN; ++j) b[j] = bn[j];
            }
        }
    };

    if (k > 0) fetch(0);
    for (int k0 = 0; k0 < k; k0 += BK) {
        __syncthreads();  // previous panel fully consumed
        stash();
        __syncthreads();
        if (k0 + BK < k) fetch(k0 + BK);  // overlaps the MACs below
        const int kend = k - k0;
        if (kend >= BK) {
            if constexpr (PF) {
                panel_pf();
            } else {
#pragma unroll
                for (int kk = 0; kk < BK; ++kk) mac_step(kk);
            }
        } else {
            for (int kk = 0; kk < kend; ++kk) mac_step(kk);
        }
    }

#pragma unroll
    for (int i = 0; i < TM; ++i) {
        const int r = m0 + ty + 16 * i;
        if (r >= m) continue;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int cidx = n0 + tx + 16 * j;
            if (cidx < n) mp_store<T, K>(C, psC, (long long)r * ldc + cidx, acc[i][j]);
        }
    }
}


template <typename T, int K, int TM, int TN, int BK, bool TA, bool TB, int AR, bool PF = false>
__global__ void __launch_bounds__(kGemmThreads)
k_gemm(int m, int n, int k, const T* __restrict__ A, long long lda, long long psA,
       const T* __restrict__ B, long long ldb, long long psB, T* __restrict__ C,
       long long ldc, long long psC, int tiles_n, int tiles_total) {
    constexpr int BM = 16 * TM, BN = 16 * TN;
    __shared__ T sA[K][BK][BM];
    __shared__ T sB[K][BK][BN + lds_pad_b<TB>()];

    // XCD-aware tile order: workgroup w runs on XCD w % 8; each XCD gets a
    // contiguous range of virtual tile ids, and virtual ids walk the tile grid
    // in groups of 8 tile rows (column-major inside a group), so the
    // workgroups resident on one XCD at a time cover a square block of C and
    // share its A and B panels in that XCD's L2.
    const int w = blockIdx.x;
    const int per_xcd = (tiles_total + 7) / 8;
    const int xcd = w % 8, slot = w / 8;
    int v = xcd * per_xcd + slot;
    if (per_xcd * 8 != tiles_total) v = w;  // uneven split: plain order
    constexpr int GROUP = 8;
    const int tiles_m = tiles_total / tiles_n;
    const int in_group = GROUP * tiles_n;
    const int first_m = (v / in_group) * GROUP;
    const int rows_here = tiles_m - first_m < GROUP ? tiles_m - first_m : GROUP;
    const int r = v % in_group;
    const int m0 = (first_m + r % rows_here) * BM;
    const int n0 = (r / rows_here) * BN;

    gemm_tile<T, K, TM, TN, BK, TA, TB, AR, PF>(m, n, k, A, lda, psA, B, ldb, psB, C, ldc, psC, m0,
                                                n0, sA, sB);
}

// Raw buffer loads: word 3 of a gfx9 buffer resource with a 32-bit data
// format and no swizzle; the range is left unlimited (the launcher bounds
// every offset).
constexpr int kBufWord3 = 0x00020000;
template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, unsigned voff, int soff) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, soff, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, soff, 0));
}

// Row-wave tiling, for products too small to give every SIMD several waves of
// the LDS-tiled kernel: each wave64 owns R rows x 64 columns of C, one column
// per lane, so at every step all lanes of a wave multiply by the same A
// entries.  Those are read with scalar loads into scalar registers (one copy
// per wave, no LDS traffic), and each lane loads its own B entry from global
// memory at a wave-uniform base plus a 32-bit per-lane byte offset (64
// consecutive doubles per component when B is not transposed; the four waves
// of a workgroup read the same B columns, which the vector L1 cache shares).
// With no LDS there are no barriers: every wave runs its R multiply-add chains
// on its own.  Panels of BK steps alternate between two register buffers;
// the next panel's loads are issued after the first step of the current one
// (so the wait for the current panel's scalar loads, which return out of
// order and are waited for all at once, comes before them) and overlap the
// remaining steps.  Each C_ij is still accumulated in ascending l from zero
// with the same operation, so the bits equal those of every other tiling.
// The launcher checks that B's byte offsets from a panel's first row (or
// column) fit in 31 bits, and runs an LDS tiling where they would not.
template <typename T, int K, int R, int BK, bool TA, bool TB, int AR>
__global__ void __launch_bounds__(kGemmThreads)
k_gemm_rw(int m, int n, int k, const T* __restrict__ A, long long lda, long long psA,
          const T* __restrict__ B, long long ldb, long long psB, T* __restrict__ C,
          long long ldc, long long psC, int groups_n) {
    constexpr int WAVES = kGemmThreads / 64;
    const int lane = threadIdx.x & 63;
    // workgroup = WAVES consecutive row blocks of one 64-column group; the
    // wave index is made explicitly uniform so the A addresses are scalar
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int cg = blockIdx.x % groups_n;
    const int r0 = ((blockIdx.x / groups_n) * WAVES + w) * R;
    if (r0 >= m) return;
    const int j = cg * 64 + lane;
    const int jl = j < n ? j : n - 1;  // loads stay inside B; results of j >= n are dropped
    const unsigned boff = (unsigned)((TB ? (long long)jl * ldb : (long long)jl) * (long long)sizeof(T));
    int rows[R];
#pragma unroll
    for (int i = 0; i < R; ++i) rows[i] = r0 + i < m ? r0 + i : m - 1;

    mpn<T, K> acc[R];
#pragma unroll
    for (int i = 0; i < R; ++i) acc[i] = mp_zero<T, K>();

    auto a_at = [&](int i, int l, int c) -> T {
        return A[c * psA + (TA ? (long long)l * lda + rows[i] : (long long)rows[i] * lda + l)];
    };
    // B entries (l .. l + BK - 1, column j) of component c: a buffer resource
    // at the wave-uniform address of entry (l, column 0), the lane's byte
    // offset, and a uniform byte offset per step
    const int bstep = (int)((TB ? 1LL : ldb) * (long long)sizeof(T));
    auto b_rsrc = [&](int l, int c) {
        const T* base = B + c * psB + (TB ? (long long)l : (long long)l * ldb);
        return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, -1, kBufWord3);
    };
    auto b_at = [&](int l, int c) -> T { return buf_load<T>(b_rsrc(l, c), boff, 0); };
    using PanelA = T[R][BK][K];
    using PanelB = T[BK][K];
    auto load = [&](int k0, PanelA& a, PanelB& b) {
#pragma unroll
        for (int c = 0; c < K; ++c) {
            const auto rs = b_rsrc(k0, c);
#pragma unroll
            for (int kk = 0; kk < BK; ++kk) b[kk][c] = buf_load<T>(rs, boff, kk * bstep);
        }
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int kk = 0; kk < BK; ++kk)
#pragma unroll
                for (int c = 0; c < K; ++c) a[i][kk][c] = a_at(i, k0 + kk, c);
    };
    auto step = [&](const PanelA& a, const PanelB& b, int kk) {
        mpn<T, K> bv;
#pragma unroll
        for (int c = 0; c < K; ++c) bv.c[c] = b[kk][c];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            mpn<T, K> av;
#pragma unroll
            for (int c = 0; c < K; ++c) av.c[c] = a[i][kk][c];
            acc[i] = ar_add<AR>(acc[i], ar_mul<AR>(av, bv));
        }
    };
    auto consume = [&](const PanelA& a, const PanelB& b) {
#pragma unroll
        for (int kk = 0; kk < BK; ++kk) step(a, b, kk);
    };
    // consume (a, b) while loading the panel at k0 into (na, nb)
    auto consume_next = [&](const PanelA& a, const PanelB& b, int k0, PanelA& na, PanelB& nb) {
        step(a, b, 0);
        __builtin_amdgcn_sched_barrier(0);
        load(k0, na, nb);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int kk = 1; kk < BK; ++kk) step(a, b, kk);
    };

    const int npan = k / BK;
    if (npan > 0) {
        T ax[R][BK][K], bx[BK][K], ay[R][BK][K], by[BK][K];
        load(0, ax, bx);
        int p = 0;
        for (; p + 2 <= npan; p += 2) {  // panel p is in x
            consume_next(ax, bx, (p + 1) * BK, ay, by);
            if (p + 2 < npan) consume_next(ay, by, (p + 2) * BK, ax, bx);
            else consume(ay, by);
        }
        if (p < npan) consume(ax, bx);
    }
    for (int l = npan * BK; l < k; ++l) {
        T a1[R][1][K], b1[1][K];
#pragma unroll
        for (int c = 0; c < K; ++c) b1[0][c] = b_at(l, c);
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int c = 0; c < K; ++c) a1[i][0][c] = a_at(i, l, c);
        mpn<T, K> bv;
#pragma unroll
        for (int c = 0; c < K; ++c) bv.c[c] = b1[0][c];
#pragma unroll
        for (int i = 0; i < R; ++i) {
            mpn<T, K> av;
#pragma unroll
            for (int c = 0; c < K; ++c) av.c[c] = a1[i][0][c];
            acc[i] = ar_add<AR>(acc[i], ar_mul<AR>(av, bv));
        }
    }

    if (j < n) {
#pragma unroll
        for (int i = 0; i < R; ++i)
            if (r0 + i < m) mp_store<T, K>(C, psC, (long long)(r0 + i) * ldc + j, acc[i]);
    }
}

// ----------------------------------------------------------- variants ----

struct GemmArgs {
    int m, n, k, tA, tB;
    const void* A; long long lda, psA;
    const void* B; long long ldb, psB;
    void* C; long long ldc, psC;
};

template <typename T, int K, int TM, int TN, int BK, int AR, bool PF = false>
static int run_variant(const GemmArgs& g, hipStream_t s) {
    constexpr int BM = 16 * TM, BN = 16 * TN;
    const long long tiles = ceil_div(g.n, BN) * ceil_div(g.m, BM);
    if (tiles > INT32_MAX / 2) return MPX_ENOTSUP;  // one workgroup per tile (int grid)
    const int tn = (int)ceil_div(g.n, BN);
    const int total = (int)tiles;
    if (total == 0) return MPX_OK;
#define MPX_GEMM_LAUNCH(TA_, TB_)                                                           \
    k_gemm<T, K, TM, TN, BK, TA_, TB_, AR, PF><<<total, kGemmThreads, 0, s>>>(              \
        g.m, g.n, g.k, (const T*)g.A, g.lda, g.psA, (const T*)g.B, g.ldb, g.psB, (T*)g.C,   \
        g.ldc, g.psC, tn, total)
    if (!g.tA && !g.tB) MPX_GEMM_LAUNCH(false, false);
    else if (g.tA && !g.tB) MPX_GEMM_LAUNCH(true, false);
    else if (!g.tA && g.tB) MPX_GEMM_LAUNCH(false, true);
    else MPX_GEMM_LAUNCH(true, true);
#undef MPX_GEMM_LAUNCH
    return launch_status();
}

// The row-wave kernel addresses B with 32-bit byte offsets from a panel's
// first row (or column); where they would not fit, the LDS-tiled 16 x 16 tiling runs instead (same
// operations in the same order, so the same bits).
template <typename T, int K, int R, int BK, int AR>
static int run_variant_rw(const GemmArgs& g, hipStream_t s) {
    constexpr int WAVES = kGemmThreads / 64;
    // lane offset + step offset, in bytes, of the farthest B entry of a panel
    const long long lane_off = g.n <= 0 ? 0 : (g.tB ? (long long)(g.n - 1) * g.ldb : (long long)(g.n - 1));
    const long long step_off = (long long)(BK - 1) * (g.tB ? 1LL : g.ldb);
    if ((lane_off + step_off + 1) * (long long)sizeof(T) > (long long)INT32_MAX)
        return run_variant<T, K, 1, 1, 16, AR, true>(g, s);
    const long long groups_n = ceil_div(g.n, 64);
    const long long wgs = groups_n * ceil_div(g.m, (long long)WAVES * R);
    if (wgs > INT32_MAX / 2) return MPX_ENOTSUP;
    if (wgs == 0) return MPX_OK;
#define MPX_GEMM_LAUNCH(TA_, TB_)                                                              \
    k_gemm_rw<T, K, R, BK, TA_, TB_, AR><<<(int)wgs, kGemmThreads, 0, s>>>(                    \
        g.m, g.n, g.k, (const T*)g.A, g.lda, g.psA, (const T*)g.B, g.ldb, g.psB, (T*)g.C,      \
        g.ldc, g.psC, (int)groups_n)
    if (!g.tA && !g.tB) MPX_GEMM_LAUNCH(false, false);
    else if (g.tA && !g.tB) MPX_GEMM_LAUNCH(true, false);
    else if (!g.tA && g.tB) MPX_GEMM_LAUNCH(false, true);
    else MPX_GEMM_LAUNCH(true, true);
#undef MPX_GEMM_LAUNCH
    return launch_status();
}

using VariantFn = int (*)(const GemmArgs&, hipStream_t);

struct Variant {
    VariantFn fn;
    int bm, bn;
    const char* name;
    bool small_only = false;  // autotuned only for small products
};

// The row-wave tilings re-read a whole B column strip for every 4R rows of C
// (at 2048^3 in QD that is about 70 GB of L2 reads and 10.9 GB of HBM traffic
// per launch, against 16 GB and 3.4 GB for the 32 x 32 LDS tiling), and they
// run no faster there.  They pay off where the LDS tilings leave the SIMDs
// with few waves, so the autotuner tries them only for products with fewer
// than 4096 tiles of 32 x 32 (16 per CU).
static bool small_product(const GemmArgs& g) { return ceil_div(g.m, 32) * ceil_div(g.n, 32) < 4096; }

// Candidate tilings per precision and arithmetic (row-wave panel depths: the
// deepest whose double-buffered A panels fit the scalar registers without
// spill code inside the loop, or a shallower one where that measured faster;
// DD with two rows and 4-deep panels keeps a few spills in its prologue).
// The conventional lists
// (AR = 1, 2) hold exactly the branch-free ones, so the comparison of the two
// arithmetics gives each its best tiling from the same set.
#define MPX_TILES_DD(AR_, P_)                                                            \
    {run_variant<double, 2, 4, 4, 8, AR_>, 64, 64, P_ "_4x4_k8"},                        \
    {run_variant<double, 2, 2, 4, 16, AR_, true>, 32, 64, P_ "_2x4_k16_pf"},             \
    {run_variant<double, 2, 2, 4, 8, AR_>, 32, 64, P_ "_2x4_k8"},                        \
    {run_variant<double, 2, 2, 2, 16, AR_>, 32, 32, P_ "_2x2_k16"},                      \
    {run_variant<double, 2, 1, 2, 16, AR_>, 16, 32, P_ "_1x2_k16"},                      \
    {run_variant<double, 2, 1, 1, 16, AR_>, 16, 16, P_ "_1x1_k16"},                      \
    {run_variant<double, 2, 1, 2, 16, AR_, true>, 16, 32, P_ "_1x2_k16_pf"},             \
    {run_variant<double, 2, 1, 1, 16, AR_, true>, 16, 16, P_ "_1x1_k16_pf"},             \
    {run_variant<double, 2, 2, 2, 16, AR_, true>, 32, 32, P_ "_2x2_k16_pf"},             \
    {run_variant<double, 2, 2, 4, 8, AR_, true>, 32, 64, P_ "_2x4_k8_pf"},               \
    {run_variant<double, 2, 2, 2, 32, AR_, true>, 32, 32, P_ "_2x2_k32_pf"},             \
    {run_variant<double, 2, 1, 2, 32, AR_, true>, 16, 32, P_ "_1x2_k32_pf"},             \
    {run_variant_rw<double, 2, 1, 4, AR_>, 4, 64, P_ "_rw1_k4", true},                   \
    {run_variant_rw<double, 2, 2, 2, AR_>, 8, 64, P_ "_rw2_k2", true},                  \
    {run_variant_rw<double, 2, 2, 4, AR_>, 8, 64, P_ "_rw2_k4", true}
#define MPX_TILES_TD(AR_, P_)                                                            \
    {run_variant<double, 3, 2, 4, 8, AR_>, 32, 64, P_ "_2x4_k8"},                        \
    {run_variant<double, 3, 2, 2, 8, AR_>, 32, 32, P_ "_2x2_k8"},                        \
    {run_variant<double, 3, 1, 2, 16, AR_>, 16, 32, P_ "_1x2_k16"},                      \
    {run_variant<double, 3, 1, 1, 16, AR_>, 16, 16, P_ "_1x1_k16"},                      \
    {run_variant<double, 3, 1, 1, 16, AR_, true>, 16, 16, P_ "_1x1_k16_pf"},             \
    {run_variant<double, 3, 1, 2, 16, AR_, true>, 16, 32, P_ "_1x2_k16_pf"},             \
    {run_variant<double, 3, 2, 2, 8, AR_, true>, 32, 32, P_ "_2x2_k8_pf"},               \
    {run_variant_rw<double, 3, 1, 4, AR_>, 4, 64, P_ "_rw1_k4", true},                   \
    {run_variant_rw<double, 3, 2, 2, AR_>, 8, 64, P_ "_rw2_k2", true}
#define MPX_TILES_QD(AR_, P_)                                                            \
    {run_variant<double, 4, 2, 2, 8, AR_>, 32, 32, P_ "_2x2_k8"},                        \
    {run_variant<double, 4, 1, 2, 16, AR_>, 16, 32, P_ "_1x2_k16"},                      \
    {run_variant<double, 4, 1, 1, 16, AR_>, 16, 16, P_ "_1x1_k16"},                      \
    {run_variant<double, 4, 1, 1, 16, AR_, true>, 16, 16, P_ "_1x1_k16_pf"},             \
    {run_variant<double, 4, 1, 2, 16, AR_, true>, 16, 32, P_ "_1x2_k16_pf"},             \
    {run_variant<double, 4, 2, 2, 8, AR_, true>, 32, 32, P_ "_2x2_k8_pf"},               \
    {run_variant_rw<double, 4, 1, 2, AR_>, 4, 64, P_ "_rw1_k2", true}

static const std::vector<Variant>& variants(int prec) {
    // DD also offers 16 x 32 and 16 x 16 tiles: at n = 512 the 32 x 32 tile
    // leaves one workgroup per CU
    // (the 2 x 4 tile with a 16-deep prefetched panel comes before the other
    // 32 x 64 tilings: the size heuristic takes the first of equal areas, and
    // it is the fastest DD tiling at 2048).  The row-wave tilings ("rw", a
    // workgroup of 4R x 64) come last, so the untuned heuristic keeps the LDS
    // tilings; the autotuner tries them for small products (small_product)
    // and picks them where they win (n = 512 and 1024).
    static const std::vector<Variant> dd = {MPX_TILES_DD(AR_BF, "dd")};
    static const std::vector<Variant> td = {MPX_TILES_TD(AR_BF, "td")};
    static const std::vector<Variant> qd = {MPX_TILES_QD(AR_BF, "qd")};
    static const std::vector<Variant> ff = {
        {run_variant<float, 2, 4, 8, 8, AR_BF>, 64, 128, "ff_4x8_k8"},
        {run_variant<float, 2, 4, 4, 8, AR_BF>, 64, 64, "ff_4x4_k8"},
        {run_variant<float, 2, 2, 4, 8, AR_BF>, 32, 64, "ff_2x4_k8"},
        {run_variant<float, 2, 2, 2, 16, AR_BF>, 32, 32, "ff_2x2_k16"},
        {run_variant<float, 2, 4, 4, 8, AR_BF, true>, 64, 64, "ff_4x4_k8_pf"},
        {run_variant<float, 2, 2, 4, 8, AR_BF, true>, 32, 64, "ff_2x4_k8_pf"},
        {run_variant<float, 2, 2, 2, 16, AR_BF, true>, 32, 32, "ff_2x2_k16_pf"},
        {run_variant<float, 2, 1, 1, 16, AR_BF, true>, 16, 16, "ff_1x1_k16_pf"},
        {run_variant_rw<float, 2, 1, 8, AR_BF>, 4, 64, "ff_rw1_k8", true},
        {run_variant_rw<float, 2, 2, 4, AR_BF>, 8, 64, "ff_rw2_k4", true},
    };
    static const std::vector<Variant> dd_nobf = {MPX_TILES_DD(AR_NOBF, "dd_nobf")};
    static const std::vector<Variant> td_nobf = {MPX_TILES_TD(AR_NOBF, "td_nobf")};
    static const std::vector<Variant> qd_nobf = {MPX_TILES_QD(AR_NOBF, "qd_nobf")};
    static const std::vector<Variant> dd_acc = {MPX_TILES_DD(AR_NOBF_ACC, "dd_nobf_acc")};
    static const std::vector<Variant> none;
    switch (prec) {
        case MPX_DD: return dd;
        case MPX_TD: return td;
        case MPX_QD: return qd;
        case MPX_FF: return ff;
        case MPX_DD | MPX_NOBF: return dd_nobf;
        case MPX_TD | MPX_NOBF: return td_nobf;
        case MPX_QD | MPX_NOBF: return qd_nobf;
        case MPX_DD | MPX_NOBF_ACC: return dd_acc;
        default: return none;
    }
}
#undef MPX_TILES_DD
#undef MPX_TILES_TD
#undef MPX_TILES_QD

// Tuned choices, keyed by (prec, tA, tB, log2 buckets of m, n, k), live in
// the tune cache as "gemm <prec> <tA> <tB> <bm> <bn> <bk>" -> tiling name.
static int ilog2_bucket(long long v) {
    int b = 0;
    while ((1LL << (b + 1)) <= v) ++b;
    return b;
}
static std::string tune_key(int prec, const GemmArgs& g) {
    char buf[96];
    std::snprintf(buf, sizeof buf, "gemm %d %d %d %d %d %d", prec, g.tA, g.tB, ilog2_bucket(g.m),
                  ilog2_bucket(g.n), ilog2_bucket(g.k));
    return buf;
}

static int variant_by_name(int prec, const std::string& name) {
    const auto& v = variants(prec);
    for (size_t i = 0; i < v.size(); ++i)
        if (name == v[i].name) return (int)i;
    return -1;
}

// Untuned default: the largest tile that still yields at least 2048
// workgroups (8 per CU), else the smallest tile; among equal tiles the first
// listed.
static int default_variant(int prec, const GemmArgs& g) {
    const auto& v = variants(prec);
    int best = -1, smallest = 0;
    for (size_t i = 0; i < v.size(); ++i) {
        const long long area = (long long)v[i].bm * v[i].bn;
        const long long wg = ceil_div(g.m, v[i].bm) * ceil_div(g.n, v[i].bn);
        if (wg >= 2048 && (best < 0 || area > (long long)v[best].bm * v[best].bn)) best = (int)i;
        if (area < (long long)v[smallest].bm * v[smallest].bn) smallest = (int)i;
    }
    return best >= 0 ? best : smallest;
}

// A tiling forced by MPX_GEMM_VARIANT (comma-separated names), else the tuned
// choice for this bucket, else the size heuristic.
static int pick_variant(int prec, const GemmArgs& g) {
    if (const char* f = std::getenv("MPX_GEMM_VARIANT")) {
        std::string names(f);
        size_t pos = 0;
        while (pos <= names.size()) {
            const size_t end = std::min(names.find(',', pos), names.size());
            const int v = variant_by_name(prec, names.substr(pos, end - pos));
            if (v >= 0) return v;
            pos = end + 1;
        }
    }
    std::string choice;
    if (tune_lookup(tune_key(prec, g), choice)) {
        const int v = variant_by_name(prec, choice);
        if (v >= 0) return v;
    }
    return default_variant(prec, g);
}

static int check_gemm(int prec, int tA, int tB, int64_t m, int64_t n, int64_t k, const void* A,
                      int64_t lda, int64_t psA, const void* B, int64_t ldb, int64_t psB,
                      const void* C, int64_t ldc, int64_t psC) {
    if (!prec_k_ar(prec)) return MPX_EPREC;
    if (m < 0 || n < 0 || k < 0 || (tA != 0 && tA != 1) || (tB != 0 && tB != 1))
        return MPX_EINVAL;
    if (m > INT32_MAX / 2 || n > INT32_MAX / 2 || k > INT32_MAX / 2) return MPX_ENOTSUP;
    const int64_t ar = tA ? k : m, ac = tA ? m : k;  // stored shape of A
    const int64_t br = tB ? n : k, bc = tB ? k : n;  // stored shape of B
    if (ar > 0 && ac > 0 && (A == nullptr || !span_fits(ar, ac, lda, psA))) return MPX_EINVAL;
    if (br > 0 && bc > 0 && (B == nullptr || !span_fits(br, bc, ldb, psB))) return MPX_EINVAL;
    if (m > 0 && n > 0 && (C == nullptr || !span_fits(m, n, ldc, psC))) return MPX_EINVAL;
    // C must not overlap A or B (the kernels read them while C is written)
    const int K = prec_k_ar(prec);
    const size_t elt = is_ff(prec) ? sizeof(float) : sizeof(double);
    const uint64_t bc_ = planes_bytes(K, m, n, ldc, psC, elt);
    if (overlaps(C, bc_, A, planes_bytes(K, ar, ac, lda, psA, elt)) ||
        overlaps(C, bc_, B, planes_bytes(K, br, bc, ldb, psB, elt)))
        return MPX_EINVAL;
    return MPX_OK;
}

}  // namespace mpx

using namespace mpx;

extern "C" int mpx_gemm(int prec, int transA, int transB, int64_t m, int64_t n, int64_t k,
                        const void* A, int64_t lda, int64_t psA, const void* B, int64_t ldb,
                        int64_t psB, void* C, int64_t ldc, int64_t psC, void* stream) {
    int st = check_gemm(prec, transA, transB, m, n, k, A, lda, psA, B, ldb, psB, C, ldc, psC);
    if (st) return st;
    if (m == 0 || n == 0) return MPX_OK;
    GemmArgs g{(int)m, (int)n, (int)k, transA, transB, A, lda, psA, B, ldb, psB, C, ldc, psC};
    return variants(prec)[pick_variant(prec, g)].fn(g, as_stream(stream));
}

// The tiling mpx_gemm would use for this shape (forced, tuned or default).
extern "C" int mpx_gemm_selected_variant(int prec, int transA, int transB, int64_t m, int64_t n,
                                         int64_t k) {
    if (!prec_k_ar(prec)) return MPX_EPREC;
    if (m < 1 || n < 1 || k < 0 || m > INT32_MAX / 2 || n > INT32_MAX / 2 || k > INT32_MAX / 2 ||
        (transA != 0 && transA != 1) || (transB != 0 && transB != 1))
        return MPX_EINVAL;
    GemmArgs g{(int)m, (int)n, (int)k, transA, transB, nullptr, 0, 0, nullptr, 0, 0, nullptr, 0, 0};
    return pick_variant(prec, g);
}

// Number of kernel variants available for a precision, and their names.
extern "C" int mpx_gemm_variant_count(int prec) { return (int)variants(prec).size(); }

extern "C" const char* mpx_gemm_variant_name(int prec, int v) {
    const auto& vs = variants(prec);
    return (v >= 0 && v < (int)vs.size()) ? vs[v].name : nullptr;
}

// Run one specific variant (used by the autotuner and by tests that check
// that every tiling produces identical bits).
extern "C" int mpx_gemm_variant(int prec, int variant, int transA, int transB, int64_t m,
                                int64_t n, int64_t k, const void* A, int64_t lda, int64_t psA,
                                const void* B, int64_t ldb, int64_t psB, void* C, int64_t ldc,
                                int64_t psC, void* stream) {
    int st = check_gemm(prec, transA, transB, m, n, k, A, lda, psA, B, ldb, psB, C, ldc, psC);
    if (st) return st;
    if (variant < 0 || variant >= (int)variants(prec).size()) return MPX_EINVAL;
    if (m == 0 || n == 0) return MPX_OK;
    GemmArgs g{(int)m, (int)n, (int)k, transA, transB, A, lda, psA, B, ldb, psB, C, ldc, psC};
    return variants(prec)[variant].fn(g, as_stream(stream));
}

// Autotuner: time every variant `reps` times on the caller's buffers (C is
// overwritten) with HIP events on `stream`, in two rounds over all variants,
// each variant's time being its faster round (the engine clock may still be
// ramping up during the first round, which would favour the variants timed
// last); remember the fastest for this (precision, transposes, size bucket)
// and return its index.  Synchronises the stream; not capture-safe.
extern "C" int mpx_gemm_autotune(int prec, int transA, int transB, int64_t m, int64_t n,
                                 int64_t k, const void* A, int64_t lda, int64_t psA,
                                 const void* B, int64_t ldb, int64_t psB, void* C, int64_t ldc,
                                 int64_t psC, int reps, float* best_ms, void* stream) {
    int st = check_gemm(prec, transA, transB, m, n, k, A, lda, psA, B, ldb, psB, C, ldc, psC);
    if (st) return st;
    if (m == 0 || n == 0 || reps < 1) return MPX_EINVAL;
    GemmArgs g{(int)m, (int)n, (int)k, transA, transB, A, lda, psA, B, ldb, psB, C, ldc, psC};
    hipStream_t s = as_stream(stream);
    EventPair ev;
    if (!ev.ok) return MPX_EDEVICE;
    const auto& vs = variants(prec);
    const int v0 = default_variant(prec, g);
    st = warm_clock(ev, s, [&] { return vs[v0].fn(g, s); });
    int best = -1;
    float best_t = 0.f;
    const bool small = small_product(g);
    std::vector<float> t(vs.size(), -1.f);  // each tiling's faster round
    for (int round = 0; round < 2 && !st; ++round)
        for (int v = 0; v < (int)vs.size(); ++v) {
            if (vs[v].small_only && !small) continue;
            if (!ev.start(s)) { st = MPX_EDEVICE; break; }
            for (int r = 0; r < reps && !st; ++r) st = vs[v].fn(g, s);
            float ms = 0.f;
            if (st || !ev.stop(s) || !ev.elapsed(&ms)) { st = st ? st : MPX_EDEVICE; break; }
            ms /= reps;
            if (t[v] < 0.f || ms < t[v]) t[v] = ms;
            if (best < 0 || ms < best_t) { best = v; best_t = ms; }
        }
    if (st) return st;
    // Keep the size heuristic's tiling unless another is at least 1 % faster:
    // tilings within run-to-run noise of each other (the QD ones at 2048 are
    // within 1-2 %) would otherwise be picked at random, and the heuristic's
    // larger tile reads less from HBM.
    if (t[v0] > 0.f && t[v0] <= 1.01f * best_t) {
        best = v0;
        best_t = t[v0];
    }
    tune_store(tune_key(prec, g), vs[best].name);
    if (best_ms) *best_ms = best_t;
    return best;
}

// Forget this process's tuned GEMM choices (back to the size heuristic); the
// cache file, if any, is left as it is.
extern "C" void mpx_gemm_autotune_reset(void) { tune_forget("gemm"); }

// ------------------------------------------------------- batched GEMM ----
//
// Many independent products C_p = A_p B_p of ragged shapes in one persistent
// launch (the batching pattern applied to small GEMMs).  A plan lists every
// (problem, tile) work item of every tiling variant, longest k first; the
// workgroups of one launch pull items from a counter and run the same tile
// routine as k_gemm, so each entry is the naive triple loop's sequence.
// Operands are packed: A_p (m_p x k_p, row-major) starts at element
// sum_{q<p} m_q k_q of every component plane, likewise B_p (k_p x n_p) and
// C_p (m_p x n_p).

namespace mpx {

struct GbProb {
    int m, n, k;
    long long a, b, c;  // first element of A_p, B_p, C_p in their planes
};
struct GbItem {
    int p, m0, n0;
};

__global__ void k_gb_reset(int* c) { *c = 0; }

template <typename T, int K, int TM, int TN, int BK, int AR, bool PF = false>
__global__ void __launch_bounds__(kGemmThreads)
k_gemm_batched(int nitems, const GbItem* __restrict__ items, const GbProb* __restrict__ probs,
               const T* __restrict__ A, long long psA, const T* __restrict__ B, long long psB,
               T* __restrict__ C, long long psC, int* counter) {
    __shared__ T sA[K][BK][16 * TM];
    __shared__ T sB[K][BK][16 * TN];
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int it = next;
        __syncthreads();  // all have read `next` before it is overwritten
        if (it >= nitems) break;  // the same value in every thread: uniform exit
        const GbItem w = items[it];
        const GbProb q = probs[w.p];
        gemm_tile<T, K, TM, TN, BK, false, false, AR, PF>(q.m, q.n, q.k, A + q.a, q.k, psA, B + q.b,
                                                          q.n, psB, C + q.c, q.n, psC, w.m0, w.n0,
                                                          sA, sB);
    }
}

// Wave tiles: each wave of the workgroup pulls its own 8 x 8 item (so the
// padding of ragged m and n is at most 7 rows / columns) and lane l computes
// entry (l / 8, l % 8) with the sequential-k multiply-add of the naive loop,
// operands read straight from global memory (the eight lanes of a row share
// each A load, the eight of a column each B load).  Loads of U consecutive
// k are issued before their multiply-adds.  Lanes outside the problem read a
// clamped (valid) row / column and store nothing.
template <typename T, int K, int U, int AR>
__device__ __forceinline__ void wave_tile(const GbItem& w, const GbProb& q, const T* __restrict__ A,
                                          long long psA, const T* __restrict__ B, long long psB,
                                          T* __restrict__ C, long long psC) {
    const int lane = threadIdx.x & 63;
    const int lr = lane >> 3, lc = lane & 7;
    {
        const int row = w.m0 + lr, col = w.n0 + lc;
        const long long ar = (long long)(row < q.m ? row : q.m - 1) * q.k;
        const long long bc = col < q.n ? col : q.n - 1;
        const T* __restrict__ Ap = A + q.a;
        const T* __restrict__ Bp = B + q.b;
        mpn<T, K> acc = mp_zero<T, K>();
        int l = 0;
        for (; l + U <= q.k; l += U) {
            mpn<T, K> a[U], b[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                a[u] = mp_load<T, K>(Ap, psA, ar + l + u);
                b[u] = mp_load<T, K>(Bp, psB, (long long)(l + u) * q.n + bc);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) acc = ar_add<AR>(acc, ar_mul<AR>(a[u], b[u]));
        }
        for (; l < q.k; ++l)
            acc = ar_add<AR>(acc, ar_mul<AR>(mp_load<T, K>(Ap, psA, ar + l),
                                              mp_load<T, K>(Bp, psB, (long long)l * q.n + bc)));
        if (row < q.m && col < q.n) mp_store<T, K>(C + q.c, psC, (long long)row * q.n + col, acc);
    }
}

// A flat edge item of the mixed tiling: 64 consecutive entries, in row-major
// order, of one of a product's two edge strips left by its BM x BN interior
// tiles (n0 = -1: the bottom strip, rows [fm, m) x columns [0, n); n0 = -2:
// the right strip, rows [0, fm) x columns [fn, n)), starting at entry m0 of
// the strip.  Each lane computes its entry like wave_tile; only the strip's
// last item has idle lanes.
template <typename T, int K, int U, int AR, int BM, int BN>
__device__ __forceinline__ void wave_flat(const GbItem& w, const GbProb& q, const T* __restrict__ A,
                                          long long psA, const T* __restrict__ B, long long psB,
                                          T* __restrict__ C, long long psC) {
    const int fm = q.m / BM * BM, fn = q.n / BN * BN;
    const int r0 = w.n0 == -1 ? fm : 0, c0 = w.n0 == -1 ? 0 : fn;
    const int wid = w.n0 == -1 ? q.n : q.n - fn;
    const int cnt = w.n0 == -1 ? (q.m - fm) * q.n : fm * (q.n - fn);
    const int t = w.m0 + (int)(threadIdx.x & 63);
    const int tt = t < cnt ? t : cnt - 1;  // idle lanes repeat the last entry, unstored
    const int row = r0 + tt / wid, col = c0 + tt % wid;
    const long long ar = (long long)row * q.k;
    const T* __restrict__ Ap = A + q.a;
    const T* __restrict__ Bp = B + q.b;
    mpn<T, K> acc = mp_zero<T, K>();
    int l = 0;
    for (; l + U <= q.k; l += U) {
        mpn<T, K> a[U], b[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a[u] = mp_load<T, K>(Ap, psA, ar + l + u);
            b[u] = mp_load<T, K>(Bp, psB, (long long)(l + u) * q.n + col);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) acc = ar_add<AR>(acc, ar_mul<AR>(a[u], b[u]));
    }
    for (; l < q.k; ++l)
        acc = ar_add<AR>(acc, ar_mul<AR>(mp_load<T, K>(Ap, psA, ar + l),
                                          mp_load<T, K>(Bp, psB, (long long)l * q.n + col)));
    if (t < cnt) mp_store<T, K>(C + q.c, psC, (long long)row * q.n + col, acc);
}

template <typename T, int K, int U, int AR>
__global__ void __launch_bounds__(kGemmThreads)
k_gemm_batched_wave(int nitems, const GbItem* __restrict__ items,
                    const GbProb* __restrict__ probs, const T* __restrict__ A, long long psA,
                    const T* __restrict__ B, long long psB, T* __restrict__ C, long long psC,
                    int* counter) {
    const int lane = threadIdx.x & 63;
    for (;;) {
        int it = 0;
        if (lane == 0) it = atomicAdd(counter, 1);
        it = __shfl(it, 0, 64);
        if (it >= nitems) break;  // the same value in every lane: uniform exit
        const GbItem w = items[it];
        wave_tile<T, K, U, AR>(w, probs[w.p], A, psA, B, psB, C, psC);
    }
}

// Mixed tiling: the interior of each product in 16 TM x 16 TN workgroup
// tiles and its ragged edges in 8 x 8 wave tiles, or (flat edges) in waves of
// 64 consecutive entries of each edge strip.  A work unit is four
// consecutive items: a workgroup tile (item 1 has p = kGbTileUnit, items 2
// and 3 unused) or up to four wave tiles, one per wave (p = -1: none).  The
// unit kind is read by the whole workgroup, so the barriers inside the
// workgroup tile are reached by every thread.
constexpr int kGbTileUnit = -2;

template <typename T, int K, int TM, int TN, int BK, int U, int AR, bool PF = false>
__global__ void __launch_bounds__(kGemmThreads)
k_gemm_batched_mixed(int nunits, const GbItem* __restrict__ items,
                     const GbProb* __restrict__ probs, const T* __restrict__ A, long long psA,
                     const T* __restrict__ B, long long psB, T* __restrict__ C, long long psC,
                     int* counter) {
    __shared__ T sA[K][BK][16 * TM];
    __shared__ T sB[K][BK][16 * TN];
    __shared__ int next;
    const int wv = threadIdx.x >> 6;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int u = next;
        __syncthreads();  // all have read `next` before it is overwritten
        if (u >= nunits) break;  // the same value in every thread: uniform exit
        const GbItem* unit = items + 4LL * u;
        if (unit[1].p == kGbTileUnit) {
            const GbItem w = unit[0];
            const GbProb q = probs[w.p];
            gemm_tile<T, K, TM, TN, BK, false, false, AR, PF>(q.m, q.n, q.k, A + q.a, q.k, psA,
                                                              B + q.b, q.n, psB, C + q.c, q.n, psC,
                                                              w.m0, w.n0, sA, sB);
        } else {
            const GbItem w = unit[wv];
            if (w.p >= 0) {
                if (w.n0 < 0)
                    wave_flat<T, K, U, AR, 16 * TM, 16 * TN>(w, probs[w.p], A, psA, B, psB, C, psC);
                else
                    wave_tile<T, K, U, AR>(w, probs[w.p], A, psA, B, psB, C, psC);
            }
        }
    }
}

struct GbVariant {
    int (*launch)(int nitems, const GbItem*, const GbProb*, const void*, long long, const void*,
                  long long, void*, long long, int*, int grid, hipStream_t);
    int bm, bn;
    int per_wg;  // items a workgroup runs at once (4 for wave tiles)
    bool mixed;  // work units of the mixed tiling (bm x bn interior, 8 x 8 edges)
    bool flat = false;  // mixed, with the edges as flat 64-entry waves
};

template <typename T, int K, int TM, int TN, int BK, int AR, bool PF = false>
static int gb_launch(int nitems, const GbItem* items, const GbProb* probs, const void* A,
                     long long psA, const void* B, long long psB, void* C, long long psC,
                     int* counter, int grid, hipStream_t s) {
    k_gemm_batched<T, K, TM, TN, BK, AR, PF><<<grid, kGemmThreads, 0, s>>>(
        nitems, items, probs, (const T*)A, psA, (const T*)B, psB, (T*)C, psC, counter);
    return launch_status();
}

template <typename T, int K, int TM, int TN, int BK, int U, int AR, bool PF = false>
static int gb_launch_mixed(int nunits, const GbItem* items, const GbProb* probs, const void* A,
                           long long psA, const void* B, long long psB, void* C, long long psC,
                           int* counter, int grid, hipStream_t s) {
    k_gemm_batched_mixed<T, K, TM, TN, BK, U, AR, PF><<<grid, kGemmThreads, 0, s>>>(
        nunits, items, probs, (const T*)A, psA, (const T*)B, psB, (T*)C, psC, counter);
    return launch_status();
}

template <typename T, int K, int U, int AR>
static int gb_launch_wave(int nitems, const GbItem* items, const GbProb* probs, const void* A,
                          long long psA, const void* B, long long psB, void* C, long long psC,
                          int* counter, int grid, hipStream_t s) {
    k_gemm_batched_wave<T, K, U, AR><<<grid, kGemmThreads, 0, s>>>(
        nitems, items, probs, (const T*)A, psA, (const T*)B, psB, (T*)C, psC, counter);
    return launch_status();
}

// Tilings offered for batches: 8 x 8 wave tiles, then the regular GEMM's,
// smallest tiles first (small problems need many tiles to fill the chip, and
// small tiles waste less on ragged edges).
static std::vector<GbVariant> gb_variants(int prec) {
#define MPX_GB(T_, K_, TM_, TN_, BK_, AR_) GbVariant{gb_launch<T_, K_, TM_, TN_, BK_, AR_>, 16 * TM_, 16 * TN_, 1, false}
#define MPX_GBW(T_, K_, U_, AR_) GbVariant{gb_launch_wave<T_, K_, U_, AR_>, 8, 8, kGemmThreads / 64, false}
#define MPX_GBM(T_, K_, TM_, TN_, BK_, U_, AR_) \
    GbVariant{gb_launch_mixed<T_, K_, TM_, TN_, BK_, U_, AR_>, 16 * TM_, 16 * TN_, 1, true}
    // the same workgroup tiles with the LDS-prefetching panel loop
#define MPX_GBP(T_, K_, TM_, TN_, BK_, AR_) GbVariant{gb_launch<T_, K_, TM_, TN_, BK_, AR_, true>, 16 * TM_, 16 * TN_, 1, false}
#define MPX_GBMP(T_, K_, TM_, TN_, BK_, U_, AR_) \
    GbVariant{gb_launch_mixed<T_, K_, TM_, TN_, BK_, U_, AR_, true>, 16 * TM_, 16 * TN_, 1, true}
    // mixed with flat edges (the same kernels; only the work list differs)
#define MPX_GBMF(T_, K_, TM_, TN_, BK_, U_, AR_) \
    GbVariant{gb_launch_mixed<T_, K_, TM_, TN_, BK_, U_, AR_, true>, 16 * TM_, 16 * TN_, 1, true, true}
    switch (prec) {
        case MPX_DD: return {MPX_GBW(double, 2, 4, AR_BF), MPX_GB(double, 2, 2, 2, 16, AR_BF), MPX_GB(double, 2, 2, 4, 8, AR_BF), MPX_GB(double, 2, 4, 4, 8, AR_BF),
                             MPX_GBP(double, 2, 2, 2, 16, AR_BF), MPX_GBMP(double, 2, 1, 1, 16, 4, AR_BF),
                             MPX_GBMF(double, 2, 1, 1, 16, 4, AR_BF)};
        case MPX_TD: return {MPX_GBM(double, 3, 1, 2, 16, 2, AR_BF), MPX_GBW(double, 3, 2, AR_BF), MPX_GB(double, 3, 1, 2, 16, AR_BF), MPX_GB(double, 3, 2, 2, 8, AR_BF), MPX_GB(double, 3, 2, 4, 8, AR_BF),
                             MPX_GBMP(double, 3, 1, 2, 16, 2, AR_BF), MPX_GBMP(double, 3, 1, 1, 16, 2, AR_BF),
                             MPX_GBMF(double, 3, 1, 2, 16, 2, AR_BF), MPX_GBMF(double, 3, 1, 1, 16, 2, AR_BF)};
        case MPX_QD: return {MPX_GBM(double, 4, 1, 1, 16, 2, AR_BF), MPX_GBW(double, 4, 2, AR_BF), MPX_GB(double, 4, 1, 1, 16, AR_BF), MPX_GB(double, 4, 1, 2, 16, AR_BF), MPX_GB(double, 4, 2, 2, 8, AR_BF),
                             MPX_GBMP(double, 4, 1, 1, 16, 2, AR_BF), MPX_GBMP(double, 4, 1, 2, 16, 2, AR_BF),
                             MPX_GBMF(double, 4, 1, 1, 16, 2, AR_BF), MPX_GBMF(double, 4, 1, 2, 16, 2, AR_BF)};
        case MPX_FF: return {MPX_GBW(float, 2, 4, AR_BF), MPX_GB(float, 2, 2, 2, 16, AR_BF), MPX_GB(float, 2, 2, 4, 8, AR_BF), MPX_GB(float, 2, 4, 4, 8, AR_BF),
                             MPX_GBP(float, 2, 2, 2, 16, AR_BF), MPX_GBMP(float, 2, 1, 1, 16, 4, AR_BF),
                             MPX_GBMF(float, 2, 1, 1, 16, 4, AR_BF)};
        default: return {};
    }
#undef MPX_GBMF
#undef MPX_GBMP
#undef MPX_GBP
#undef MPX_GBM
#undef MPX_GBW
#undef MPX_GB
}

}  // namespace mpx

struct mpx_gemm_plan_s {
    int prec = 0, count = 0, variant = 0, cus = 256;
    long long totA = 0, totB = 0, totC = 0;
    std::vector<mpx::GbVariant> vars;
    std::vector<int> nitems;           // per variant
    std::vector<long long> item_off;   // per variant: first item in the device array
    void* dev = nullptr;               // probs, items of every variant, counter
    mpx::GbProb* probs = nullptr;
    mpx::GbItem* items = nullptr;
    int* counter = nullptr;
};

static int gemm_batched_plan(mpx_gemm_plan* out, int prec, int64_t count, const int64_t* m,
                             const int64_t* n, const int64_t* k) {
    using namespace mpx;
    if (out == nullptr) return MPX_EINVAL;
    *out = nullptr;
    if (!prec_k(prec)) return MPX_EPREC;
    if (count < 0 || count > INT32_MAX || (count > 0 && (!m || !n || !k))) return MPX_EINVAL;
    std::unique_ptr<mpx_gemm_plan_s> holder(new (std::nothrow) mpx_gemm_plan_s());
    if (!holder) return MPX_EDEVICE;
    mpx_gemm_plan_s* p = holder.get();
    p->prec = prec;
    p->count = (int)count;
    p->vars = gb_variants(prec);
    std::vector<GbProb> probs(count);
    for (int64_t i = 0; i < count; ++i) {
        if (m[i] < 0 || n[i] < 0 || k[i] < 0 || m[i] > (1 << 20) || n[i] > (1 << 20) ||
            k[i] > (1 << 20))
            return MPX_EINVAL;
        probs[i] = GbProb{(int)m[i], (int)n[i], (int)k[i], p->totA, p->totB, p->totC};
        p->totA += m[i] * k[i];
        p->totB += k[i] * n[i];
        p->totC += m[i] * n[i];
    }
    // work items of every variant, longest k first (ties: problem, tile order)
    std::vector<GbItem> all;
    for (const auto& v : p->vars) {
        long long nit = 0;  // items (tiles; for the mixed tiling at most 4 items per tile or edge tile)
        for (int64_t i = 0; i < count; ++i)
            nit += (v.mixed ? 4 * ceil_div(probs[i].m, 8) * ceil_div(probs[i].n, 8)
                            : ceil_div(probs[i].m, v.bm) * ceil_div(probs[i].n, v.bn));
        if (nit > INT32_MAX / 2) return MPX_ENOTSUP;  // the work counter is an int
    }
    auto by_k = [&](const GbItem& a, const GbItem& b) { return probs[a.p].k > probs[b.p].k; };
    for (const auto& v : p->vars) {
        std::vector<GbItem> items;
        int nunits = 0;
        if (!v.mixed) {
            for (int64_t i = 0; i < count; ++i)
                for (int r = 0; r < probs[i].m; r += v.bm)
                    for (int c = 0; c < probs[i].n; c += v.bn) items.push_back(GbItem{(int)i, r, c});
            std::stable_sort(items.begin(), items.end(), by_k);
            nunits = (int)items.size();
        } else {
            // interior bm x bn tiles over [0, fm) x [0, fn); 8 x 8 edge tiles over
            // the rest; units of one tile or four edge tiles, longest k first
            std::vector<GbItem> tiles, edges;
            for (int64_t i = 0; i < count; ++i) {
                const int m = probs[i].m, n = probs[i].n;
                const int fm = m / v.bm * v.bm, fn = n / v.bn * v.bn;
                for (int r = 0; r < fm; r += v.bm)
                    for (int c = 0; c < fn; c += v.bn) tiles.push_back(GbItem{(int)i, r, c});
                if (v.flat) {
                    // 64-entry runs of the bottom strip (n0 = -1) and the right strip (n0 = -2)
                    const long long bottom = (long long)(m - fm) * n, right = (long long)fm * (n - fn);
                    for (long long t = 0; t < bottom; t += 64) edges.push_back(GbItem{(int)i, (int)t, -1});
                    for (long long t = 0; t < right; t += 64) edges.push_back(GbItem{(int)i, (int)t, -2});
                } else {
                    for (int r = fm; r < m; r += 8)
                        for (int c = 0; c < n; c += 8) edges.push_back(GbItem{(int)i, r, c});
                    for (int r = 0; r < fm; r += 8)
                        for (int c = fn; c < n; c += 8) edges.push_back(GbItem{(int)i, r, c});
                }
            }
            std::stable_sort(tiles.begin(), tiles.end(), by_k);
            std::stable_sort(edges.begin(), edges.end(), by_k);
            const GbItem none{-1, 0, 0}, tile_mark{kGbTileUnit, 0, 0};
            size_t a = 0, e = 0;
            while (a < tiles.size() || e < edges.size()) {
                const bool take_tile = e >= edges.size() ||
                                       (a < tiles.size() && probs[tiles[a].p].k >= probs[edges[e].p].k);
                if (take_tile) {
                    items.insert(items.end(), {tiles[a++], tile_mark, none, none});
                } else {
                    for (int w = 0; w < 4; ++w) items.push_back(e < edges.size() ? edges[e++] : none);
                }
                ++nunits;
            }
        }
        p->item_off.push_back((long long)all.size());
        p->nitems.push_back(nunits);
        all.insert(all.end(), items.begin(), items.end());
    }
    const size_t sz_p = std::max<size_t>(probs.size(), 1) * sizeof(GbProb);
    const size_t sz_i = std::max<size_t>(all.size(), 1) * sizeof(GbItem);
    const size_t off_i = (sz_p + 255) & ~size_t(255), off_c = (off_i + sz_i + 255) & ~size_t(255);
    if (hipMalloc(&p->dev, off_c + 256) != hipSuccess) {
        p->dev = nullptr;
        return MPX_EDEVICE;
    }
    p->probs = (GbProb*)p->dev;
    p->items = (GbItem*)((char*)p->dev + off_i);
    p->counter = (int*)((char*)p->dev + off_c);
    if ((!probs.empty() && hipMemcpy(p->probs, probs.data(), probs.size() * sizeof(GbProb),
                                     hipMemcpyHostToDevice) != hipSuccess) ||
        (!all.empty() && hipMemcpy(p->items, all.data(), all.size() * sizeof(GbItem),
                                   hipMemcpyHostToDevice) != hipSuccess)) {
        (void)hipFree(p->dev);
        p->dev = nullptr;
        return MPX_EDEVICE;
    }
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        p->cus = prop.multiProcessorCount;
    *out = holder.release();
    return MPX_OK;
}

// Host allocation failures (the schedule's vectors) end as MPX_EDEVICE: no
// exception crosses the C boundary.
extern "C" int mpx_gemm_batched_plan(mpx_gemm_plan* out, int prec, int64_t count,
                                     const int64_t* m, const int64_t* n, const int64_t* k) {
    try {
        return gemm_batched_plan(out, prec, count, m, n, k);
    } catch (const std::bad_alloc&) {
        return MPX_EDEVICE;
    }
}

extern "C" int mpx_gemm_plan_destroy(mpx_gemm_plan p) {
    if (!p) return MPX_EINVAL;
    if (p->dev) (void)hipFree(p->dev);
    delete p;
    return MPX_OK;
}

extern "C" int mpx_gemm_batched_variant_count(mpx_gemm_plan p) {
    return p ? (int)p->vars.size() : 0;
}

extern "C" int mpx_gemm_batched_set_variant(mpx_gemm_plan p, int v) {
    if (!p || v < 0 || v >= (int)p->vars.size()) return MPX_EINVAL;
    p->variant = v;
    return MPX_OK;
}

static int gb_check(mpx_gemm_plan p, const void* A, int64_t psA, const void* B, int64_t psB,
                    const void* C, int64_t psC) {
    if (!p) return MPX_EINVAL;
    if (p->totA > 0 && (!A || psA < p->totA)) return MPX_EINVAL;
    if (p->totB > 0 && (!B || psB < p->totB)) return MPX_EINVAL;
    if (p->totC > 0 && (!C || psC < p->totC)) return MPX_EINVAL;
    const int K = mpx::prec_k(p->prec);
    const size_t elt = mpx::is_ff(p->prec) ? sizeof(float) : sizeof(double);
    const uint64_t bc = mpx::planes_bytes(K, 1, p->totC, p->totC, psC, elt);
    if (mpx::overlaps(C, bc, A, mpx::planes_bytes(K, 1, p->totA, p->totA, psA, elt)) ||
        mpx::overlaps(C, bc, B, mpx::planes_bytes(K, 1, p->totB, p->totB, psB, elt)))
        return MPX_EINVAL;  // C must not overlap A or B
    return MPX_OK;
}

static int gb_run(mpx_gemm_plan p, int v, const void* A, int64_t psA, const void* B,
                  int64_t psB, void* C, int64_t psC, hipStream_t s) {
    using namespace mpx;
    const int ni = p->nitems[v];
    if (ni == 0) return MPX_OK;
    k_gb_reset<<<1, 1, 0, s>>>(p->counter);
    int st = launch_status();
    if (st) return st;
    const int per = p->vars[v].per_wg;
    const int grid = (int)std::min<long long>((ni + per - 1) / per, (long long)p->cus * 8);
    return p->vars[v].launch(ni, p->items + p->item_off[v], p->probs, A, psA, B, psB, C, psC,
                             p->counter, grid, s);
}

extern "C" int mpx_gemm_batched(mpx_gemm_plan p, const void* A, int64_t psA, const void* B,
                                int64_t psB, void* C, int64_t psC, void* stream) {
    int st = gb_check(p, A, psA, B, psB, C, psC);
    if (st) return st;
    return gb_run(p, p->variant, A, psA, B, psB, C, psC, mpx::as_stream(stream));
}

extern "C" int mpx_gemm_batched_autotune(mpx_gemm_plan p, const void* A, int64_t psA,
                                         const void* B, int64_t psB, void* C, int64_t psC,
                                         int reps, float* best_ms, void* stream) {
    int st = gb_check(p, A, psA, B, psB, C, psC);
    if (st) return st;
    if (reps < 1) return MPX_EINVAL;
    hipStream_t s = mpx::as_stream(stream);
    mpx::EventPair ev;
    if (!ev.ok) return MPX_EDEVICE;
    st = mpx::warm_clock(ev, s, [&] { return gb_run(p, p->variant, A, psA, B, psB, C, psC, s); });
    int best = -1;
    float best_t = 0.f;
    // two rounds over all variants, each variant's faster round counts (as
    // in mpx_gemm_autotune)
    for (int round = 0; round < 2 && !st; ++round)
        for (int v = 0; v < (int)p->vars.size() && !st; ++v) {
            if (!ev.start(s)) { st = MPX_EDEVICE; break; }
            for (int r = 0; r < reps && !st; ++r) st = gb_run(p, v, A, psA, B, psB, C, psC, s);
            float ms = 0.f;
            if (st || !ev.stop(s) || !ev.elapsed(&ms)) { st = st ? st : MPX_EDEVICE; break; }
            ms /= reps;
            if (best < 0 || ms < best_t) { best = v; best_t = ms; }
        }
    if (st) return st;
    p->variant = best < 0 ? 0 : best;
    if (best_ms) *best_ms = best_t;
    return p->variant;
}
