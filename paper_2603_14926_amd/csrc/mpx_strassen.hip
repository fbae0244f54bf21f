// mpx_strassen.hip -- C := A B by Strassen's recursion on gfx950.
//
// Section 3.1 runs its matrix benchmarks with Strassen's algorithm (recursion
// stopped below 32 x 32 on the CPU).  The classic seven-product form is used
// (Strassen, Numer. Math. 13, 1969):
//   M1 = (A11 + A22)(B11 + B22)   M2 = (A21 + A22) B11   M3 = A11 (B12 - B22)
//   M4 = A22 (B21 - B11)          M5 = (A11 + A12) B22   M6 = (A21 - A11)(B11 + B12)
//   M7 = (A12 - A22)(B21 + B22)
//   C11 = ((M1 + M4) - M5) + M7   C12 = M3 + M5   C21 = M2 + M4
//   C22 = ((M1 - M2) + M3) + M6
// A product (m, k) x (k, n) splits while min(m, k, n) >= cutoff; each
// dimension d splits into ceil(d/2) + floor(d/2) and trailing blocks are
// zero-padded to the leading block's shape.  Leaves are the tuned classical
// GEMM (sequential k per entry), so every result is a fixed sequence of
// multicomponent operations, identical for any tiling.
//
// On the GPU one level trades one eighth of the multiply-adds (the VALU-bound
// part) for 18 block additions (HBM-bound, a few tens of microseconds each at
// n = 2048), so it pays once the leaves are large enough to run the GEMM near
// its peak: the benchmark uses cutoff 2048 (one level at n = 2048, two at
// 4096).  The recursion runs on the host and launches into the caller's
// stream; its temporaries come from the caller's workspace: per level one
// operand sum of each side and one product block, accumulated into C in the
// order above, so a level needs K (m1 k1 + k1 n1 + m1 n1) numbers.
#include "mp_arith.hpp"
#include "mp_conv.hpp"
#include "mpx_internal.hpp"

#include <algorithm>

namespace mpx {

constexpr int kStBlock = 256;

static unsigned st_grid(long long total) {
    long long b = ceil_div(total, kStBlock);
    return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

// Z (r x c) := Xp + Yp, or Xp - Yp with neg_y, or Xp alone when Y is null;
// Xp is X (its true shape xr x xc) extended by zeros to r x c, likewise Yp.
template <typename T, int K, int AR>
__global__ void __launch_bounds__(kStBlock)
k_st_sum(int r, int c, const T* __restrict__ X, long long ldx, long long psx, int xr, int xc,
         const T* __restrict__ Y, long long ldy, long long psy, int yr, int yc, int neg_y,
         T* __restrict__ Z, long long ldz, long long psz) {
    const long long total = (long long)r * c;
    for (long long t = (long long)blockIdx.x * kStBlock + threadIdx.x; t < total;
         t += (long long)gridDim.x * kStBlock) {
        const int i = (int)(t / c), j = (int)(t % c);
        const bool inx = i < xr && j < xc;
        mpn<T, K> z;
#pragma unroll
        for (int q = 0; q < K; ++q) z.c[q] = inx ? X[q * psx + (long long)i * ldx + j] : T(0);
        if (Y != nullptr) {
            const bool iny = i < yr && j < yc;
            mpn<T, K> y;
#pragma unroll
            for (int q = 0; q < K; ++q) y.c[q] = iny ? Y[q * psy + (long long)i * ldy + j] : T(0);
            if (neg_y) y = mp_neg(y);
            z = ar_add<AR>(z, y);
        }
        mp_store<T, K>(Z, psz, (long long)i * ldz + j, z);
    }
}

// C block (its true shape cr x cc) := M (mode 0), C + M (mode 1), C - M (2).
template <typename T, int K, int AR>
__global__ void __launch_bounds__(kStBlock)
k_st_acc(int cr, int cc, T* __restrict__ C, long long ldc, long long psc,
         const T* __restrict__ M, long long ldm, long long psm, int mode) {
    const long long total = (long long)cr * cc;
    for (long long t = (long long)blockIdx.x * kStBlock + threadIdx.x; t < total;
         t += (long long)gridDim.x * kStBlock) {
        const int i = (int)(t / cc), j = (int)(t % cc);
        const long long ic = (long long)i * ldc + j;
        mpn<T, K> v = mp_load<T, K>(M, psm, (long long)i * ldm + j);
        if (mode != 0) {
            if (mode == 2) v = mp_neg(v);
            v = ar_add<AR>(mp_load<T, K>(C, psc, ic), v);
        }
        mp_store<T, K>(C, psc, ic, v);
    }
}

static bool st_split(long long m, long long k, long long n, long long cutoff) {
    return std::min(m, std::min(k, n)) >= cutoff;
}

// Levels of the recursion for a shape, and the workspace it needs (numbers).
static int st_levels(long long m, long long k, long long n, long long cutoff, long long* elems,
                     int K) {
    int lv = 0;
    long long tot = 0;
    while (st_split(m, k, n, cutoff)) {
        const long long m1 = (m + 1) / 2, k1 = (k + 1) / 2, n1 = (n + 1) / 2;
        tot += (long long)K * (m1 * k1 + k1 * n1 + m1 * n1);
        m = m1; k = k1; n = n1;
        ++lv;
    }
    if (elems) *elems = tot;
    return lv;
}

constexpr int kStMaxLevels = 8;  // 7^8 = 5.8e6 leaf products: beyond, refuse

size_t strassen_workspace(int prec, long long m, long long n, long long k, long long cutoff) {
    const int K = prec_k_ar(prec);
    if (!K || cutoff < 2) return 0;
    long long e = 0;
    st_levels(m, k, n, cutoff, &e, K);
    const size_t elt = is_ff(base_prec(prec)) ? sizeof(float) : sizeof(double);
    return (size_t)e * elt;
}

template <typename T>
struct StBlk {
    const T* p;
    long long ld, ps, r, c;  // true shape r x c
};

template <typename T, int K, int AR>
struct Strassen {
    int prec;
    long long cutoff;
    hipStream_t s;

    // Operand of a product: the sum (or difference) of two blocks, or one
    // block, as an r x c matrix.  A single block of full shape is used in
    // place; anything else is formed in buf (ld c, plane stride r c).
    int operand(const StBlk<T>& X, const StBlk<T>* Y, int neg_y, long long r, long long c,
                T* buf, StBlk<T>& out) {
        if (Y == nullptr && X.r == r && X.c == c) {
            out = X;
            return MPX_OK;
        }
        k_st_sum<T, K, AR><<<st_grid(r * c), kStBlock, 0, s>>>(
            (int)r, (int)c, X.p, X.ld, X.ps, (int)X.r, (int)X.c, Y ? Y->p : nullptr, Y ? Y->ld : 0,
            Y ? Y->ps : 0, Y ? (int)Y->r : 0, Y ? (int)Y->c : 0, neg_y, buf, c, r * c);
        out = StBlk<T>{buf, c, r * c, r, c};
        return launch_status();
    }

    int acc(const StBlk<T>& Cb, const T* M, long long ldm, long long psm, int mode) {
        k_st_acc<T, K, AR><<<st_grid(Cb.r * Cb.c), kStBlock, 0, s>>>(
            (int)Cb.r, (int)Cb.c, const_cast<T*>(Cb.p), Cb.ld, Cb.ps, M, ldm, psm, mode);
        return launch_status();
    }

    int run(long long m, long long k, long long n, const StBlk<T>& A, const StBlk<T>& B,
            T* C, long long ldc, long long psC, T* ws) {
        if (!st_split(m, k, n, cutoff))
            return mpx_gemm(prec, 0, 0, m, n, k, A.p, A.ld, A.ps, B.p, B.ld, B.ps, C, ldc, psC,
                            (void*)s);
        const long long m1 = (m + 1) / 2, m2 = m / 2, k1 = (k + 1) / 2, k2 = k / 2;
        const long long n1 = (n + 1) / 2, n2 = n / 2;
        T* S = ws;
        T* Tb = S + K * m1 * k1;
        T* M = Tb + K * k1 * n1;
        T* child = M + K * m1 * n1;
        const long long psM = m1 * n1;
        const StBlk<T> A11{A.p, A.ld, A.ps, m1, k1}, A12{A.p + k1, A.ld, A.ps, m1, k2};
        const StBlk<T> A21{A.p + m1 * A.ld, A.ld, A.ps, m2, k1};
        const StBlk<T> A22{A.p + m1 * A.ld + k1, A.ld, A.ps, m2, k2};
        const StBlk<T> B11{B.p, B.ld, B.ps, k1, n1}, B12{B.p + n1, B.ld, B.ps, k1, n2};
        const StBlk<T> B21{B.p + k1 * B.ld, B.ld, B.ps, k2, n1};
        const StBlk<T> B22{B.p + k1 * B.ld + n1, B.ld, B.ps, k2, n2};
        const StBlk<T> C11{C, ldc, psC, m1, n1}, C12{C + n1, ldc, psC, m1, n2};
        const StBlk<T> C21{C + m1 * ldc, ldc, psC, m2, n1}, C22{C + m1 * ldc + n1, ldc, psC, m2, n2};
        struct Prod {
            const StBlk<T>* lx; const StBlk<T>* ly; int lneg;
            const StBlk<T>* rx; const StBlk<T>* ry; int rneg;
        };
        const Prod P[7] = {
            {&A11, &A22, 0, &B11, &B22, 0},      // M1
            {&A21, &A22, 0, &B11, nullptr, 0},  // M2
            {&A11, nullptr, 0, &B12, &B22, 1},  // M3
            {&A22, nullptr, 0, &B21, &B11, 1},  // M4
            {&A11, &A12, 0, &B22, nullptr, 0},  // M5
            {&A21, &A11, 1, &B11, &B12, 0},      // M6
            {&A12, &A22, 1, &B21, &B22, 0},      // M7
        };
        // C-block updates after each product, in the order of the formulas
        struct Upd { const StBlk<T>* c; int mode; };
        const Upd U[7][2] = {
            {{&C11, 0}, {&C22, 0}}, {{&C21, 0}, {&C22, 2}}, {{&C12, 0}, {&C22, 1}},
            {{&C11, 1}, {&C21, 1}}, {{&C11, 2}, {&C12, 1}}, {{&C22, 1}, {nullptr, 0}},
            {{&C11, 1}, {nullptr, 0}},
        };
        int st;
        for (int t = 0; t < 7; ++t) {
            StBlk<T> L, R;
            if ((st = operand(*P[t].lx, P[t].ly, P[t].lneg, m1, k1, S, L))) return st;
            if ((st = operand(*P[t].rx, P[t].ry, P[t].rneg, k1, n1, Tb, R))) return st;
            if ((st = run(m1, k1, n1, L, R, M, n1, psM, child))) return st;
            for (int u = 0; u < 2; ++u)
                if (U[t][u].c && (st = acc(*U[t][u].c, M, n1, psM, U[t][u].mode))) return st;
        }
        return MPX_OK;
    }
};

template <typename T, int K, int AR>
static int strassen_t(int prec, long long m, long long n, long long k, const void* A,
                      long long lda, long long psA, const void* B, long long ldb, long long psB,
                      void* C, long long ldc, long long psC, long long cutoff, void* ws,
                      hipStream_t s) {
    Strassen<T, K, AR> st{prec, cutoff, s};
    const StBlk<T> a{(const T*)A, lda, psA, m, k}, b{(const T*)B, ldb, psB, k, n};
    return st.run(m, k, n, a, b, (T*)C, ldc, psC, (T*)ws);
}

}  // namespace mpx

using namespace mpx;

extern "C" int mpx_gemm_strassen(int prec, int64_t m, int64_t n, int64_t k, const void* A,
                                 int64_t lda, int64_t psA, const void* B, int64_t ldb,
                                 int64_t psB, void* C, int64_t ldc, int64_t psC, int64_t cutoff,
                                 void* ws, size_t ws_bytes, void* stream) {
    const int K = prec_k_ar(prec);
    if (!K || base_prec(prec) == MPX_FF) return MPX_EPREC;
    if (m < 0 || n < 0 || k < 0 || cutoff < 2) return MPX_EINVAL;
    if (m > INT32_MAX / 2 || n > INT32_MAX / 2 || k > INT32_MAX / 2) return MPX_ENOTSUP;
    if (m > 0 && k > 0 && (A == nullptr || !span_fits(m, k, lda, psA))) return MPX_EINVAL;
    if (k > 0 && n > 0 && (B == nullptr || !span_fits(k, n, ldb, psB))) return MPX_EINVAL;
    if (m > 0 && n > 0 && (C == nullptr || !span_fits(m, n, ldc, psC))) return MPX_EINVAL;
    // C must not overlap A or B, nor the workspace any of them
    const uint64_t cb = planes_bytes(K, m, n, ldc, psC, sizeof(double));
    const uint64_t ab = planes_bytes(K, m, k, lda, psA, sizeof(double));
    const uint64_t bb = planes_bytes(K, k, n, ldb, psB, sizeof(double));
    if (overlaps(C, cb, A, ab) || overlaps(C, cb, B, bb)) return MPX_EINVAL;
    if (st_levels(m, k, n, cutoff, nullptr, K) > kStMaxLevels) return MPX_ENOTSUP;
    if (m == 0 || n == 0) return MPX_OK;
    const size_t need = strassen_workspace(prec, m, n, k, cutoff);
    if (need > 0 && (ws == nullptr || ws_bytes < need)) return MPX_EWORKSPACE;
    if (overlaps(ws, need, A, ab) || overlaps(ws, need, B, bb) || overlaps(ws, need, C, cb))
        return MPX_EINVAL;
    hipStream_t s = as_stream(stream);
    switch (prec) {
        case MPX_DD: return strassen_t<double, 2, AR_BF>(prec, m, n, k, A, lda, psA, B, ldb, psB, C, ldc, psC, cutoff, ws, s);
        case MPX_TD: return strassen_t<double, 3, AR_BF>(prec, m, n, k, A, lda, psA, B, ldb, psB, C, ldc, psC, cutoff, ws, s);
        case MPX_QD: return strassen_t<double, 4, AR_BF>(prec, m, n, k, A, lda, psA, B, ldb, psB, C, ldc, psC, cutoff, ws, s);
        case MPX_DD | MPX_NOBF: return strassen_t<double, 2, AR_NOBF>(prec, m, n, k, A, lda, psA, B, ldb, psB, C, ldc, psC, cutoff, ws, s);
        case MPX_TD | MPX_NOBF: return strassen_t<double, 3, AR_NOBF>(prec, m, n, k, A, lda, psA, B, ldb, psB, C, ldc, psC, cutoff, ws, s);
        case MPX_QD | MPX_NOBF: return strassen_t<double, 4, AR_NOBF>(prec, m, n, k, A, lda, psA, B, ldb, psB, C, ldc, psC, cutoff, ws, s);
        case MPX_DD | MPX_NOBF_ACC: return strassen_t<double, 2, AR_NOBF_ACC>(prec, m, n, k, A, lda, psA, B, ldb, psB, C, ldc, psC, cutoff, ws, s);
        default: return MPX_EPREC;
    }
}
