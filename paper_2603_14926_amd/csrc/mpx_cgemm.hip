// mpx_cgemm.hip -- complex matrix product by the 3M method (Section 3.2):
//   C1 = Re(A) Re(B),  C2 = Im(A) Im(B),  C3 = (Re(A) + Im(A)) (Re(B) + Im(B)),
//   Re(C) = C1 - C2,   Im(C) = (C3 - C1) - C2.
// Three real products run through the tuned branch-free GEMM (so each is the
// naive triple loop's per-entry sequence); the operand sums and the final
// combination are elementwise BF additions in one pass each.  C1 is built in
// Re(C) and C3 in Im(C); the workspace holds Re(A)+Im(A), Re(B)+Im(B) and C2.
#include "mp_arith.hpp"
#include "mpx_internal.hpp"

namespace mpx {

// Z = X + Y elementwise over a rows x cols matrix (each operand with its own
// leading dimension and plane stride).
template <typename T, int K>
__global__ void __launch_bounds__(256)
k_add2d(long long rows, long long cols, const T* __restrict__ X, long long ldx, long long psx,
        const T* __restrict__ Y, long long ldy, long long psy, T* __restrict__ Z,
        long long ldz, long long psz) {
    const long long total = rows * cols;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (long long)gridDim.x * 256) {
        const long long r = t / cols, c = t % cols;
        mp_store<T, K>(Z, psz, r * ldz + c,
                       bf_add(mp_load<T, K>(X, psx, r * ldx + c), mp_load<T, K>(Y, psy, r * ldy + c)));
    }
}

// Re = C1 - C2 (C1 read from Re), Im = (C3 - C1) - C2 (C3 read from Im).
template <typename T, int K>
__global__ void __launch_bounds__(256)
k_cgemm_combine(long long m, long long n, T* __restrict__ Re, T* __restrict__ Im, long long ldc,
                long long psC, const T* __restrict__ C2, long long ps2) {
    const long long total = m * n;
    for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (long long)gridDim.x * 256) {
        const long long r = t / n, c = t % n, idx = r * ldc + c;
        const mpn<T, K> c1 = mp_load<T, K>(Re, psC, idx);
        const mpn<T, K> c3 = mp_load<T, K>(Im, psC, idx);
        const mpn<T, K> c2 = mp_load<T, K>(C2, ps2, t);
        mp_store<T, K>(Im, psC, idx, bf_sub(bf_sub(c3, c1), c2));
        mp_store<T, K>(Re, psC, idx, bf_sub(c1, c2));
    }
}

static unsigned grid_for(long long total) {
    long long b = ceil_div(total, 256);
    return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

template <typename T, int K>
static int cgemm_t(int prec, long long m, long long n, long long k, const void* Are,
                   const void* Aim, long long lda, long long psA, const void* Bre,
                   const void* Bim, long long ldb, long long psB, void* Cre, void* Cim,
                   long long ldc, long long psC, void* ws, hipStream_t s) {
    T* SA = (T*)ws;                       // K planes of m x k
    T* SB = SA + (size_t)K * m * k;       // K planes of k x n
    T* C2 = SB + (size_t)K * k * n;       // K planes of m x n
    int st;
    if (m * k > 0) {
        k_add2d<T, K><<<grid_for(m * k), 256, 0, s>>>(m, k, (const T*)Are, lda, psA, (const T*)Aim,
                                                      lda, psA, SA, k, m * k);
        if ((st = launch_status())) return st;
    }
    if (k * n > 0) {
        k_add2d<T, K><<<grid_for(k * n), 256, 0, s>>>(k, n, (const T*)Bre, ldb, psB, (const T*)Bim,
                                                      ldb, psB, SB, n, k * n);
        if ((st = launch_status())) return st;
    }
    void* stream = (void*)s;
    if ((st = mpx_gemm(prec, 0, 0, m, n, k, Are, lda, psA, Bre, ldb, psB, Cre, ldc, psC, stream)))
        return st;
    if ((st = mpx_gemm(prec, 0, 0, m, n, k, Aim, lda, psA, Bim, ldb, psB, C2, n, m * n, stream)))
        return st;
    if ((st = mpx_gemm(prec, 0, 0, m, n, k, SA, k, m * k, SB, n, k * n, Cim, ldc, psC, stream)))
        return st;
    k_cgemm_combine<T, K><<<grid_for(m * n), 256, 0, s>>>(m, n, (T*)Cre, (T*)Cim, ldc, psC, C2,
                                                          m * n);
    return launch_status();
}

size_t cgemm_workspace(int prec, long long m, long long n, long long k) {
    const size_t elt = is_ff(prec) ? sizeof(float) : sizeof(double);
    return elt * (size_t)prec_k(prec) * (size_t)(m * k + k * n + m * n);
}

}  // namespace mpx

using namespace mpx;

extern "C" int mpx_cgemm_3m(int prec, int64_t m, int64_t n, int64_t k, const void* Are,
                            const void* Aim, int64_t lda, int64_t psA, const void* Bre,
                            const void* Bim, int64_t ldb, int64_t psB, void* Cre, void* Cim,
                            int64_t ldc, int64_t psC, void* ws, size_t ws_bytes, void* stream) {
    if (!prec_k(prec)) return MPX_EPREC;
    if (m < 0 || n < 0 || k < 0) return MPX_EINVAL;
    if (m > 0 && k > 0 && (!Are || !Aim || !span_fits(m, k, lda, psA))) return MPX_EINVAL;
    if (k > 0 && n > 0 && (!Bre || !Bim || !span_fits(k, n, ldb, psB))) return MPX_EINVAL;
    if (m > 0 && n > 0 && (!Cre || !Cim || !span_fits(m, n, ldc, psC))) return MPX_EINVAL;
    // the outputs must not overlap the inputs or each other, nor the
    // workspace any operand
    const int K = prec_k(prec);
    const size_t elt = is_ff(prec) ? sizeof(float) : sizeof(double);
    const uint64_t cb = planes_bytes(K, m, n, ldc, psC, elt);
    const uint64_t ab = planes_bytes(K, m, k, lda, psA, elt), bb = planes_bytes(K, k, n, ldb, psB, elt);
    for (const void* c : {(const void*)Cre, (const void*)Cim})
        if (overlaps(c, cb, Are, ab) || overlaps(c, cb, Aim, ab) || overlaps(c, cb, Bre, bb) ||
            overlaps(c, cb, Bim, bb))
            return MPX_EINVAL;
    if (overlaps(Cre, cb, Cim, cb)) return MPX_EINVAL;
    if (m == 0 || n == 0) return MPX_OK;
    const size_t need = cgemm_workspace(prec, m, n, k);
    if (!ws || ws_bytes < need) return MPX_EWORKSPACE;
    for (const void* q : {(const void*)Are, (const void*)Aim})
        if (overlaps(ws, need, q, ab)) return MPX_EINVAL;
    for (const void* q : {(const void*)Bre, (const void*)Bim})
        if (overlaps(ws, need, q, bb)) return MPX_EINVAL;
    if (overlaps(ws, need, Cre, cb) || overlaps(ws, need, Cim, cb)) return MPX_EINVAL;
    hipStream_t s = as_stream(stream);
    switch (prec) {
        case MPX_DD: return cgemm_t<double, 2>(prec, m, n, k, Are, Aim, lda, psA, Bre, Bim, ldb, psB, Cre, Cim, ldc, psC, ws, s);
        case MPX_TD: return cgemm_t<double, 3>(prec, m, n, k, Are, Aim, lda, psA, Bre, Bim, ldb, psB, Cre, Cim, ldc, psC, ws, s);
        case MPX_QD: return cgemm_t<double, 4>(prec, m, n, k, Are, Aim, lda, psA, Bre, Bim, ldb, psB, Cre, Cim, ldc, psC, ws, s);
        default: return cgemm_t<float, 2>(prec, m, n, k, Are, Aim, lda, psA, Bre, Bim, ldb, psB, Cre, Cim, ldc, psC, ws, s);
    }
}
