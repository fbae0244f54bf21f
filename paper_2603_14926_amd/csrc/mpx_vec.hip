// mpx_vec.hip -- vector layer of libmpx on gfx950: elementwise BF add / mul,
// AXPY, dot product and GEMV over component planes (Section 3 uses these
// BF operations inside its linear kernels).
//
// All of these are memory-bound at large sizes (QD AXPY: 209 FP64 operations
// per 96 bytes, below the MI355X balance of ~4.9 operations per byte), so
// the kernels are written for coalescing: consecutive lanes touch
// consecutive elements of each component plane, every plane load is a
// 512-byte wave-wide transaction, and each thread keeps several elements in
// flight.  Reductions (dot, GEMV) are deterministic: per-thread sequential
// BF multiply-adds, then a fixed butterfly across the 64 lanes of a wave,
// then a fixed sequential combine across waves and blocks.
#include "mp_arith.hpp"
#include "mp_conv.hpp"
#include "mpx_internal.hpp"

#include <mutex>

namespace mpx {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

// Streaming access to data touched once per call (the vectors of the
// elementwise ops, AXPY and dot, the matrix of GEMV): nontemporal loads and
// stores, which streamed 3-16 % faster on MI355X at n = 2^24 .. 2^26 than
// plain ones.  The values are the same; only the cache policy differs.
template <typename T, int K>
__device__ __forceinline__ mpn<T, K> mp_load_stream(const T* base, long long ps, long long idx) {
    mpn<T, K> r;
#pragma unroll
    for (int i = 0; i < K; ++i) r.c[i] = __builtin_nontemporal_load(&base[i * ps + idx]);
    return r;
}

template <typename T, int K>
__device__ __forceinline__ void mp_store_stream(T* base, long long ps, long long idx,
                                                const mpn<T, K>& v) {
#pragma unroll
    for (int i = 0; i < K; ++i) __builtin_nontemporal_store(v.c[i], &base[i * ps + idx]);
}

// ------------------------------------------------------------ elementwise --

// AR selects the branch-free (0) or conventional (1, 2) operations.
template <typename T, int K, int OP, int AR>
__global__ void __launch_bounds__(kBlock)
k_elementwise(long long n, const T* x, long long psx, const T* y, long long psy, T* z,
              long long psz) {
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const mpn<T, K> a = mp_load_stream<T, K>(x, psx, i);
        const mpn<T, K> b = mp_load_stream<T, K>(y, psy, i);
        mpn<T, K> c;
        if constexpr (OP == 0) c = ar_add<AR>(a, b);
        else c = ar_mul<AR>(a, b);
        mp_store_stream<T, K>(z, psz, i, c);
    }
}

template <typename T, int K, int AR>
__global__ void __launch_bounds__(kBlock)
k_axpy(long long n, mpn<T, K> alpha, const T* __restrict__ x, long long psx, T* y,
       long long psy) {
    const long long stride = (long long)gridDim.x * kBlock;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
        const mpn<T, K> a = mp_load_stream<T, K>(x, psx, i);
        const mpn<T, K> b = mp_load_stream<T, K>(y, psy, i);
        mp_store_stream<T, K>(y, psy, i, ar_add<AR>(ar_mul<AR>(alpha, a), b));
    }
}

static int elementwise_blocks(long long n) {
    long long b = ceil_div(n, kBlock);
    // one element per thread up to 2^28 threads (grid-stride beyond): on
    // MI355X a 65536-block launch streams 8-15 % faster at n = 2^24 than a
    // grid-stride launch capped at 8192 blocks
    if (b > (1LL << 20)) b = 1LL << 20;
    return (int)(b < 1 ? 1 : b);
}

template <typename T, int K, int AR>
static int launch_elementwise(int op, long long n, const void* x, long long psx, const void* y,
                              long long psy, void* z, long long psz, hipStream_t s) {
    const int blocks = elementwise_blocks(n);
    if (op == 0)
        k_elementwise<T, K, 0, AR><<<blocks, kBlock, 0, s>>>(n, (const T*)x, psx, (const T*)y, psy,
                                                          (T*)z, psz);
    else
        k_elementwise<T, K, 1, AR><<<blocks, kBlock, 0, s>>>(n, (const T*)x, psx, (const T*)y, psy,
                                                          (T*)z, psz);
    return launch_status();
}

// -------------------------------------------------------- block reduction --

// Butterfly across the 64 lanes of a wave: every lane ends with the same sum
// (BF addition and the conventional additions are bitwise commutative, so
// partners compute identical bits).
template <typename T, int K, int AR = AR_BF>
__device__ __forceinline__ mpn<T, K> wave_sum(mpn<T, K> v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = ar_add<AR>(v, mp_shfl_xor<T, K>(v, off));
    return v;
}

// Sum over a 256-thread block: wave butterflies, then the four wave sums
// pairwise, (w0 + w1) + (w2 + w3).  Result valid in thread 0.
template <typename T, int K, int AR>
__device__ __forceinline__ mpn<T, K> block_sum(mpn<T, K> v) {
    __shared__ T sh[K][kWaves];
    v = wave_sum<T, K, AR>(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < K; ++c) sh[c][w] = v.c[c];
    }
    __syncthreads();
    mpn<T, K> t[kWaves];
#pragma unroll
    for (int j = 0; j < kWaves; ++j)
#pragma unroll
        for (int c = 0; c < K; ++c) t[j].c[c] = sh[c][j];
#pragma unroll
    for (int step = 1; step < kWaves; step *= 2)
#pragma unroll
        for (int j = 0; j + step < kWaves; j += 2 * step) t[j] = ar_add<AR>(t[j], t[j + step]);
    return t[0];
}

// ------------------------------------------------------------------- dot --

// Stage 1: block b owns a grid-strided subset of the elements; each thread
// accumulates its elements sequentially; the block sum goes to part[b]
// (K planes of nblocks values) or, for a single block, straight to `out`.
template <typename T, int K, int AR>
__global__ void __launch_bounds__(kBlock)
k_dot_partial(long long n, const T* __restrict__ x, long long psx, const T* __restrict__ y,
              long long psy, T* __restrict__ out, long long pso) {
    const long long stride = (long long)gridDim.x * kBlock;
    long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
    // the first product starts the sum (no addition to zero on the chain)
    mpn<T, K> acc = mp_zero<T, K>();
    if (i < n) acc = ar_mul<AR>(mp_load_stream<T, K>(x, psx, i), mp_load_stream<T, K>(y, psy, i));
    for (i += stride; i < n; i += stride)
        acc = ar_add<AR>(acc, ar_mul<AR>(mp_load_stream<T, K>(x, psx, i),
                                         mp_load_stream<T, K>(y, psy, i)));
    acc = block_sum<T, K, AR>(acc);
    if (threadIdx.x == 0) mp_store<T, K>(out, pso, blockIdx.x, acc);
}

// Stage 2 for more than 64 partials: one block adds the nparts partials
// (thread-sequential, then the block tree) into K contiguous values.
template <typename T, int K, int AR>
__global__ void __launch_bounds__(kBlock)
k_sum_parts(long long nparts, const T* __restrict__ part, long long psp, T* __restrict__ out) {
    mpn<T, K> acc = mp_zero<T, K>();
    if (threadIdx.x < nparts) acc = mp_load<T, K>(part, psp, threadIdx.x);
    for (long long i = threadIdx.x + kBlock; i < nparts; i += kBlock)
        acc = ar_add<AR>(acc, mp_load<T, K>(part, psp, i));
    acc = block_sum<T, K, AR>(acc);
    if (threadIdx.x == 0) mp_store<T, K>(out, 1, 0, acc);
}

// Stage 2 for at most 64 partials: one wave, lane l holding partial l (zero
// beyond), a butterfly over the smallest power of two `width` >= nparts
// lanes (log2(width) dependent additions instead of the block tree's ten).
template <typename T, int K, int AR>
__global__ void __launch_bounds__(64)
k_sum_parts_wave(long long nparts, int width, const T* __restrict__ part, long long psp,
                 T* __restrict__ out) {
    const int lane = threadIdx.x;
    mpn<T, K> v = lane < nparts ? mp_load<T, K>(part, psp, lane) : mp_zero<T, K>();
    for (int off = width / 2; off >= 1; off >>= 1) v = ar_add<AR>(v, mp_shfl_xor<T, K>(v, off));
    if (lane == 0) mp_store<T, K>(out, 1, 0, v);
}

// Number of stage-1 blocks: a function of n alone (the summation tree, and so
// the rounding, depends on it).  Up to one block's worth of elements uses one
// block and no stage 2; up to 64 Ki elements, one element per thread (the
// dependent multiply-add chain per thread is what bounds small dots); beyond,
// four or more per thread.
static long long dot_blocks(long long n) {
    if (n <= kBlock) return 1;
    if (n <= 256LL * kBlock) return ceil_div(n, kBlock);
    long long b = ceil_div(n, 4LL * kBlock);
    return b > 1024 ? 1024 : b;  // 1024 partials stream faster than 2048 or more
}

template <typename T, int K, int AR>
static int launch_dot(long long n, const void* x, long long psx, const void* y, long long psy,
                      void* result, void* ws, hipStream_t s) {
    const long long nb = dot_blocks(n);
    if (nb == 1) {
        k_dot_partial<T, K, AR><<<1, kBlock, 0, s>>>(n, (const T*)x, psx, (const T*)y, psy,
                                                  (T*)result, 1);
        return launch_status();
    }
    k_dot_partial<T, K, AR><<<(int)nb, kBlock, 0, s>>>(n, (const T*)x, psx, (const T*)y, psy,
                                                    (T*)ws, nb);
    int st = launch_status();
    if (st != MPX_OK) return st;
    if (nb <= 64) {
        int width = 1;
        while (width < nb) width *= 2;
        k_sum_parts_wave<T, K, AR><<<1, 64, 0, s>>>(nb, width, (const T*)ws, nb, (T*)result);
    } else {
        k_sum_parts<T, K, AR><<<1, kBlock, 0, s>>>(nb, (const T*)ws, nb, (T*)result);
    }
    return launch_status();
}

// ------------------------------------------------------------------ GEMV --

// y = A x, A m x n row-major.  A wave owns R consecutive rows and one column
// chunk; lane l walks columns c0 + l, c0 + l + 64, ... sequentially with R
// accumulators, reusing each x_j for its R rows; the wave butterfly then sums
// the 64 lane partials of each row.
constexpr int kGemvRows = 4;

template <typename T, int K, int R>
__global__ void __launch_bounds__(kBlock)
k_gemv_n(long long m, long long n, const T* __restrict__ A, long long lda, long long psA,
         const T* __restrict__ x, long long psx, T* __restrict__ out, long long pso,
         long long chunk) {
    constexpr int U = 2;  // columns per lane whose loads are issued together
    const int lane = threadIdx.x & 63;
    const long long wave = (long long)blockIdx.x * kWaves + (threadIdx.x >> 6);
    const long long r0 = wave * R;
    if (r0 >= m) return;  // whole wave leaves together (no block barrier below)
    const long long c0 = (long long)blockIdx.y * chunk;
    const long long c1 = c0 + chunk < n ? c0 + chunk : n;
    long long rows[R];
#pragma unroll
    for (int r = 0; r < R; ++r) rows[r] = r0 + r < m ? r0 + r : m - 1;  // clamped, unused
    mpn<T, K> acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = mp_zero<T, K>();
    long long j = c0 + lane;
    // full groups: U columns per lane, all loads first, then the
    // multiply-adds in ascending column order
    for (; j + 64 * (U - 1) < c1; j += 64 * U) {
        mpn<T, K> xv[U], av[U][R];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            xv[u] = mp_load<T, K>(x, psx, j + 64 * u);
#pragma unroll
            for (int r = 0; r < R; ++r)
                av[u][r] = mp_load_stream<T, K>(A, psA, rows[r] * lda + j + 64 * u);
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] = bf_add(acc[r], bf_mul(av[u][r], xv[u]));
    }
    for (; j < c1; j += 64) {
        const mpn<T, K> xv = mp_load<T, K>(x, psx, j);
#pragma unroll
        for (int r = 0; r < R; ++r)
            acc[r] = bf_add(acc[r], bf_mul(mp_load_stream<T, K>(A, psA, rows[r] * lda + j), xv));
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const mpn<T, K> sum = wave_sum<T, K>(acc[r]);
        if (lane == 0 && r0 + r < m) mp_store<T, K>(out, pso, blockIdx.y * m + r0 + r, sum);
    }
}

// y = A^T x: thread t owns column j and walks rows i0 .. i1-1 sequentially
// (coalesced across the wave, x_i broadcast).
template <typename T, int K>
__global__ void __launch_bounds__(kBlock)
k_gemv_t(long long m, long long n, const T* __restrict__ A, long long lda, long long psA,
         const T* __restrict__ x, long long psx, T* __restrict__ out, long long pso,
         long long chunk) {
    const long long j = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const long long i0 = (long long)blockIdx.y * chunk;
    const long long i1 = i0 + chunk < m ? i0 + chunk : m;
    mpn<T, K> acc = mp_zero<T, K>();
    for (long long i = i0; i < i1; ++i)
        acc = bf_add(acc, bf_mul(mp_load_stream<T, K>(A, psA, i * lda + j), mp_load<T, K>(x, psx, i)));
    mp_store<T, K>(out, pso, blockIdx.y * n + j, acc);
}

// Combine split partials part[s*rows + r] in split order.
template <typename T, int K>
__global__ void __launch_bounds__(kBlock)
k_gemv_combine(long long rows, long long splits, const T* __restrict__ part, long long psp,
               T* __restrict__ y, long long psy) {
    const long long r = (long long)blockIdx.x * kBlock + threadIdx.x;
    if (r >= rows) return;
    mpn<T, K> acc = mp_load<T, K>(part, psp, r);
    for (long long s = 1; s < splits; ++s) acc = bf_add(acc, mp_load<T, K>(part, psp, s * rows + r));
    mp_store<T, K>(y, psy, r, acc);
}

struct GemvPlan {
    long long splits, chunk, rows;
};

// Split of the reduction dimension: enough waves to fill 256 CUs at ~4 waves
// per SIMD, each split at least 256 long.  A function of the shape only.
static GemvPlan gemv_plan(int trans, long long m, long long n) {
    GemvPlan p;
    const long long len = trans ? m : n;
    p.rows = trans ? n : m;
    long long units = trans ? ceil_div(n, 64) : ceil_div(m, kGemvRows);  // waves per split
    long long splits = units >= 4096 ? 1 : ceil_div(4096, units);
    long long maxs = ceil_div(len, 256);
    if (splits > maxs) splits = maxs;
    if (splits < 1) splits = 1;
    p.chunk = ceil_div(len, splits);
    p.splits = len == 0 ? 1 : ceil_div(len, p.chunk);
    return p;
}

template <typename T, int K>
static int launch_gemv(int trans, long long m, long long n, const void* A, long long lda,
                       long long psA, const void* x, long long psx, void* y, long long psy,
                       void* ws, hipStream_t s) {
    const GemvPlan p = gemv_plan(trans, m, n);
    if (p.rows == 0) return MPX_OK;
    T* out = p.splits == 1 ? (T*)y : (T*)ws;
    const long long pso = p.splits == 1 ? psy : p.splits * p.rows;
    if (!trans) {
        dim3 grid((unsigned)ceil_div(ceil_div(m, kGemvRows), kWaves), (unsigned)p.splits);
        k_gemv_n<T, K, kGemvRows><<<grid, kBlock, 0, s>>>(m, n, (const T*)A, lda, psA,
                                                           (const T*)x, psx, out, pso, p.chunk);
    } else {
        dim3 grid((unsigned)ceil_div(n, kBlock), (unsigned)p.splits);
        k_gemv_t<T, K><<<grid, kBlock, 0, s>>>(m, n, (const T*)A, lda, psA, (const T*)x, psx, out,
                                               pso, p.chunk);
    }
    int st = launch_status();
    if (st != MPX_OK || p.splits == 1) return st;
    k_gemv_combine<T, K><<<(unsigned)ceil_div(p.rows, kBlock), kBlock, 0, s>>>(
        p.rows, p.splits, (const T*)ws, pso, (T*)y, psy);
    return launch_status();
}

size_t gemv_workspace(int prec, long long m, long long n, int trans) {
    const GemvPlan p = gemv_plan(trans, m, n);
    if (p.splits == 1) return 0;
    const size_t elt = is_ff(prec) ? sizeof(float) : sizeof(double);
    return elt * (size_t)prec_k(prec) * (size_t)(p.splits * p.rows);
}

size_t dot_workspace(int prec, long long n) {
    const long long nb = dot_blocks(n);
    if (nb == 1) return 0;
    const size_t elt = is_ff(base_prec(prec)) ? sizeof(float) : sizeof(double);
    return elt * (size_t)prec_k_ar(prec) * (size_t)nb;
}

}  // namespace mpx

using namespace mpx;

// ---------------------------------------------------------------- C ABI ----

#define MPX_DISPATCH(prec, FN, ...)                                        \
    switch (prec) {                                                        \
        case MPX_DD: return FN<double, 2>(__VA_ARGS__);                    \
        case MPX_TD: return FN<double, 3>(__VA_ARGS__);                    \
        case MPX_QD: return FN<double, 4>(__VA_ARGS__);                    \
        case MPX_FF: return FN<float, 2>(__VA_ARGS__);                     \
        default: return MPX_EPREC;                                         \
    }

// The same with the arithmetic flag as the last template argument.
#define MPX_DISPATCH_AR(prec, FN, ...)                                                  \
    switch (prec) {                                                                     \
        case MPX_DD: return FN<double, 2, AR_BF>(__VA_ARGS__);                          \
        case MPX_TD: return FN<double, 3, AR_BF>(__VA_ARGS__);                          \
        case MPX_QD: return FN<double, 4, AR_BF>(__VA_ARGS__);                          \
        case MPX_FF: return FN<float, 2, AR_BF>(__VA_ARGS__);                           \
        case MPX_DD | MPX_NOBF: return FN<double, 2, AR_NOBF>(__VA_ARGS__);             \
        case MPX_TD | MPX_NOBF: return FN<double, 3, AR_NOBF>(__VA_ARGS__);             \
        case MPX_QD | MPX_NOBF: return FN<double, 4, AR_NOBF>(__VA_ARGS__);             \
        case MPX_DD | MPX_NOBF_ACC: return FN<double, 2, AR_NOBF_ACC>(__VA_ARGS__);     \
        default: return MPX_EPREC;                                                      \
    }

// Vector operand check; accepts the arithmetic flags (GEMV rejects them
// before calling this).
static int check_vec(int prec, int64_t n, const void* p, int64_t ps) {
    if (!prec_k_ar(prec)) return MPX_EPREC;
    if (n < 0) return MPX_EINVAL;
    if (n > 0 && (p == nullptr || ps < n)) return MPX_EINVAL;
    return MPX_OK;
}

static int elementwise(int op, int prec, int64_t n, const void* x, int64_t psx, const void* y,
                       int64_t psy, void* z, int64_t psz, void* stream) {
    int st;
    if ((st = check_vec(prec, n, x, psx)) || (st = check_vec(prec, n, y, psy)) ||
        (st = check_vec(prec, n, z, psz)))
        return st;
    if (n == 0) return MPX_OK;
    MPX_DISPATCH_AR(prec, launch_elementwise, op, n, x, psx, y, psy, z, psz, as_stream(stream));
}

extern "C" int mpx_add(int prec, int64_t n, const void* x, int64_t psx, const void* y,
                       int64_t psy, void* z, int64_t psz, void* stream) {
    return elementwise(0, prec, n, x, psx, y, psy, z, psz, stream);
}

extern "C" int mpx_mul(int prec, int64_t n, const void* x, int64_t psx, const void* y,
                       int64_t psy, void* z, int64_t psz, void* stream) {
    return elementwise(1, prec, n, x, psx, y, psy, z, psz, stream);
}

template <typename T, int K, int AR>
static int axpy_t(int64_t n, const void* alpha_host, const void* x, int64_t psx, void* y,
                  int64_t psy, hipStream_t s) {
    mpn<T, K> a;
    for (int c = 0; c < K; ++c) a.c[c] = ((const T*)alpha_host)[c];
    k_axpy<T, K, AR><<<elementwise_blocks(n), kBlock, 0, s>>>(n, a, (const T*)x, psx, (T*)y, psy);
    return launch_status();
}

extern "C" int mpx_axpy(int prec, int64_t n, const void* alpha_host, const void* x,
                        int64_t psx, void* y, int64_t psy, void* stream) {
    int st;
    if ((st = check_vec(prec, n, x, psx)) || (st = check_vec(prec, n, y, psy))) return st;
    if (alpha_host == nullptr) return MPX_EINVAL;
    if (n == 0) return MPX_OK;
    MPX_DISPATCH_AR(prec, axpy_t, n, alpha_host, x, psx, y, psy, as_stream(stream));
}

extern "C" int mpx_dot(int prec, int64_t n, const void* x, int64_t psx, const void* y,
                       int64_t psy, void* result, void* ws, size_t ws_bytes, void* stream) {
    int st;
    if ((st = check_vec(prec, n, x, psx)) || (st = check_vec(prec, n, y, psy))) return st;
    if (result == nullptr) return MPX_EINVAL;
    const size_t need = dot_workspace(prec, n);
    if (need > 0 && (ws == nullptr || ws_bytes < need)) return MPX_EWORKSPACE;
    // neither the result nor the workspace may overlap an input or each other
    const int K = prec_k_ar(prec);
    const size_t elt = is_ff(base_prec(prec)) ? sizeof(float) : sizeof(double);
    const uint64_t xb = planes_bytes(K, 1, n, n, psx, elt), yb = planes_bytes(K, 1, n, n, psy, elt);
    const uint64_t rb = (uint64_t)K * elt;
    if (overlaps(result, rb, x, xb) || overlaps(result, rb, y, yb) || overlaps(ws, need, x, xb) ||
        overlaps(ws, need, y, yb) || overlaps(ws, need, result, rb))
        return MPX_EINVAL;
    MPX_DISPATCH_AR(prec, launch_dot, n, x, psx, y, psy, result, ws, as_stream(stream));
}

// ------------------------------------------------- allocation-free dot ----
//
// mpx_dot_noalloc keeps the multi-block dot's block partials in this
// file-scope array instead of a caller workspace: up to 1024 partials of up
// to four binary64 components (every multi-block dot fits), 32 KiB held by
// each GPU the library runs on until the process ends.  Every partial is
// written by the first kernel before the second reads it, so nothing needs
// clearing.  Host code never uses the array's name as an address: the
// per-device address comes from hipGetSymbolAddress, taken once per device
// with that device current.
constexpr size_t kDotScratchBytes = 4 * sizeof(double) * 1024;
static __device__ __align__(256) unsigned char scratch[kDotScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device.
static int scratch_address(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return MPX_EDEVICE;
    if (dev < 0 || dev >= kMaxDevices) return MPX_ENOTSUP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
            return MPX_EDEVICE;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MPX_OK;
}

extern "C" int mpx_dot_noalloc(int prec, int64_t n, const void* x, int64_t psx, const void* y,
                               int64_t psy, void* result, void* stream) {
    int st;
    if ((st = check_vec(prec, n, x, psx)) || (st = check_vec(prec, n, y, psy))) return st;
    if (result == nullptr) return MPX_EINVAL;
    const size_t need = dot_workspace(prec, n);
    if (need > kDotScratchBytes) return MPX_EWORKSPACE;  // larger than the static scratch
    const int K = prec_k_ar(prec);
    const size_t elt = is_ff(base_prec(prec)) ? sizeof(float) : sizeof(double);
    const uint64_t xb = planes_bytes(K, 1, n, n, psx, elt), yb = planes_bytes(K, 1, n, n, psy, elt);
    const uint64_t rb = (uint64_t)K * elt;
    if (overlaps(result, rb, x, xb) || overlaps(result, rb, y, yb)) return MPX_EINVAL;
    void* ws = nullptr;
    if (need > 0 && (st = scratch_address(&ws)) != MPX_OK) return st;
    MPX_DISPATCH_AR(prec, launch_dot, n, x, psx, y, psy, result, ws, as_stream(stream));
}

extern "C" int mpx_gemv(int prec, int trans, int64_t m, int64_t n, const void* A, int64_t lda,
                        int64_t psA, const void* x, int64_t psx, void* y, int64_t psy, void* ws,
                        size_t ws_bytes, void* stream) {
    if (!prec_k(prec)) return MPX_EPREC;
    if (m < 0 || n < 0 || (trans != 0 && trans != 1)) return MPX_EINVAL;
    if (m > INT32_MAX || n > INT32_MAX) return MPX_ENOTSUP;  // grid dimensions
    const int64_t xlen = trans ? m : n, ylen = trans ? n : m;
    if (m > 0 && n > 0 && (A == nullptr || !span_fits(m, n, lda, psA))) return MPX_EINVAL;
    int st;
    if ((st = check_vec(prec, xlen, x, psx)) || (st = check_vec(prec, ylen, y, psy))) return st;
    // y must not overlap A or x, nor the workspace any of them
    const int K = prec_k(prec);
    const size_t elt = is_ff(prec) ? sizeof(float) : sizeof(double);
    const uint64_t ab = planes_bytes(K, m, n, lda, psA, elt);
    const uint64_t xb = planes_bytes(K, 1, xlen, xlen, psx, elt), yb = planes_bytes(K, 1, ylen, ylen, psy, elt);
    if (overlaps(y, yb, A, ab) || overlaps(y, yb, x, xb)) return MPX_EINVAL;
    if (ylen == 0) return MPX_OK;
    const size_t need = gemv_workspace(prec, m, n, trans);
    if (need > 0 && (ws == nullptr || ws_bytes < need)) return MPX_EWORKSPACE;
    if (overlaps(ws, need, A, ab) || overlaps(ws, need, x, xb) || overlaps(ws, need, y, yb))
        return MPX_EINVAL;
    MPX_DISPATCH(prec, launch_gemv, trans, m, n, A, lda, psA, x, psx, y, psy, ws,
                 as_stream(stream));
}
