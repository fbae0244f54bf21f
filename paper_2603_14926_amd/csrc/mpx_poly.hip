// mpx_poly.hip -- polynomial kernels of libmpx on gfx950:
//   * real Horner evaluation of a batch of polynomials and its reverse-mode
//     derivative (Section 4.1 evaluates p_n(x) = sum a_i x^i by Horner);
//   * the batched Durand-Kerner (Weierstrass) simultaneous iteration with
//     the Aberth start (Section 4.2), as one persistent kernel.
//
// Durand-Kerner design.  A polynomial of degree n costs ~1672 n FP64 VALU
// instructions per root per iteration in QD (Horner: n complex multiply-adds;
// root-difference product: n-1 complex subtract-multiplies), i.e. O(n^2) per
// iteration, all VALU.  One wave64 owns one polynomial at a time: lane l
// updates roots l, l+64, ... (R of them interleaved for instruction-level
// parallelism), reading the wave-uniform coefficient c_k and root z_j from
// global memory (one cache line per load, broadcast to the 64 lanes).  The
// iterate lives in two ping-pong buffers (the caller's roots and a plan-owned
// copy); a workgroup barrier between iterations makes every update of
// iterate t visible before iterate t+1 is read (Jacobi, as in the DK
// equation: all new roots come from the previous iterate).  Waves take
// polynomials from a longest-processing-time order (descending n^2) through
// an atomic counter, so thousands of ragged degrees load-balance in one
// launch.
//
// Overflow: Horner values grow like |z|^n (random degree-512 polynomials
// start at |z| ~ 10^2), beyond binary64.  Values are therefore kept as
// (mantissa, 2^E) with exact power-of-two rescaling after each step: the
// Horner value is scaled down whenever its larger leading component reaches
// 1 (the coefficient term is added as c_k 2^-E); the root-difference product
// is rescaled to [0.5, 1) after every factor; the correction is
// q/P * 2^(E - F).  Power-of-two scaling commutes with rounding, so this only
// changes behaviour where the unscaled computation would overflow.
//
// Every per-root operation sequence equals the sequential definition (Horner
// from the leading coefficient, j ascending in the product, Newton reciprocal
// for the division), so results are bit-identical for every launch shape.
#include "mp_arith.hpp"
#include "mp_conv.hpp"
#include "mpx_internal.hpp"
#include "dk_sched.hpp"

#include <algorithm>
#include <string>
#include <thread>
#include <cstdlib>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <map>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

namespace mpx {

// ------------------------------------------------------- real Horner ----

// y_b = p_b(x_b): h = a_deg; h := h * x + a_i (i = deg-1 .. 0).  One thread
// per polynomial; coefficients for the next steps are loaded ahead of the
// dependent multiply-add chain.  AR selects branch-free (0) or conventional
// (1) operations (Section 4.1 compares the two).
template <int K, int AR>
__global__ void __launch_bounds__(64)
k_polyval(long long batch, long long deg, const double* __restrict__ coef, long long psc,
          const double* __restrict__ x, long long psx, double* __restrict__ y, long long psy) {
    using V = mpn<double, K>;
    const long long b = (long long)blockIdx.x * 64 + threadIdx.x;
    if (b >= batch) return;
    const long long off = b * (deg + 1);
    const V xv = mp_load<double, K>(x, psx, b);
    V h = mp_load<double, K>(coef, psc, off + deg);
    long long i = deg - 1;
    for (; i >= 3; i -= 4) {
        const V a0 = mp_load<double, K>(coef, psc, off + i);
        const V a1 = mp_load<double, K>(coef, psc, off + i - 1);
        const V a2 = mp_load<double, K>(coef, psc, off + i - 2);
        const V a3 = mp_load<double, K>(coef, psc, off + i - 3);
        h = ar_add<AR>(ar_mul<AR>(h, xv), a0);
        h = ar_add<AR>(ar_mul<AR>(h, xv), a1);
        h = ar_add<AR>(ar_mul<AR>(h, xv), a2);
        h = ar_add<AR>(ar_mul<AR>(h, xv), a3);
    }
    for (; i >= 0; --i) h = ar_add<AR>(ar_mul<AR>(h, xv), mp_load<double, K>(coef, psc, off + i));
    mp_store<double, K>(y, psy, b, h);
}

// Estrin's method (Section 4.1 compares it with Horner), one wave per
// polynomial.  The coefficients are padded with zeros to N = 2^L; level l
// replaces the list c by c'_j = c_{2j} + c_{2j+1} X_{l-1} (X_0 = x,
// X_l = X_{l-1}^2).  Lane t owns the aligned block of B = 2^LB coefficients
// starting at t*B (B = 1 when N <= 64): the first LB levels stay inside the
// lane and are evaluated as a binary counter (a stack of one pending value
// per level, fully unrolled), the remaining L - LB levels combine lanes t and
// t + s with a shuffle.  The dependent chain is B + log2(N/B) steps instead
// of Horner's N, for the same operation count.
constexpr int trailing_ones(int t) { return (t & 1) ? 1 + trailing_ones(t >> 1) : 0; }

// One step of the lane-local binary counter, unrolled at compile time for
// every position T of the lane's block: position T completes levels
// 1..trailing_ones(T) (each c_even + c_odd X_{l-1}), then parks its value.
template <int K, int LB, int T>
struct EstrinLocal {
    static __device__ __forceinline__ void run(mpn<double, K>* st, const mpn<double, K>* Xl,
                                               const double* __restrict__ coef, long long psc,
                                               long long base, long long deg, long long off) {
        constexpr int tz = trailing_ones(T);
        const long long i = base + T;
        mpn<double, K> cur = i <= deg ? mp_load<double, K>(coef, psc, off + i) : mp_zero<double, K>();
#pragma unroll
        for (int l = 0; l < tz; ++l) cur = bf_add(st[l], bf_mul(cur, Xl[l]));
        st[tz] = cur;
        // issue loads eight coefficients at a time (register pressure)
        if constexpr ((T & 7) == 7) asm volatile("" ::: "memory");
        EstrinLocal<K, LB, T + 1>::run(st, Xl, coef, psc, base, deg, off);
    }
};
template <int K, int LB>
struct EstrinLocal<K, LB, (1 << LB)> {
    static __device__ __forceinline__ void run(mpn<double, K>*, const mpn<double, K>*,
                                               const double* __restrict__, long long, long long,
                                               long long, long long) {}
};

template <int K, int LB>
__global__ void __launch_bounds__(256)
k_estrin(long long batch, long long deg, int L, const double* __restrict__ coef, long long psc,
         const double* __restrict__ x, long long psx, double* __restrict__ y, long long psy) {
    using V = mpn<double, K>;
    constexpr int B = 1 << LB;
    const long long b = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= batch) return;  // whole wave
    const long long off = b * (deg + 1);
    V st[LB + 1];
    V Xl[LB + 1];
    Xl[0] = mp_load<double, K>(x, psx, b);
#pragma unroll
    for (int l = 1; l <= LB; ++l) Xl[l] = bf_mul(Xl[l - 1], Xl[l - 1]);
    EstrinLocal<K, LB, 0>::run(st, Xl, coef, psc, (long long)lane * B, deg, off);
    V c = st[LB];
    V Xc = Xl[LB];
    // cross-lane levels
    for (int lev = LB; lev < L; ++lev) {
        const int sft = 1 << (lev - LB);
        V other;
#pragma unroll
        for (int q = 0; q < K; ++q) other.c[q] = __shfl_down(c.c[q], sft, 64);
        const V comb = bf_add(c, bf_mul(other, Xc));
        const bool leader = (lane & (2 * sft - 1)) == 0;
#pragma unroll
        for (int q = 0; q < K; ++q) c.c[q] = leader ? comb.c[q] : c.c[q];
        Xc = bf_mul(Xc, Xc);
    }
    if (lane == 0) mp_store<double, K>(y, psy, b, c);
}

// Estrin for the long lists (N = 2^L, L = LB + 8): one 256-thread workgroup
// per polynomial, so a lane still holds at most 2^LB <= 32 coefficients.
// Thread t owns the block of B = 2^LB coefficients from t B; levels 1..LB
// run lane-locally as above, the next six across the lanes of each wave,
// and the last two combine the four waves' values (waves 0..3 hold the
// level LB + 6 entries 0..3) through LDS in the same pairing order.
template <int K, int LB>
__global__ void __launch_bounds__(256)
k_estrin_wg(long long deg, const double* __restrict__ coef, long long psc,
            const double* __restrict__ x, long long psx, double* __restrict__ y, long long psy) {
    using V = mpn<double, K>;
    constexpr int B = 1 << LB;
    const long long b = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const long long off = b * (deg + 1);
    __shared__ double s_top[4][K];
    V st[LB + 1];
    V Xl[LB + 1];
    Xl[0] = mp_load<double, K>(x, psx, b);
#pragma unroll
    for (int l = 1; l <= LB; ++l) Xl[l] = bf_mul(Xl[l - 1], Xl[l - 1]);
    EstrinLocal<K, LB, 0>::run(st, Xl, coef, psc, (long long)threadIdx.x * B, deg, off);
    V c = st[LB];
    V Xc = Xl[LB];
#pragma unroll
    for (int lev = 0; lev < 6; ++lev) {
        const int sft = 1 << lev;
        V other;
#pragma unroll
        for (int q = 0; q < K; ++q) other.c[q] = __shfl_down(c.c[q], sft, 64);
        const V comb = bf_add(c, bf_mul(other, Xc));
        const bool leader = (lane & (2 * sft - 1)) == 0;
#pragma unroll
        for (int q = 0; q < K; ++q) c.c[q] = leader ? comb.c[q] : c.c[q];
        Xc = bf_mul(Xc, Xc);
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < K; ++q) s_top[wv][q] = c.c[q];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        V v[4];
#pragma unroll
        for (int w = 0; w < 4; ++w)
#pragma unroll
            for (int q = 0; q < K; ++q) v[w].c[q] = s_top[w][q];
        const V lo = bf_add(v[0], bf_mul(v[1], Xc));
        const V hi = bf_add(v[2], bf_mul(v[3], Xc));
        Xc = bf_mul(Xc, Xc);
        mp_store<double, K>(y, psy, b, bf_add(lo, bf_mul(hi, Xc)));
    }
}

// Gradients of L = sum_b g_b p_b(x_b):
//   dL/da_{b,i} = t_i with t_0 = g_b, t_{i+1} = t_i * x_b   (adjoint of Horner)
//   dL/dx_b     = g_b * d, d from  d := d * x + h  before  h := h * x + a_i
// (d = 0, h = a_deg initially).  Either output may be null.
//
// The chains run in separate waves, 128-thread blocks, one polynomial per
// lane.  Coefficient blocks (the first ncb blocks when gcoef is requested):
// both waves run t-chains for 128 polynomials.  x blocks: 64 polynomials;
// wave 0 runs the Horner chain h and hands every pre-update h to wave 1
// through LDS, wave 1 runs the d chain on them, one chunk of kBwdChunk
// steps behind (double-buffered, a barrier per chunk), so the x gradient
// costs about one Horner pass instead of two.
constexpr int kBwdChunk = 8;

template <int K>
__global__ void __launch_bounds__(128)
k_polyval_bwd(long long batch, long long deg, const double* __restrict__ coef, long long psc,
              const double* __restrict__ x, long long psx, const double* __restrict__ g,
              long long psg, double* __restrict__ gcoef, long long psgc,
              double* __restrict__ gx, long long psgx, unsigned ncb) {
    using V = mpn<double, K>;
    if (blockIdx.x < ncb) {  // coefficient gradients
        const long long b = (long long)blockIdx.x * 128 + threadIdx.x;
        if (b >= batch) return;
        const long long off = b * (deg + 1);
        const V xv = mp_load<double, K>(x, psx, b);
        V t = mp_load<double, K>(g, psg, b);
        mp_store<double, K>(gcoef, psgc, off, t);
        for (long long i = 1; i <= deg; ++i) {
            t = bf_mul(t, xv);
            mp_store<double, K>(gcoef, psgc, off + i, t);
        }
        return;
    }
    // x gradients; the whole block stays to the end (it meets every barrier)
    __shared__ double hbuf[2][kBwdChunk][K][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const long long b = (long long)(blockIdx.x - ncb) * 64 + lane;
    const bool live = b < batch;
    const long long bb = live ? b : 0;
    const long long off = bb * (deg + 1);
    const V xv = mp_load<double, K>(x, psx, bb);
    const long long nch = (deg + kBwdChunk - 1) / kBwdChunk;  // chunks of steps
    V h = mp_load<double, K>(coef, psc, off + deg);           // wave 0's Horner value
    V d = mp_zero<double, K>();                               // wave 1's derivative
    for (long long t = 0; t <= nch; ++t) {
        if (wv == 0 && t < nch) {  // steps t C .. t C + C - 1 (i = deg - 1 - step)
            const long long s0 = t * kBwdChunk;
            const int cnt = (int)(deg - s0 < kBwdChunk ? deg - s0 : kBwdChunk);
            for (int j = 0; j < cnt; ++j) {
#pragma unroll
                for (int c = 0; c < K; ++c) hbuf[t & 1][j][c][lane] = h.c[c];
                h = bf_add(bf_mul(h, xv), mp_load<double, K>(coef, psc, off + deg - 1 - s0 - j));
            }
        }
        if (wv == 1 && t > 0) {    // the chunk wave 0 wrote one round earlier
            const long long s0 = (t - 1) * kBwdChunk;
            const int cnt = (int)(deg - s0 < kBwdChunk ? deg - s0 : kBwdChunk);
            for (int j = 0; j < cnt; ++j) {
                V hs;
#pragma unroll
                for (int c = 0; c < K; ++c) hs.c[c] = hbuf[(t - 1) & 1][j][c][lane];
                d = bf_add(bf_mul(d, xv), hs);
            }
        }
        __syncthreads();  // chunk t written before it is read; chunk t-1 read before reuse
    }
    if (wv == 1 && live) mp_store<double, K>(gx, psgx, b, bf_mul(mp_load<double, K>(g, psg, b), d));
}

// ------------------------------------------------- complex arithmetic ----

template <int K>
struct cplx {
    mpn<double, K> re, im;
};

// (a+bi)(c+di): ac - bd, ad + bc (four products, two sums).  AR selects the
// branch-free (0) or conventional (1, 2) real operations.
template <int K, int AR = AR_BF>
__device__ __forceinline__ cplx<K> c_mul(const cplx<K>& x, const cplx<K>& y) {
    const auto ac = ar_mul<AR>(x.re, y.re);
    const auto bd = ar_mul<AR>(x.im, y.im);
    const auto ad = ar_mul<AR>(x.re, y.im);
    const auto bc = ar_mul<AR>(x.im, y.re);
    cplx<K> r;
    r.re = ar_sub<AR>(ac, bd);
    r.im = ar_add<AR>(ad, bc);
    return r;
}
template <int K, int AR = AR_BF>
__device__ __forceinline__ cplx<K> c_add(const cplx<K>& x, const cplx<K>& y) {
    return {ar_add<AR>(x.re, y.re), ar_add<AR>(x.im, y.im)};
}
template <int K, int AR = AR_BF>
__device__ __forceinline__ cplx<K> c_sub(const cplx<K>& x, const cplx<K>& y) {
    return {ar_sub<AR>(x.re, y.re), ar_sub<AR>(x.im, y.im)};
}

// Newton's iteration for 1/d (division through Newton, Section 2): y0 is the
// correctly rounded binary64 1/d_0; each step y := y + y (1 - d y) doubles
// the correct bits (one step for DD, two for TD / QD).
template <int K, int AR = AR_BF>
__device__ __forceinline__ mpn<double, K> mp_recip(const mpn<double, K>& d) {
    const auto one = mp_from<double, K>(1.0);
    auto y = mp_from<double, K>(1.0 / d.c[0]);
    constexpr int steps = K == 2 ? 1 : 2;
#pragma unroll
    for (int s = 0; s < steps; ++s) {
        const auto e = ar_sub<AR>(one, ar_mul<AR>(d, y));
        y = ar_add<AR>(y, ar_mul<AR>(y, e));
    }
    return y;
}

// x / y = (x conj y) (1 / |y|^2).
template <int K, int AR = AR_BF>
__device__ __forceinline__ cplx<K> c_div(const cplx<K>& x, const cplx<K>& y) {
    const auto den = ar_add<AR>(ar_mul<AR>(y.re, y.re), ar_mul<AR>(y.im, y.im));
    const auto inv = mp_recip<K, AR>(den);
    const auto nr = ar_add<AR>(ar_mul<AR>(x.re, y.re), ar_mul<AR>(x.im, y.im));
    const auto ni = ar_sub<AR>(ar_mul<AR>(x.im, y.re), ar_mul<AR>(x.re, y.im));
    return {ar_mul<AR>(nr, inv), ar_mul<AR>(ni, inv)};
}

// Component-wise select (a select on whole aggregates would go through memory).
template <int K>
__device__ __forceinline__ cplx<K> c_select(bool t, const cplx<K>& a, const cplx<K>& b) {
    cplx<K> r;
#pragma unroll
    for (int c = 0; c < K; ++c) {
        r.re.c[c] = t ? a.re.c[c] : b.re.c[c];
        r.im.c[c] = t ? a.im.c[c] : b.im.c[c];
    }
    return r;
}

__device__ __forceinline__ int clamp_exp(long long e) {
    return e > 100000 ? 100000 : (e < -100000 ? -100000 : (int)e);
}

template <int K>
__device__ __forceinline__ cplx<K> c_ldexp(const cplx<K>& x, int e) {
    cplx<K> r;
#pragma unroll
    for (int c = 0; c < K; ++c) {
        r.re.c[c] = __builtin_amdgcn_ldexp(x.re.c[c], e);
        r.im.c[c] = __builtin_amdgcn_ldexp(x.im.c[c], e);
    }
    return r;
}

// Rescale so the larger leading component lies in [0.5, 1) and add the
// exponent to E; with down_only, only magnitudes >= 1 are rescaled.  Zero
// and non-finite values are left alone.  Branch-free: the exponent used is
// zero when no rescaling applies, and ldexp by zero is exact.
template <int K, bool down_only>
__device__ __forceinline__ void c_rescale(cplx<K>& z, long long& E) {
    const double m = fmax(fabs(z.re.c[0]), fabs(z.im.c[0]));
    const int e = __builtin_amdgcn_frexp_exp(m);  // m = f 2^e, 0.5 <= f < 1
    const bool apply = (m != 0.0) && isfinite(m) && (!down_only || e >= 1);
    const int s = apply ? e : 0;
    z = c_ldexp<K>(z, -s);
    E += s;
}

template <int K>
__device__ __forceinline__ cplx<K> c_load(const double* __restrict__ re,
                                          const double* __restrict__ im, long long ps,
                                          long long idx) {
    return {mp_load<double, K>(re, ps, idx), mp_load<double, K>(im, ps, idx)};
}
template <int K>
__device__ __forceinline__ void c_store(double* __restrict__ re, double* __restrict__ im,
                                        long long ps, long long idx, const cplx<K>& v) {
    mp_store<double, K>(re, ps, idx, v.re);
    mp_store<double, K>(im, ps, idx, v.im);
}

// ------------------------------------- real polynomials, complex point ----

// Real-coefficient polynomial at a complex point (Section 4.1's second
// benchmark), Horner: h = (a_n, 0); h := h z + a_i, the product in the 4M
// form and the real coefficient added to the real part only.  One thread per
// polynomial; AR selects branch-free or conventional operations.
template <int K, int AR>
__global__ void __launch_bounds__(64)
k_polyval_cplx(long long batch, long long deg, const double* __restrict__ coef, long long psc,
               const double* __restrict__ xre, const double* __restrict__ xim, long long psx,
               double* __restrict__ yre, double* __restrict__ yim, long long psy) {
    using V = mpn<double, K>;
    const long long b = (long long)blockIdx.x * 64 + threadIdx.x;
    if (b >= batch) return;
    const long long off = b * (deg + 1);
    const cplx<K> z = c_load<K>(xre, xim, psx, b);
    cplx<K> h;
    h.re = mp_load<double, K>(coef, psc, off + deg);
    h.im = mp_zero<double, K>();
    long long i = deg - 1;
    for (; i >= 3; i -= 4) {
        const V a0 = mp_load<double, K>(coef, psc, off + i);
        const V a1 = mp_load<double, K>(coef, psc, off + i - 1);
        const V a2 = mp_load<double, K>(coef, psc, off + i - 2);
        const V a3 = mp_load<double, K>(coef, psc, off + i - 3);
        h = c_mul<K, AR>(h, z); h.re = ar_add<AR>(h.re, a0);
        h = c_mul<K, AR>(h, z); h.re = ar_add<AR>(h.re, a1);
        h = c_mul<K, AR>(h, z); h.re = ar_add<AR>(h.re, a2);
        h = c_mul<K, AR>(h, z); h.re = ar_add<AR>(h.re, a3);
    }
    for (; i >= 0; --i) {
        h = c_mul<K, AR>(h, z);
        h.re = ar_add<AR>(h.re, mp_load<double, K>(coef, psc, off + i));
    }
    c_store<K>(yre, yim, psy, b, h);
}

// Estrin at a complex point: the list halving of the real-argument kernel
// (lane t owns the block of B = 2^LB coefficients from t B; the first LB
// levels run as a lane-local binary counter, the rest across lanes).  The
// first level pairs real coefficients, c' = (a_even + a_odd x_re,
// a_odd x_im); later levels are complex, c' = c_even + c_odd X, and
// X := X^2 after every level.
template <int K, int LB, int T>
struct EstrinCplxLocal {
    static __device__ __forceinline__ void run(mpn<double, K>& st0, cplx<K>* st, const cplx<K>* Xl,
                                               const double* __restrict__ coef, long long psc,
                                               long long base, long long deg, long long off) {
        constexpr int tz = trailing_ones(T);
        const long long i = base + T;
        const mpn<double, K> a = i <= deg ? mp_load<double, K>(coef, psc, off + i) : mp_zero<double, K>();
        if constexpr (tz == 0) {
            st0 = a;
        } else {
            cplx<K> cur;
            cur.re = bf_add(st0, bf_mul(a, Xl[0].re));
            cur.im = bf_mul(a, Xl[0].im);
#pragma unroll
            for (int l = 1; l < tz; ++l) cur = c_add<K>(st[l], c_mul<K>(cur, Xl[l]));
            st[tz] = cur;
        }
        if constexpr ((T & 3) == 3) asm volatile("" ::: "memory");
        EstrinCplxLocal<K, LB, T + 1>::run(st0, st, Xl, coef, psc, base, deg, off);
    }
};
template <int K, int LB>
struct EstrinCplxLocal<K, LB, (1 << LB)> {
    static __device__ __forceinline__ void run(mpn<double, K>&, cplx<K>*, const cplx<K>*,
                                               const double* __restrict__, long long, long long,
                                               long long, long long) {}
};

template <int K, int LB>
__global__ void __launch_bounds__(256)
k_estrin_cplx(long long batch, long long deg, int L, const double* __restrict__ coef,
              long long psc, const double* __restrict__ xre, const double* __restrict__ xim,
              long long psx, double* __restrict__ yre, double* __restrict__ yim, long long psy) {
    using C = cplx<K>;
    constexpr int B = 1 << LB;
    const long long b = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= batch) return;  // whole wave
    const long long off = b * (deg + 1);
    C Xl[LB + 1];
    Xl[0] = c_load<K>(xre, xim, psx, b);
#pragma unroll
    for (int l = 1; l <= LB; ++l) Xl[l] = c_mul<K>(Xl[l - 1], Xl[l - 1]);
    C c;
    if constexpr (LB == 0) {
        const long long i = lane;
        c.re = i <= deg ? mp_load<double, K>(coef, psc, off + i) : mp_zero<double, K>();
        c.im = mp_zero<double, K>();
    } else {
        mpn<double, K> st0;
        C st[LB + 1];
        EstrinCplxLocal<K, LB, 0>::run(st0, st, Xl, coef, psc, (long long)lane * B, deg, off);
        c = st[LB];
    }
    C Xc = Xl[LB];
    for (int lev = LB; lev < L; ++lev) {
        const int sft = 1 << (lev - LB);
        C other;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            other.re.c[q] = __shfl_down(c.re.c[q], sft, 64);
            other.im.c[q] = __shfl_down(c.im.c[q], sft, 64);
        }
        C comb;
        if (lev == 0) {  // first level with one coefficient per lane: real pairs
            comb.re = bf_add(c.re, bf_mul(other.re, Xc.re));
            comb.im = bf_mul(other.re, Xc.im);
        } else {
            comb = c_add<K>(c, c_mul<K>(other, Xc));
        }
        const bool leader = (lane & (2 * sft - 1)) == 0;
        c = c_select<K>(leader, comb, c);
        Xc = c_mul<K>(Xc, Xc);
    }
    if (lane == 0) c_store<K>(yre, yim, psy, b, c);
}

// Complex-point Estrin for the long lists (N = 2^L, L = LB + 8, LB >= 1):
// one 256-thread workgroup per polynomial, lane-local levels as in
// k_estrin_cplx (the first pairs real coefficients), six levels across the
// lanes of each wave, the last two across the four waves through LDS.
template <int K, int LB>
__global__ void __launch_bounds__(256)
k_estrin_cplx_wg(long long deg, const double* __restrict__ coef, long long psc,
                 const double* __restrict__ xre, const double* __restrict__ xim, long long psx,
                 double* __restrict__ yre, double* __restrict__ yim, long long psy) {
    static_assert(LB >= 1, "the first level must be lane-local");
    using C = cplx<K>;
    constexpr int B = 1 << LB;
    const long long b = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const long long off = b * (deg + 1);
    __shared__ double s_top[4][2][K];
    C Xl[LB + 1];
    Xl[0] = c_load<K>(xre, xim, psx, b);
#pragma unroll
    for (int l = 1; l <= LB; ++l) Xl[l] = c_mul<K>(Xl[l - 1], Xl[l - 1]);
    mpn<double, K> st0;
    C st[LB + 1];
    EstrinCplxLocal<K, LB, 0>::run(st0, st, Xl, coef, psc, (long long)threadIdx.x * B, deg, off);
    C c = st[LB];
    C Xc = Xl[LB];
#pragma unroll
    for (int lev = 0; lev < 6; ++lev) {
        const int sft = 1 << lev;
        C other;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            other.re.c[q] = __shfl_down(c.re.c[q], sft, 64);
            other.im.c[q] = __shfl_down(c.im.c[q], sft, 64);
        }
        const C comb = c_add<K>(c, c_mul<K>(other, Xc));
        const bool leader = (lane & (2 * sft - 1)) == 0;
        c = c_select<K>(leader, comb, c);
        Xc = c_mul<K>(Xc, Xc);
    }
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            s_top[wv][0][q] = c.re.c[q];
            s_top[wv][1][q] = c.im.c[q];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        C v[4];
#pragma unroll
        for (int w = 0; w < 4; ++w)
#pragma unroll
            for (int q = 0; q < K; ++q) {
                v[w].re.c[q] = s_top[w][0][q];
                v[w].im.c[q] = s_top[w][1][q];
            }
        const C lo = c_add<K>(v[0], c_mul<K>(v[1], Xc));
        const C hi = c_add<K>(v[2], c_mul<K>(v[3], Xc));
        Xc = c_mul<K>(Xc, Xc);
        c_store<K>(yre, yim, psy, b, c_add<K>(lo, c_mul<K>(hi, Xc)));
    }
}

// ------------------------------------------------------ Durand-Kerner ----

struct DkPlanDev {
    const int* order;          // polynomial indices, LPT order
    const int* degree;         // per polynomial
    const long long* coef_off; // first coefficient column of polynomial b
    const long long* root_off; // first root column of polynomial b
    double* mre;               // monic coefficient planes (same columns as coefficients)
    double* mim;
    double* zre;               // second iterate buffer (same columns as roots)
    double* zim;
    int* counter;              // work counter
    long long psm, psz;        // plane strides of the plan buffers
    // packed schedule (4-wave jobs): job j owns items job_off[j] .. job_off[j+1]-1,
    // item i = (polynomial, 64-root chunk, wave) at items[3 i .. 3 i + 2]
    const int* job_off;
    const int* items;
    int njobs;
};

__global__ void k_reset_counter(int* c) { *c = 0; }

constexpr double kPi = 3.141592653589793238462643383279502884;

// Prologue, one wave per polynomial: monic coefficients c_i = a_i / a_n and,
// with init, the Aberth start values (binary64, leading components).
template <int K, int AR>
__global__ void __launch_bounds__(64)
k_dk_prologue(int batch, DkPlanDev P, const double* __restrict__ are,
              const double* __restrict__ aim, long long psc, double* rre, double* rim,
              long long psr, int init) {
    using C = cplx<K>;
    const int lane = threadIdx.x;
    for (int b = blockIdx.x; b < batch; b += gridDim.x) {
        const int n = P.degree[b];
        const long long co = P.coef_off[b], ro = P.root_off[b];
        const C an = c_load<K>(are, aim, psc, co + n);
        for (int i = lane; i < n; i += 64)
            c_store<K>(P.mre, P.mim, P.psm, co + i, c_div<K, AR>(c_load<K>(are, aim, psc, co + i), an));
        if (!init) continue;
        __syncthreads();
        int nnz = 0;
        for (int i = lane; i < n; i += 64)
            nnz += (P.mre[co + i] != 0.0 || P.mim[co + i] != 0.0) ? 1 : 0;
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) nnz += __shfl_xor(nnz, off, 64);
        double r = 0.0;
        for (int i = lane; i < n; i += 64) {
            const double mag = hypot(P.mre[co + i], P.mim[co + i]) * (double)nnz;
            const double t = pow(mag, 1.0 / (double)(n - i));
            if (t > r) r = t;
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) r = fmax(r, __shfl_xor(r, off, 64));
        const double cre = -P.mre[co + n - 1] / (double)n;
        const double cim = -P.mim[co + n - 1] / (double)n;
        for (int i = lane; i < n; i += 64) {
            const double th = 2.0 * (double)i * kPi / (double)n + 3.0 / (2.0 * (double)n);
            C z;
            z.re = mp_from<double, K>(cre + r * cos(th));
            z.im = mp_from<double, K>(cim + r * sin(th));
            c_store<K>(rre, rim, psr, ro + i, z);
        }
        __syncthreads();
    }
}

// One DK update of the roots base, base + 64, ..., base + 64 (R - 1) (those
// below n) of one polynomial: Horner for q(z_i) on the monic coefficients
// (mre, mim), the product over j != i of (z_i - z_j) in ascending j, both
// with power-of-two rescaling, then z_i - q(z_i) / prod, read from the
// source iterate (sre, sim) and written to the destination (dre, dim).
template <int K, int R, int AR>
__device__ __forceinline__ void dk_roots(const DkPlanDev& P, const double* mre, const double* mim,
                                         const double* sre, const double* sim, long long pss,
                                         double* dre, double* dim, long long psd, int n,
                                         long long ro, int base) {
    using C = cplx<K>;
    int idx[R];
    C z[R], h[R];
    long long E[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        idx[r] = base + 64 * r;
        const int ic = idx[r] < n ? idx[r] : n - 1;
        z[r] = c_load<K>(sre, sim, pss, ro + ic);
        h[r].re = mp_from<double, K>(1.0);
        h[r].im = mp_zero<double, K>();
        E[r] = 0;
    }
    // q(z) by Horner on the monic coefficients
#pragma nounroll
    for (int k = n - 1; k >= 0; --k) {
        const C ck = c_load<K>(mre, mim, P.psm, k);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            h[r] = c_add<K, AR>(c_mul<K, AR>(h[r], z[r]), c_ldexp<K>(ck, clamp_exp(-E[r])));
            c_rescale<K, true>(h[r], E[r]);
        }
    }
    // prod_{j != i} (z_i - z_j), j ascending
    C Pp[R];
    long long F[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        Pp[r].re = mp_from<double, K>(1.0);
        Pp[r].im = mp_zero<double, K>();
        F[r] = 0;
    }
#pragma nounroll
    for (int j = 0; j < n; ++j) {
        const C zj = c_load<K>(sre, sim, pss, ro + j);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            C t = c_mul<K, AR>(Pp[r], c_sub<K, AR>(z[r], zj));
            long long Ft = F[r];
            c_rescale<K, false>(t, Ft);
            const bool take = j != idx[r];
            Pp[r] = c_select<K>(take, t, Pp[r]);
            F[r] = take ? Ft : F[r];
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const C w = c_ldexp<K>(c_div<K, AR>(h[r], Pp[r]), clamp_exp(E[r] - F[r]));
        if (idx[r] < n) c_store<K>(dre, dim, psd, ro + idx[r], c_sub<K, AR>(z[r], w));
    }
}

// Persistent iteration kernel: one-wave workgroups pull polynomials in LPT
// order.  The slot goes through LDS rather than a lane shuffle, so the
// compiler keeps the per-polynomial values (degree, offsets) in scalar
// registers.  The barrier after each sweep orders sweep t's writes before
// sweep t + 1's reads; every lane runs the same number of barriers (the
// slot, iters and status are the same in every lane).
template <int K, int R, int AR>
__global__ void __launch_bounds__(64)
k_durand_kerner(int batch, DkPlanDev P, double* rre, double* rim, long long psr, int* status,
                int iters) {
    const int lane = threadIdx.x;
    __shared__ int s_slot;
    for (;;) {
        if (threadIdx.x == 0) s_slot = atomicAdd(P.counter, 1);
        __syncthreads();
        const int slot = s_slot;
        __syncthreads();  // all have read s_slot before it is overwritten
        if (slot >= batch) break;  // the same value in every thread: uniform exit
        const int b = P.order[slot];
        const int n = P.degree[b];
        const long long co = P.coef_off[b], ro = P.root_off[b];

        const double* mre = P.mre + co;
        const double* mim = P.mim + co;
        for (int it = 0; it < iters; ++it) {
            const bool from_user = (it & 1) == 0;
            const double* sre = from_user ? rre : P.zre;
            const double* sim = from_user ? rim : P.zim;
            double* dre = from_user ? P.zre : rre;
            double* dim = from_user ? P.zim : rim;
            const long long pss = from_user ? psr : P.psz;
            const long long psd = from_user ? P.psz : psr;
            for (int base = lane; base < n; base += 64 * R)
                dk_roots<K, R, AR>(P, mre, mim, sre, sim, pss, dre, dim, psd, n, ro, base);
            __syncthreads();  // iterate t complete before t+1 reads it
        }
        if (iters & 1) {  // result is in the plan buffer: copy back to the caller's
            for (int i = lane; i < n; i += 64)
                c_store<K>(rre, rim, psr, ro + i, c_load<K>(P.zre, P.zim, P.psz, ro + i));
            __syncthreads();
        }
        if (status) {
            int bad = 0;
            for (int i = lane; i < n; i += 64) {
#pragma unroll
                for (int c = 0; c < K; ++c)
                    bad |= !isfinite(rre[c * psr + ro + i]) || !isfinite(rim[c * psr + ro + i]);
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) bad |= __shfl_xor(bad, off, 64);
            if (lane == 0) status[b] = bad;
        }
        __syncthreads();
    }
}

// Packed persistent kernel: 4-wave workgroups pull jobs (heaviest first); a
// job holds whole polynomials whose 64-root chunks the plan spread over the
// four waves so that their per-sweep loads are nearly equal (a polynomial
// larger than a wave's share is split across waves, small ones are packed
// together).  The barrier after each sweep orders sweep t's writes before
// sweep t + 1's reads for every polynomial of the job; every thread runs the
// same number of barriers (the job index, iters and status are uniform).
constexpr int kDkPackedWaves = 4;

template <int K, int AR>
__global__ void __launch_bounds__(64 * kDkPackedWaves)
k_dk_packed(DkPlanDev P, double* rre, double* rim, long long psr, int* status, int iters) {
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    __shared__ int s_slot;
    for (;;) {
        if (threadIdx.x == 0) s_slot = atomicAdd(P.counter, 1);
        __syncthreads();
        const int slot = s_slot;
        __syncthreads();  // all have read s_slot before it is overwritten
        if (slot >= P.njobs) break;  // the same value in every thread: uniform exit
        const int i0 = P.job_off[slot], i1 = P.job_off[slot + 1];
        for (int it = 0; it < iters; ++it) {
            const bool from_user = (it & 1) == 0;
            const double* sre = from_user ? rre : P.zre;
            const double* sim = from_user ? rim : P.zim;
            double* dre = from_user ? P.zre : rre;
            double* dim = from_user ? P.zim : rim;
            const long long pss = from_user ? psr : P.psz;
            const long long psd = from_user ? P.psz : psr;
            for (int i = i0; i < i1; ++i) {
                if (P.items[3 * i + 2] != wv) continue;  // the same in every lane of the wave
                const int b = P.items[3 * i], ch = P.items[3 * i + 1];
                const long long co = P.coef_off[b];
                dk_roots<K, 1, AR>(P, P.mre + co, P.mim + co, sre, sim, pss, dre, dim, psd,
                                   P.degree[b], P.root_off[b], 64 * ch + lane);
            }
            __syncthreads();  // iterate t complete before t+1 reads it
        }
        if (iters & 1) {  // result is in the plan buffer: each wave copies its chunks back
            for (int i = i0; i < i1; ++i) {
                if (P.items[3 * i + 2] != wv) continue;
                const int b = P.items[3 * i], r = 64 * P.items[3 * i + 1] + lane;
                const long long ro = P.root_off[b];
                if (r < P.degree[b])
                    c_store<K>(rre, rim, psr, ro + r, c_load<K>(P.zre, P.zim, P.psz, ro + r));
            }
            __syncthreads();
        }
        if (status) {  // the wave holding chunk 0 of a polynomial checks all its roots
            for (int i = i0; i < i1; ++i) {
                if (P.items[3 * i + 2] != wv || P.items[3 * i + 1] != 0) continue;
                const int b = P.items[3 * i], n = P.degree[b];
                const long long ro = P.root_off[b];
                int bad = 0;
                for (int r = lane; r < n; r += 64) {
#pragma unroll
                    for (int c = 0; c < K; ++c)
                        bad |= !isfinite(rre[c * psr + ro + r]) || !isfinite(rim[c * psr + ro + r]);
                }
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) bad |= __shfl_xor(bad, off, 64);
                if (lane == 0) status[b] = bad;
            }
        }
        __syncthreads();
    }
}

// Lane-packed schedule: a job's polynomials (descending degree, with small
// ones filling lanes its larger ones leave idle) have their roots laid out
// over 64-lane items; an item's lanes may belong to several polynomials, and
// its loops run to the largest degree among them (a lane stops at its own
// degree).  Items of (job j, wave w) are wave_off[j W + w] ..
// wave_off[j W + w + 1] - 1.
struct DkLaneSched {
    const int* wave_off;   // njobs W + 1 entries
    const int* item_len;   // per item: loop length
    const int2* lanes;     // per item: 64 (polynomial, root index), polynomial -1 = idle lane
    const int* poly_off;   // njobs + 1: polynomials of job j are polys[poly_off[j] .. poly_off[j+1]-1]
    const int* polys;
    const int* wg_off;     // static schedule: nbins + 1 job offsets, one range per workgroup; else null
    int njobs;
    int nbins;             // static schedule: workgroups (the launch's grid); else 0
};

// One DK update of root idx of polynomial b (b < 0: an idle lane, which loads
// and stores nothing) inside an item whose loops run len steps: the same
// Horner and root-difference product as dk_roots, each step taken only
// while the step index is below the lane's own degree.
template <int K, int AR>
__device__ __forceinline__ void dk_root_lane(const DkPlanDev& P, int b, int idx, int len,
                                             const double* sre, const double* sim, long long pss,
                                             double* dre, double* dim, long long psd) {
    using C = cplx<K>;
    const bool live = b >= 0;
    const int n = live ? P.degree[b] : 0;
    const long long co = live ? P.coef_off[b] : 0;
    const long long ro = live ? P.root_off[b] : 0;
    C z;
    z.re = mp_zero<double, K>();
    z.im = mp_zero<double, K>();
    if (live) z = c_load<K>(sre, sim, pss, ro + idx);
    C h;
    h.re = mp_from<double, K>(1.0);
    h.im = mp_zero<double, K>();
    long long E = 0;
#pragma nounroll
    for (int k = len - 1; k >= 0; --k) {
        if (k < n) {
            const C ck = c_load<K>(P.mre, P.mim, P.psm, co + k);
            h = c_add<K, AR>(c_mul<K, AR>(h, z), c_ldexp<K>(ck, clamp_exp(-E)));
            c_rescale<K, true>(h, E);
        }
    }
    C Pp;
    Pp.re = mp_from<double, K>(1.0);
    Pp.im = mp_zero<double, K>();
    long long F = 0;
#pragma nounroll
    for (int j = 0; j < len; ++j) {
        if (j < n) {
            const C zj = c_load<K>(sre, sim, pss, ro + j);
            C t = c_mul<K, AR>(Pp, c_sub<K, AR>(z, zj));
            long long Ft = F;
            c_rescale<K, false>(t, Ft);
            const bool take = j != idx;
            Pp = c_select<K>(take, t, Pp);
            F = take ? Ft : F;
        }
    }
    if (live) {
        const C w = c_ldexp<K>(c_div<K, AR>(h, Pp), clamp_exp(E - F));
        c_store<K>(dre, dim, psd, ro + idx, c_sub<K, AR>(z, w));
    }
}

// One job of the lane-packed schedule, swept by a W-wave workgroup: the
// barrier after each sweep orders sweep t's writes before sweep t + 1's reads
// for every polynomial of the job, and every thread runs the same number of
// barriers (slot, iters and status are uniform).  The copy-back of an odd
// sweep count and the status flags go over the job's polynomial list, one
// polynomial per wave at a time.
template <int K, int AR, int W>
__device__ __forceinline__ void dk_lane_job(const DkPlanDev& P, const DkLaneSched& S, int slot,
                                            double* rre, double* rim, long long psr,
                                            int* status, int iters) {
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int i0 = S.wave_off[slot * W + wv], i1 = S.wave_off[slot * W + wv + 1];
    for (int it = 0; it < iters; ++it) {
        const bool from_user = (it & 1) == 0;
        const double* sre = from_user ? rre : P.zre;
        const double* sim = from_user ? rim : P.zim;
        double* dre = from_user ? P.zre : rre;
        double* dim = from_user ? P.zim : rim;
        const long long pss = from_user ? psr : P.psz;
        const long long psd = from_user ? P.psz : psr;
        for (int i = i0; i < i1; ++i) {
            const int2 e = S.lanes[64LL * i + lane];
            dk_root_lane<K, AR>(P, e.x, e.y, S.item_len[i], sre, sim, pss, dre, dim, psd);
        }
        __syncthreads();  // iterate t complete before t+1 reads it
    }
    const int q0 = S.poly_off[slot], q1 = S.poly_off[slot + 1];
    if (iters & 1) {  // result is in the plan buffer: copy the job's roots back
        for (int q = q0 + wv; q < q1; q += W) {
            const int b = S.polys[q], n = P.degree[b];
            const long long ro = P.root_off[b];
            for (int r = lane; r < n; r += 64)
                c_store<K>(rre, rim, psr, ro + r, c_load<K>(P.zre, P.zim, P.psz, ro + r));
        }
        __syncthreads();
    }
    if (status) {
        for (int q = q0 + wv; q < q1; q += W) {
            const int b = S.polys[q], n = P.degree[b];
            const long long ro = P.root_off[b];
            int bad = 0;
            for (int r = lane; r < n; r += 64) {
#pragma unroll
                for (int c = 0; c < K; ++c)
                    bad |= !isfinite(rre[c * psr + ro + r]) || !isfinite(rim[c * psr + ro + r]);
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) bad |= __shfl_xor(bad, off, 64);
            if (lane == 0) status[b] = bad;
        }
    }
    __syncthreads();
}

// Lane-packed persistent kernel.  Dynamic schedule: W-wave workgroups pull
// jobs (heaviest first) from the plan's counter until none is left.  Static
// schedule: workgroup g sweeps the jobs wg_off[g] .. wg_off[g+1]-1 (the grid
// is exactly the schedule's nbins workgroups).
template <int K, int AR, int W>
__global__ void __launch_bounds__(64 * W)
k_dk_lanes(DkPlanDev P, DkLaneSched S, double* rre, double* rim, long long psr, int* status,
           int iters) {
    if (S.wg_off) {
        const int j1 = S.wg_off[blockIdx.x + 1];
        for (int slot = S.wg_off[blockIdx.x]; slot < j1; ++slot)
            dk_lane_job<K, AR, W>(P, S, slot, rre, rim, psr, status, iters);
        return;
    }
    __shared__ int s_slot;
    for (;;) {
        if (threadIdx.x == 0) s_slot = atomicAdd(P.counter, 1);
        __syncthreads();
        const int slot = s_slot;
        __syncthreads();  // all have read s_slot before it is overwritten
        if (slot >= S.njobs) break;  // the same value in every thread: uniform exit
        dk_lane_job<K, AR, W>(P, S, slot, rre, rim, psr, status, iters);
    }
}

// ---------------------------------------------------------------- plan ----

enum { DK_WAVE = 0, DK_PACKED = 1, DK_LANES = 2 };

struct DkVariant {
    int r;          // roots per lane processed together (one-wave kernel)
    int waves_cu;   // resident waves per CU targeted by the grid size
    int kind;       // DK_WAVE: a wave per polynomial; DK_PACKED: 4-wave jobs of
                    // 64-root chunks; DK_LANES: W-wave jobs of lane-packed items
    int w;          // waves per job (DK_LANES)
    int lscale;     // job cap, percent of the largest polynomial's heaviest wave (DK_LANES)
    int sched;      // index of the plan's lane-packed schedule (DK_LANES)
    int stat;       // 1: static job-to-workgroup schedule (DK_LANES); 0: shared counter
};
static const DkVariant kDkVariants[] = {
    {1, 8, DK_WAVE, 1, 0, -1, 0},     {2, 8, DK_WAVE, 1, 0, -1, 0},
    {1, 16, DK_WAVE, 1, 0, -1, 0},    {2, 12, DK_WAVE, 1, 0, -1, 0},
    {1, 8, DK_PACKED, 4, 0, -1, 0},   {1, 12, DK_PACKED, 4, 0, -1, 0},
    {1, 12, DK_LANES, 4, 100, 0, 0},  {1, 12, DK_LANES, 4, 150, 1, 0},
    {1, 8, DK_LANES, 4, 100, 2, 0},   {1, 12, DK_LANES, 12, 200, 3, 0},
    {1, 16, DK_LANES, 16, 100, 4, 0}, {1, 16, DK_LANES, 16, 200, 5, 0},
    {1, 16, DK_LANES, 4, 100, 6, 0},  {1, 16, DK_LANES, 16, 100, 7, 1},
    {1, 12, DK_LANES, 12, 200, 8, 1}, {1, 16, DK_LANES, 16, 200, 9, 1}};
constexpr int kDkVariantCount = sizeof(kDkVariants) / sizeof(kDkVariants[0]);
constexpr int kDkLaneScheds = 10;
// A new plan's variant: lane-packed 16-wave jobs (four waves per SIMD) on a
// static schedule, every CU sweeping its own list of jobs.  On 4096 QD
// polynomials of degrees 16..512 over 200 sweeps it took 3.57 s, against
// 3.75 s for the same jobs taken from the shared counter (heaviest first to
// the first free workgroup leaves some CUs a job short near the end), 3.80 s
// for 12-wave jobs, 4.15 s for the packed 4-wave chunks and 4.3 s with 24
// resident waves per CU; the job cap moved it by under 1 %.  On 4096 copies
// of one degree-64 polynomial (every polynomial one 64-lane item) it is
// within 3 % of the fastest variant.
constexpr int kDkDefaultVariant = 13;

}  // namespace mpx

// Opaque plan (declared in mpx.h as struct mpx_plan_s).
struct mpx_plan_s {
    int prec = 0, K = 0, batch = 0, iters = 0;
    unsigned flags = 0;
    int variant = mpx::kDkDefaultVariant;
    int max_degree = 0;
    long long total_coef = 0, total_roots = 0;
    int cus = 256;
    void* dev = nullptr;            // one allocation: schedule + offsets + buffers
    mpx::DkPlanDev d{};
    void* lane_dev[mpx::kDkLaneScheds] = {};   // lane-packed schedules, one allocation each
    mpx::DkLaneSched lane[mpx::kDkLaneScheds] = {};
    // graph cache
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void* g_key[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    long long g_ps[2] = {0, 0};
    hipStream_t g_stream = nullptr;
    int g_variant = -1;
};

namespace mpx {

template <int K, int R, int AR, int KIND, int W>
static int launch_dk_t(mpx_plan_s* p, const DkVariant& v, const void* are, const void* aim,
                       long long psc, void* rre, void* rim, long long psr, int* status,
                       hipStream_t s) {
    k_reset_counter<<<1, 1, 0, s>>>(p->d.counter);
    int st = launch_status();
    if (st) return st;
    long long grid = (long long)p->cus * v.waves_cu;
    if (grid > p->batch) grid = p->batch;
    if (grid < 1) grid = 1;
    k_dk_prologue<K, AR><<<(unsigned)grid, 64, 0, s>>>(p->batch, p->d, (const double*)are,
                                                  (const double*)aim, psc, (double*)rre,
                                                  (double*)rim, psr,
                                                  (p->flags & MPX_DK_INIT) ? 1 : 0);
    if ((st = launch_status())) return st;
    if constexpr (KIND == DK_PACKED) {
        long long groups = (long long)p->cus * v.waves_cu / kDkPackedWaves;
        if (groups > p->d.njobs) groups = p->d.njobs;
        if (groups < 1) groups = 1;
        k_dk_packed<K, AR><<<(unsigned)groups, 64 * kDkPackedWaves, 0, s>>>(
            p->d, (double*)rre, (double*)rim, psr, status, p->iters);
    } else if constexpr (KIND == DK_LANES) {
        const DkLaneSched& S = p->lane[v.sched];
        long long groups = (long long)p->cus * v.waves_cu / W;
        if (groups > S.njobs) groups = S.njobs;
        if (groups < 1) groups = 1;
        if (S.wg_off) groups = S.nbins;  // one workgroup per range of the static schedule
        k_dk_lanes<K, AR, W><<<(unsigned)groups, 64 * W, 0, s>>>(p->d, S, (double*)rre,
                                                              (double*)rim, psr, status, p->iters);
    } else {
        k_durand_kerner<K, R, AR><<<(unsigned)grid, 64, 0, s>>>(p->batch, p->d, (double*)rre,
                                                            (double*)rim, psr, status, p->iters);
    }
    return launch_status();
}

static int launch_dk(mpx_plan_s* p, int variant, const void* are, const void* aim, long long psc,
                     void* rre, void* rim, long long psr, int* status, hipStream_t s) {
    const DkVariant& v = kDkVariants[variant];
#define MPX_DK_CASE(KK, AR_)                                                                  \
    if (p->K == KK && ar == AR_) {                                                            \
        if (v.kind == DK_PACKED)                                                              \
            return launch_dk_t<KK, 1, AR_, DK_PACKED, 4>(p, v, are, aim, psc, rre, rim, psr,  \
                                                         status, s);                          \
        if (v.kind == DK_LANES) {                                                             \
            if (v.w == 4)                                                                     \
                return launch_dk_t<KK, 1, AR_, DK_LANES, 4>(p, v, are, aim, psc, rre, rim,    \
                                                            psr, status, s);                  \
            if (v.w == 8)                                                                     \
                return launch_dk_t<KK, 1, AR_, DK_LANES, 8>(p, v, are, aim, psc, rre, rim,    \
                                                            psr, status, s);                  \
            if (v.w == 16)                                                                    \
                return launch_dk_t<KK, 1, AR_, DK_LANES, 16>(p, v, are, aim, psc, rre, rim,   \
                                                             psr, status, s);                 \
            return launch_dk_t<KK, 1, AR_, DK_LANES, 12>(p, v, are, aim, psc, rre, rim, psr,  \
                                                         status, s);                          \
        }                                                                                     \
        if (v.r == 1)                                                                         \
            return launch_dk_t<KK, 1, AR_, DK_WAVE, 1>(p, v, are, aim, psc, rre, rim, psr,    \
                                                       status, s);                            \
        return launch_dk_t<KK, 2, AR_, DK_WAVE, 1>(p, v, are, aim, psc, rre, rim, psr,        \
                                                   status, s);                                \
    }
    const int ar = arith_of(p->prec);
    MPX_DK_CASE(2, AR_BF)
    MPX_DK_CASE(3, AR_BF)
    MPX_DK_CASE(4, AR_BF)
    MPX_DK_CASE(2, AR_NOBF)
    MPX_DK_CASE(3, AR_NOBF)
    MPX_DK_CASE(4, AR_NOBF)
    MPX_DK_CASE(2, AR_NOBF_ACC)
#undef MPX_DK_CASE
    return MPX_EPREC;
}

}  // namespace mpx

using namespace mpx;

// ---------------------------------------------------------------- C ABI ----

// Byte extent of K planes of n binary64 values at plane stride ps.
static uint64_t vec_bytes(int K, int64_t n, int64_t ps) {
    return planes_bytes(K, 1, n, n, ps, sizeof(double));
}

// Does the output range [out, out + nb) overlap the coefficient planes or any
// of the point / weight vectors (batch values per plane at stride psv)?
static bool poly_out_overlaps(int K, const void* out, uint64_t nb, int64_t batch, int64_t deg,
                              const void* coef, int64_t psc, const void* v0, const void* v1,
                              const void* v2, int64_t psv) {
    const uint64_t cb = vec_bytes(K, batch * (deg + 1), psc), vb = vec_bytes(K, batch, psv);
    return overlaps(out, nb, coef, cb) || overlaps(out, nb, v0, vb) || overlaps(out, nb, v1, vb) ||
           overlaps(out, nb, v2, vb);
}

static int polyval_check(int prec, int64_t batch, int64_t deg, const void* coef, int64_t psc,
                         const void* x, int64_t psx) {
    if (prec != MPX_DD && prec != MPX_TD && prec != MPX_QD) return MPX_EPREC;
    if (batch < 0 || deg < 0 || deg == INT64_MAX) return MPX_EINVAL;
    if (batch > INT32_MAX) return MPX_ENOTSUP;  // grid dimensions
    if (batch == 0) return MPX_OK;
    if (coef == nullptr || !prod_fits(batch, deg + 1, psc) || x == nullptr || psx < batch)
        return MPX_EINVAL;
    return MPX_OK;
}

extern "C" int mpx_polyval(int prec, int64_t batch, int64_t deg, const void* coef, int64_t psc,
                           const void* x, int64_t psx, void* y, int64_t psy, void* stream) {
    if (!prec_k_ar(prec) || base_prec(prec) == MPX_FF) return MPX_EPREC;
    int st = polyval_check(base_prec(prec), batch, deg, coef, psc, x, psx);
    if (st) return st;
    if (batch == 0) return MPX_OK;
    if (y == nullptr || psy < batch) return MPX_EINVAL;
    if (poly_out_overlaps(prec_k_ar(prec), y, vec_bytes(prec_k_ar(prec), batch, psy), batch, deg,
                          coef, psc, x, nullptr, nullptr, psx))
        return MPX_EINVAL;
    const unsigned blocks = (unsigned)ceil_div(batch, 64);
    hipStream_t s = as_stream(stream);
#define MPX_PV(K_, AR_)                                                                     \
    k_polyval<K_, AR_><<<blocks, 64, 0, s>>>(batch, deg, (const double*)coef, psc,             \
                                             (const double*)x, psx, (double*)y, psy);          \
    break
    switch (prec) {
        case MPX_DD: MPX_PV(2, AR_BF);
        case MPX_TD: MPX_PV(3, AR_BF);
        case MPX_QD: MPX_PV(4, AR_BF);
        case MPX_DD | MPX_NOBF: MPX_PV(2, AR_NOBF);
        case MPX_TD | MPX_NOBF: MPX_PV(3, AR_NOBF);
        case MPX_QD | MPX_NOBF: MPX_PV(4, AR_NOBF);
        case MPX_DD | MPX_NOBF_ACC: MPX_PV(2, AR_NOBF_ACC);
        default: return MPX_EPREC;
    }
#undef MPX_PV
    return launch_status();
}

template <int K>
static int estrin_t(long long batch, long long deg, const void* coef, long long psc, const void* x,
                    long long psx, void* y, long long psy, hipStream_t s) {
    int L = 0;
    while (L < 62 && (1LL << L) < deg + 1) ++L;  // beyond the supported depths: ENOTSUP below
    if (L >= 12) {  // 4 waves per polynomial, 2^(L-8) coefficients per lane
        if (L > 13 || batch > INT32_MAX) return MPX_ENOTSUP;
        if (L == 12)
            k_estrin_wg<K, 4><<<(unsigned)batch, 256, 0, s>>>(deg, (const double*)coef, psc,
                                                              (const double*)x, psx, (double*)y, psy);
        else
            k_estrin_wg<K, 5><<<(unsigned)batch, 256, 0, s>>>(deg, (const double*)coef, psc,
                                                              (const double*)x, psx, (double*)y, psy);
        return launch_status();
    }
    const int LB = L > 6 ? L - 6 : 0;
    const unsigned blocks = (unsigned)ceil_div(batch, 4);
#define MPX_ES(LBV)                                                                             \
    case LBV:                                                                                   \
        k_estrin<K, LBV><<<blocks, 256, 0, s>>>(batch, deg, L, (const double*)coef, psc,         \
                                               (const double*)x, psx, (double*)y, psy);         \
        break;
    switch (LB) {
        MPX_ES(0) MPX_ES(1) MPX_ES(2) MPX_ES(3) MPX_ES(4) MPX_ES(5)
        default: return MPX_ENOTSUP;
    }
#undef MPX_ES
    return launch_status();
}

template <int K>
static int estrin_cplx_t(long long batch, long long deg, const void* coef, long long psc,
                         const void* xre, const void* xim, long long psx, void* yre, void* yim,
                         long long psy, hipStream_t s) {
    int L = 0;
    while (L < 62 && (1LL << L) < deg + 1) ++L;  // beyond the supported depths: ENOTSUP below
    if (L >= 11) {  // 4 waves per polynomial, 2^(L-8) coefficients per lane
        if (L > 12 || batch > INT32_MAX) return MPX_ENOTSUP;
        if (L == 11)
            k_estrin_cplx_wg<K, 3><<<(unsigned)batch, 256, 0, s>>>(
                deg, (const double*)coef, psc, (const double*)xre, (const double*)xim, psx,
                (double*)yre, (double*)yim, psy);
        else
            k_estrin_cplx_wg<K, 4><<<(unsigned)batch, 256, 0, s>>>(
                deg, (const double*)coef, psc, (const double*)xre, (const double*)xim, psx,
                (double*)yre, (double*)yim, psy);
        return launch_status();
    }
    const int LB = L > 6 ? L - 6 : 0;
    const unsigned blocks = (unsigned)ceil_div(batch, 4);
#define MPX_EC(LBV)                                                                            \
    case LBV:                                                                                  \
        k_estrin_cplx<K, LBV><<<blocks, 256, 0, s>>>(batch, deg, L, (const double*)coef, psc,  \
                                                     (const double*)xre, (const double*)xim,   \
                                                     psx, (double*)yre, (double*)yim, psy);    \
        break;
    switch (LB) {
        MPX_EC(0) MPX_EC(1) MPX_EC(2) MPX_EC(3) MPX_EC(4)
        default: return MPX_ENOTSUP;
    }
#undef MPX_EC
    return launch_status();
}

extern "C" int mpx_polyval_cplx(int prec, int64_t batch, int64_t deg, const void* coef,
                                int64_t psc, const void* xre, const void* xim, int64_t psx,
                                void* yre, void* yim, int64_t psy, int method, void* stream) {
    if (!prec_k_ar(prec) || base_prec(prec) == MPX_FF) return MPX_EPREC;
    if (method != 0 && method != 1) return MPX_EINVAL;
    if (method == 1 && arith_of(prec) != 0) return MPX_EPREC;
    int st = polyval_check(base_prec(prec), batch, deg, coef, psc, xre, psx);
    if (st) return st;
    if (batch == 0) return MPX_OK;
    if (xim == nullptr || yre == nullptr || yim == nullptr || psy < batch) return MPX_EINVAL;
    {
        const int K = prec_k_ar(prec);
        const uint64_t yb = vec_bytes(K, batch, psy);
        if (poly_out_overlaps(K, yre, yb, batch, deg, coef, psc, xre, xim, nullptr, psx) ||
            poly_out_overlaps(K, yim, yb, batch, deg, coef, psc, xre, xim, nullptr, psx) ||
            overlaps(yre, yb, yim, yb))
            return MPX_EINVAL;
    }
    hipStream_t s = as_stream(stream);
    if (method == 1) {
        if (deg >= 4096) return MPX_ENOTSUP;  // 16 coefficients per lane at most
        switch (prec) {
            case MPX_DD: return estrin_cplx_t<2>(batch, deg, coef, psc, xre, xim, psx, yre, yim, psy, s);
            case MPX_TD: return estrin_cplx_t<3>(batch, deg, coef, psc, xre, xim, psx, yre, yim, psy, s);
            default: return estrin_cplx_t<4>(batch, deg, coef, psc, xre, xim, psx, yre, yim, psy, s);
        }
    }
    const unsigned blocks = (unsigned)ceil_div(batch, 64);
#define MPX_PC(K_, AR_)                                                                      \
    k_polyval_cplx<K_, AR_><<<blocks, 64, 0, s>>>(batch, deg, (const double*)coef, psc,     \
                                                  (const double*)xre, (const double*)xim,   \
                                                  psx, (double*)yre, (double*)yim, psy);    \
    break
    switch (prec) {
        case MPX_DD: MPX_PC(2, AR_BF);
        case MPX_TD: MPX_PC(3, AR_BF);
        case MPX_QD: MPX_PC(4, AR_BF);
        case MPX_DD | MPX_NOBF: MPX_PC(2, AR_NOBF);
        case MPX_TD | MPX_NOBF: MPX_PC(3, AR_NOBF);
        case MPX_QD | MPX_NOBF: MPX_PC(4, AR_NOBF);
        case MPX_DD | MPX_NOBF_ACC: MPX_PC(2, AR_NOBF_ACC);
        default: return MPX_EPREC;
    }
#undef MPX_PC
    return launch_status();
}

extern "C" int mpx_polyval_estrin(int prec, int64_t batch, int64_t deg, const void* coef,
                                  int64_t psc, const void* x, int64_t psx, void* y, int64_t psy,
                                  void* stream) {
    int st = polyval_check(prec, batch, deg, coef, psc, x, psx);
    if (st) return st;
    if (batch == 0) return MPX_OK;
    if (y == nullptr || psy < batch) return MPX_EINVAL;
    if (poly_out_overlaps(prec, y, vec_bytes(prec, batch, psy), batch, deg, coef, psc, x, nullptr,
                          nullptr, psx))
        return MPX_EINVAL;
    // degrees 2048..8191 run four waves per polynomial (at most 32
    // coefficients per lane); longer lists are not offered
    if (deg >= 8192) return MPX_ENOTSUP;
    hipStream_t s = as_stream(stream);
    switch (prec) {
        case MPX_DD: return estrin_t<2>(batch, deg, coef, psc, x, psx, y, psy, s);
        case MPX_TD: return estrin_t<3>(batch, deg, coef, psc, x, psx, y, psy, s);
        default: return estrin_t<4>(batch, deg, coef, psc, x, psx, y, psy, s);
    }
}

extern "C" int mpx_polyval_backward(int prec, int64_t batch, int64_t deg, const void* coef,
                                    int64_t psc, const void* x, int64_t psx, const void* gy,
                                    int64_t psg, void* gcoef, int64_t psgc, void* gx,
                                    int64_t psgx, void* stream) {
    int st = polyval_check(prec, batch, deg, coef, psc, x, psx);
    if (st) return st;
    if (batch == 0) return MPX_OK;
    if (gy == nullptr || psg < batch) return MPX_EINVAL;
    if (gcoef && !prod_fits(batch, deg + 1, psgc)) return MPX_EINVAL;
    if (gx && psgx < batch) return MPX_EINVAL;
    if (!gcoef && !gx) return MPX_OK;
    {
        // x and gy are both batch values per plane, at their own strides
        const int K = prec;
        const uint64_t gcb = gcoef ? vec_bytes(K, batch * (deg + 1), psgc) : 0;
        const uint64_t gxb = gx ? vec_bytes(K, batch, psgx) : 0;
        const uint64_t gyb = vec_bytes(K, batch, psg);
        for (const auto& o : {std::make_pair((const void*)gcoef, gcb), std::make_pair((const void*)gx, gxb)})
            if (poly_out_overlaps(K, o.first, o.second, batch, deg, coef, psc, x, nullptr, nullptr, psx) ||
                overlaps(o.first, o.second, gy, gyb))
                return MPX_EINVAL;
        if (overlaps(gcoef, gcb, gx, gxb)) return MPX_EINVAL;
    }
    const unsigned ncb = gcoef ? (unsigned)ceil_div(batch, 128) : 0u;
    const unsigned grid = ncb + (gx ? (unsigned)ceil_div(batch, 64) : 0u);
    hipStream_t s = as_stream(stream);
#define MPX_PB(KK)                                                                             \
    k_polyval_bwd<KK><<<grid, 128, 0, s>>>(batch, deg, (const double*)coef, psc,               \
                                           (const double*)x, psx, (const double*)gy, psg,      \
                                           (double*)gcoef, psgc, (double*)gx, psgx, ncb)
    switch (prec) {
        case MPX_DD: MPX_PB(2); break;
        case MPX_TD: MPX_PB(3); break;
        default: MPX_PB(4); break;
    }
#undef MPX_PB
    return launch_status();
}

// Tune-cache key of a plan: precision, log2 buckets of batch and largest degree.
static std::string dk_tune_key(const mpx_plan_s* p) {
    auto lg = [](long long v) { int b = 0; while ((2LL << b) <= v) ++b; return b; };
    char buf[64];
    std::snprintf(buf, sizeof buf, "dk %d %d %d", p->prec, lg(std::max(p->batch, 1)),
                  lg(std::max(p->max_degree, 1)));
    return buf;
}

// Variant a new plan starts on: MPX_DK_VARIANT if it names a valid index,
// else the tuned choice for its bucket, else kDkDefaultVariant.
static int dk_start_variant(const mpx_plan_s* p) {
    if (const char* f = std::getenv("MPX_DK_VARIANT")) {
        char* end = nullptr;
        const long v = std::strtol(f, &end, 10);
        if (end != f && *end == '\0' && v >= 0 && v < kDkVariantCount) return (int)v;
    }
    std::string choice;
    if (tune_lookup(dk_tune_key(p), choice)) {
        char* end = nullptr;
        const long v = std::strtol(choice.c_str(), &end, 10);
        if (end != choice.c_str() && *end == '\0' && v >= 0 && v < kDkVariantCount) return (int)v;
    }
    return kDkDefaultVariant;
}

extern "C" int mpx_plan_destroy(mpx_plan p) {
    if (!p) return MPX_OK;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->dev) (void)hipFree(p->dev);
    for (void* q : p->lane_dev)
        if (q) (void)hipFree(q);
    delete p;
    return MPX_OK;
}

// Columns of the coefficient and root planes are limited to 2^40 so every
// buffer size and offset stays far from int64 overflow.
constexpr long long kDkMaxColumns = 1LL << 40;

static int polyroots_plan(mpx_plan* out, int prec, int64_t batch, const int32_t* degree_host,
                          const int64_t* coef_off_host, const int64_t* root_off_host, int iters,
                          uint32_t flags) {
    if (out == nullptr) return MPX_EINVAL;
    *out = nullptr;
    if (!prec_k_ar(prec) || base_prec(prec) == MPX_FF) return MPX_EPREC;
    if (batch < 0 || batch > INT32_MAX || (degree_host == nullptr && batch > 0) || iters < 0)
        return MPX_EINVAL;
    if (flags & ~(uint32_t)(MPX_DK_INIT | MPX_DK_GRAPH)) return MPX_EINVAL;
    if ((coef_off_host == nullptr) != (root_off_host == nullptr)) return MPX_EINVAL;
    const bool given = coef_off_host != nullptr;
    std::vector<int> deg(batch), order(batch);
    std::vector<long long> coff(batch + 1), roff(batch + 1);
    coff[0] = given ? coef_off_host[0] : 0;
    roff[0] = given ? root_off_host[0] : 0;
    if (coff[0] < 0 || roff[0] < 0 || coff[0] > kDkMaxColumns || roff[0] > kDkMaxColumns)
        return MPX_EINVAL;
    for (int64_t b = 0; b < batch; ++b) {
        if (degree_host[b] < 1) return MPX_EINVAL;
        deg[b] = degree_host[b];
        if (given) {
            // polynomial b owns columns [coef_off[b], coef_off[b+1]) and
            // [root_off[b], root_off[b+1]): room for its n + 1 coefficients and
            // n roots, no overlap with its neighbours
            const long long c1 = coef_off_host[b + 1], r1 = root_off_host[b + 1];
            if (c1 > kDkMaxColumns || r1 > kDkMaxColumns || c1 - coff[b] < (long long)deg[b] + 1 ||
                r1 - roff[b] < (long long)deg[b])
                return MPX_EINVAL;
            coff[b + 1] = c1;
            roff[b + 1] = r1;
        } else {
            coff[b + 1] = coff[b] + deg[b] + 1;
            roff[b + 1] = roff[b] + deg[b];
            if (coff[b + 1] > kDkMaxColumns) return MPX_EINVAL;
        }
        order[b] = (int)b;
    }
    // longest-processing-time order: descending n^2 (ties: index order)
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return deg[a] > deg[b]; });

    // Packed schedule for the 4-wave kernel.  A chunk (64 roots) of a degree-n
    // polynomial costs n per sweep.  Polynomials, in LPT order, are added to
    // the open job with each chunk going to the least-loaded wave (lowest wave
    // on ties); a job is closed when adding the next polynomial would lift its
    // heaviest wave above L, the largest polynomial's cost spread over the
    // four waves.  Before it is closed, its lighter waves take the smallest
    // polynomials not yet placed, as long as its heaviest wave does not grow.
    // Jobs are then ordered heaviest first.
    std::vector<int> job_off(1, 0), items;
    {
        const int W = kDkPackedWaves;
        long long L = 0;
        for (int b = 0; b < (int)batch; ++b) {
            const long long c = (deg[b] + 63) / 64;
            L = std::max(L, (c + W - 1) / W * deg[b]);
        }
        struct Job { long long heaviest; std::vector<int> it; };
        std::vector<Job> jobs;
        long long load[kDkPackedWaves] = {0, 0, 0, 0};
        std::vector<int> cur;
        std::vector<char> placed(batch, 0);
        auto place = [&](int b, long long* ld, std::vector<int>& out) {
            const int c = (deg[b] + 63) / 64;
            for (int ch = 0; ch < c; ++ch) {
                int w = 0;
                for (int v = 1; v < W; ++v)
                    if (ld[v] < ld[w]) w = v;
                ld[w] += deg[b];
                out.insert(out.end(), {b, ch, w});
            }
        };
        auto heaviest = [&](const long long* ld) { return *std::max_element(ld, ld + W); };
        auto close = [&]() {
            const long long H = heaviest(load);
            for (int k = (int)batch - 1; k >= 0; --k) {  // smallest polynomials first
                const int b = order[k];
                if (placed[b]) continue;
                long long trial[kDkPackedWaves];
                std::copy(load, load + W, trial);
                std::vector<int> add;
                place(b, trial, add);
                if (heaviest(trial) > H) break;
                placed[b] = 1;
                std::copy(trial, trial + W, load);
                cur.insert(cur.end(), add.begin(), add.end());
            }
            jobs.push_back({heaviest(load), cur});
            cur.clear();
            std::fill(load, load + W, 0LL);
        };
        for (int b : order) {
            if (placed[b]) continue;
            long long trial[kDkPackedWaves];
            std::copy(load, load + W, trial);
            std::vector<int> add;
            place(b, trial, add);
            if (!cur.empty() && heaviest(trial) > L) {
                close();
                std::fill(trial, trial + W, 0LL);
                add.clear();
                place(b, trial, add);
            }
            placed[b] = 1;
            std::copy(trial, trial + W, load);
            cur.insert(cur.end(), add.begin(), add.end());
        }
        if (!cur.empty()) close();
        std::stable_sort(jobs.begin(), jobs.end(),
                         [](const Job& a, const Job& b) { return a.heaviest > b.heaviest; });
        size_t n_items = 0;
        for (const Job& j : jobs) n_items += j.it.size() / 3;
        if (n_items > (size_t)(INT32_MAX / 4)) return MPX_ENOTSUP;  // int job offsets and indices
        for (const Job& j : jobs) {
            items.insert(items.end(), j.it.begin(), j.it.end());
            job_off.push_back((int)(items.size() / 3));
        }
    }

    int cus = 256;
    {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
    }
    // Lane-packed schedules, one per DK_LANES variant (slots: jobs resident at once)
    // (built side by side, one host thread per schedule)
    LaneSchedHost lsh[kDkLaneScheds];
    {
        bool ok[kDkLaneScheds];
        std::vector<std::thread> th;
        for (const DkVariant& v : kDkVariants) {
            if (v.kind != DK_LANES) continue;
            ok[v.sched] = false;
            const long long slots = std::max<long long>(1, (long long)cus * v.waves_cu / v.w);
            auto job = [&deg, &lsh, &ok, v, slots] {
                try {
                    ok[v.sched] = build_lane_sched(deg, v.w, v.lscale / 100.0, slots,
                                                   lsh[v.sched], v.stat != 0);
                } catch (...) {  // out of host memory: the plan fails, the process goes on
                    ok[v.sched] = false;
                }
            };
            try {
                th.emplace_back(job);
            } catch (...) {  // no thread available: build it here
                job();
            }
        }
        for (std::thread& t : th) t.join();
        for (const DkVariant& v : kDkVariants)
            if (v.kind == DK_LANES && !ok[v.sched]) return MPX_ENOTSUP;
    }

    auto* p = new (std::nothrow) mpx_plan_s();
    if (!p) return MPX_EDEVICE;
    p->prec = prec;
    p->K = prec_k_ar(prec);
    p->batch = (int)batch;
    p->iters = iters;
    p->flags = flags;
    p->total_coef = coff[batch];
    p->total_roots = roff[batch];
    p->cus = cus;
    for (int d : deg) p->max_degree = std::max(p->max_degree, d);
    p->variant = dk_start_variant(p);

    const size_t n_i = (size_t)batch, K = (size_t)p->K;
    const size_t sz_order = n_i * sizeof(int), sz_deg = n_i * sizeof(int);
    const size_t sz_off = (n_i + 1) * sizeof(long long);
    const size_t sz_m = 2 * K * (size_t)std::max<long long>(p->total_coef, 1) * sizeof(double);
    const size_t sz_z = 2 * K * (size_t)std::max<long long>(p->total_roots, 1) * sizeof(double);
    const size_t sz_jo = job_off.size() * sizeof(int), sz_it = std::max<size_t>(items.size(), 1) * sizeof(int);
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const size_t total = al(sz_order) + al(sz_deg) + 2 * al(sz_off) + al(sz_m) + al(sz_z) + 256 +
                         al(sz_jo) + al(sz_it);
    if (hipMalloc(&p->dev, total) != hipSuccess) { delete p; return MPX_EDEVICE; }
    char* c = (char*)p->dev;
    auto take = [&](size_t v) { char* r = c; c += al(v); return r; };
    int* d_order = (int*)take(sz_order);
    int* d_deg = (int*)take(sz_deg);
    long long* d_coff = (long long*)take(sz_off);
    long long* d_roff = (long long*)take(sz_off);
    double* d_m = (double*)take(sz_m);
    double* d_z = (double*)take(sz_z);
    int* d_cnt = (int*)take(256);
    int* d_jo = (int*)take(sz_jo);
    int* d_it = (int*)take(sz_it);
    hipError_t e = hipSuccess;
    if (batch > 0) {
        e = hipMemcpy(d_order, order.data(), sz_order, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(d_deg, deg.data(), sz_deg, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemcpy(d_coff, coff.data(), sz_off, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_roff, roff.data(), sz_off, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(d_jo, job_off.data(), sz_jo, hipMemcpyHostToDevice);
    if (e == hipSuccess && !items.empty())
        e = hipMemcpy(d_it, items.data(), items.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) { (void)hipFree(p->dev); delete p; return MPX_EDEVICE; }
    const long long psm = std::max<long long>(p->total_coef, 1);
    const long long psz = std::max<long long>(p->total_roots, 1);
    p->d = DkPlanDev{d_order, d_deg, d_coff, d_roff, d_m, d_m + K * psm, d_z, d_z + K * psz,
                     d_cnt, psm, psz, d_jo, d_it, (int)(job_off.size() - 1)};
    for (int i = 0; i < kDkLaneScheds; ++i) {
        const LaneSchedHost& h = lsh[i];
        const size_t b_wo = h.wave_off.size() * sizeof(int), b_il = std::max<size_t>(h.item_len.size(), 1) * sizeof(int);
        const size_t b_ln = std::max<size_t>(h.lanes.size(), 2) * sizeof(int);
        const size_t b_po = h.poly_off.size() * sizeof(int), b_pl = std::max<size_t>(h.polys.size(), 1) * sizeof(int);
        const size_t b_wg = std::max<size_t>(h.wg_off.size(), 1) * sizeof(int);
        if (hipMalloc(&p->lane_dev[i], al(b_wo) + al(b_il) + al(b_ln) + al(b_po) + al(b_pl) + al(b_wg)) != hipSuccess) {
            mpx_plan_destroy(p);
            return MPX_EDEVICE;
        }
        c = (char*)p->lane_dev[i];
        int* wo = (int*)take(b_wo);
        int* il = (int*)take(b_il);
        int2* ln = (int2*)take(b_ln);
        int* po = (int*)take(b_po);
        int* pl = (int*)take(b_pl);
        int* wg = (int*)take(b_wg);
        e = hipMemcpy(wo, h.wave_off.data(), b_wo, hipMemcpyHostToDevice);
        if (e == hipSuccess && !h.item_len.empty())
            e = hipMemcpy(il, h.item_len.data(), h.item_len.size() * sizeof(int), hipMemcpyHostToDevice);
        if (e == hipSuccess && !h.lanes.empty())
            e = hipMemcpy(ln, h.lanes.data(), h.lanes.size() * sizeof(int), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(po, h.poly_off.data(), b_po, hipMemcpyHostToDevice);
        if (e == hipSuccess && !h.polys.empty())
            e = hipMemcpy(pl, h.polys.data(), h.polys.size() * sizeof(int), hipMemcpyHostToDevice);
        if (e == hipSuccess && !h.wg_off.empty())
            e = hipMemcpy(wg, h.wg_off.data(), h.wg_off.size() * sizeof(int), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            mpx_plan_destroy(p);
            return MPX_EDEVICE;
        }
        const int nbins = h.wg_off.empty() ? 0 : (int)h.wg_off.size() - 1;
        p->lane[i] = DkLaneSched{wo, il, ln, po, pl, nbins ? wg : nullptr, h.njobs, nbins};
    }
    *out = p;
    return MPX_OK;
}

// Host allocation failures (the schedule's vectors, all made before the plan
// itself) end as MPX_EDEVICE: no exception crosses the C boundary.
extern "C" int mpx_polyroots_plan(mpx_plan* out, int prec, int64_t batch,
                                  const int32_t* degree_host, const int64_t* coef_off_host,
                                  const int64_t* root_off_host, int iters, uint32_t flags) {
    try {
        return polyroots_plan(out, prec, batch, degree_host, coef_off_host, root_off_host, iters,
                              flags);
    } catch (const std::bad_alloc&) {
        return MPX_EDEVICE;
    }
}



static int roots_check(mpx_plan p, const void* cre, const void* cim, int64_t psc, void* rre,
                       void* rim, int64_t psr) {
    if (!p) return MPX_EINVAL;
    if (p->batch == 0) return MPX_OK;
    if (!cre || !cim || !rre || !rim) return MPX_EINVAL;
    if (psc < p->total_coef || psr < p->total_roots) return MPX_EINVAL;
    // the roots are updated in place; they must not overlap the coefficients
    // or each other
    const uint64_t cb = vec_bytes(p->K, p->total_coef, psc), rb = vec_bytes(p->K, p->total_roots, psr);
    if (overlaps(rre, rb, cre, cb) || overlaps(rre, rb, cim, cb) || overlaps(rim, rb, cre, cb) ||
        overlaps(rim, rb, cim, cb) || overlaps(rre, rb, rim, rb))
        return MPX_EINVAL;
    return MPX_OK;
}

extern "C" int mpx_polyroots(mpx_plan p, const void* coef_re, const void* coef_im, int64_t psc,
                             void* roots_re, void* roots_im, int64_t psr, int32_t* status,
                             void* stream) {
    int st = roots_check(p, coef_re, coef_im, psc, roots_re, roots_im, psr);
    if (st) return st;
    if (p->batch == 0) return MPX_OK;
    if (status) {
        const uint64_t sb = (uint64_t)p->batch * sizeof(int32_t);
        const uint64_t cb = vec_bytes(p->K, p->total_coef, psc), rb = vec_bytes(p->K, p->total_roots, psr);
        if (overlaps(status, sb, coef_re, cb) || overlaps(status, sb, coef_im, cb) ||
            overlaps(status, sb, roots_re, rb) || overlaps(status, sb, roots_im, rb))
            return MPX_EINVAL;
    }
    hipStream_t s = as_stream(stream);
    // Inside a capture the caller already owns (its graph records these
    // launches), and without the graph flag or a stream, launch directly.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (s != nullptr && hipStreamIsCapturing(s, &cap) != hipSuccess) return MPX_EDEVICE;
    if (!(p->flags & MPX_DK_GRAPH) || s == nullptr || cap != hipStreamCaptureStatusNone)
        return launch_dk(p, p->variant, coef_re, coef_im, psc, roots_re, roots_im, psr, status, s);
    // Graph path: capture the launch sequence once per (buffers, stream, variant), replay after.
    const void* key[6] = {coef_re, coef_im, roots_re, roots_im, status, nullptr};
    bool same = p->exec && p->g_stream == s && p->g_variant == p->variant && p->g_ps[0] == psc &&
                p->g_ps[1] == psr;
    for (int i = 0; i < 6 && same; ++i) same = key[i] == p->g_key[i];
    if (!same) {
        if (p->exec) { (void)hipGraphExecDestroy(p->exec); p->exec = nullptr; }
        if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return MPX_EDEVICE;
        st = launch_dk(p, p->variant, coef_re, coef_im, psc, roots_re, roots_im, psr, status, s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (st || e != hipSuccess) { if (g) (void)hipGraphDestroy(g); return st ? st : MPX_EDEVICE; }
        if (hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return MPX_EDEVICE;
        }
        p->graph = g;
        for (int i = 0; i < 6; ++i) p->g_key[i] = key[i];
        p->g_stream = s;
        p->g_variant = p->variant;
        p->g_ps[0] = psc;
        p->g_ps[1] = psr;
    }
    return hipGraphLaunch(p->exec, s) == hipSuccess ? MPX_OK : MPX_EDEVICE;
}

extern "C" int mpx_polyroots_variant_count(void) { return kDkVariantCount; }

extern "C" int mpx_polyroots_get_variant(mpx_plan p) { return p ? p->variant : MPX_EINVAL; }

extern "C" int mpx_polyroots_set_variant(mpx_plan p, int variant) {
    if (!p || variant < 0 || variant >= kDkVariantCount) return MPX_EINVAL;
    p->variant = variant;
    return MPX_OK;
}

// Autotuner: run each launch variant for `iters_probe` iterations on a copy
// of the given start roots (the caller's roots are not modified), time it
// with HIP events, and keep the fastest in the plan.  Synchronises `stream`.
extern "C" int mpx_polyroots_autotune(mpx_plan p, const void* coef_re, const void* coef_im,
                                      int64_t psc, const void* roots_re, const void* roots_im,
                                      int64_t psr, int iters_probe, float* best_ms,
                                      void* stream) {
    int st = roots_check(p, coef_re, coef_im, psc, (void*)roots_re, (void*)roots_im, psr);
    if (st) return st;
    if (p->batch == 0 || iters_probe < 1) return MPX_EINVAL;
    hipStream_t s = as_stream(stream);
    const size_t plane = (size_t)p->total_roots * sizeof(double);
    double* tmp = nullptr;
    if (hipMalloc(&tmp, 2 * p->K * plane) != hipSuccess) return MPX_EDEVICE;
    double* tre = tmp;
    double* tim = tmp + (size_t)p->K * p->total_roots;
    EventPair ev;
    if (!ev.ok) {
        (void)hipFree(tmp);
        return MPX_EDEVICE;
    }
    const int saved_iters = p->iters;
    const unsigned saved_flags = p->flags;
    p->iters = iters_probe;
    p->flags &= ~(unsigned)MPX_DK_INIT;
    float t[kDkVariantCount];
    for (int v = 0; v < kDkVariantCount; ++v) t[v] = -1.f;
    // every trial starts from a copy of the caller's roots
    auto copy_in = [&]() {
        for (int c = 0; c < p->K; ++c)
            if (hipMemcpyAsync(tre + (size_t)c * p->total_roots, (const double*)roots_re + (size_t)c * psr,
                               plane, hipMemcpyDeviceToDevice, s) != hipSuccess ||
                hipMemcpyAsync(tim + (size_t)c * p->total_roots, (const double*)roots_im + (size_t)c * psr,
                               plane, hipMemcpyDeviceToDevice, s) != hipSuccess)
                return (int)MPX_EDEVICE;
        return (int)MPX_OK;
    };
    // the engine clock ramps up under load: run the current variant first
    st = copy_in();
    if (!st)
        st = warm_clock(ev, s, [&] {
            return launch_dk(p, p->variant, coef_re, coef_im, psc, tre, tim, p->total_roots, nullptr, s);
        });
    // two rounds over all variants, each variant's faster round counts
    for (int round = 0; round < 2 && !st; ++round)
        for (int v = 0; v < kDkVariantCount && !st; ++v) {
            st = copy_in();
            if (st) break;
            if (!ev.start(s)) { st = MPX_EDEVICE; break; }
            st = launch_dk(p, v, coef_re, coef_im, psc, tre, tim, p->total_roots, nullptr, s);
            float ms = 0.f;
            if (st || !ev.stop(s) || !ev.elapsed(&ms)) { st = st ? st : MPX_EDEVICE; break; }
            if (t[v] < 0.f || ms < t[v]) t[v] = ms;
        }
    p->iters = saved_iters;
    p->flags = saved_flags;
    if (hipStreamSynchronize(s) != hipSuccess && !st) st = MPX_EDEVICE;  // before freeing tmp
    (void)hipFree(tmp);
    if (st) return st;
    // Leave the plan's current variant only for one at least 3 % faster: the
    // short probes rank variants within a few percent of each other in
    // either order from run to run, and a full-length solve at more resident
    // waves per CU has measured slower than the probes suggest.
    int best = 0;
    for (int v = 1; v < kDkVariantCount; ++v)
        if (t[v] < t[best]) best = v;
    const int cur = p->variant;
    const int keep = t[best] < 0.97f * t[cur] ? best : cur;
    p->variant = keep;
    tune_store(dk_tune_key(p), std::to_string(keep));
    if (best_ms) *best_ms = t[keep];
    return keep;
}
