// mp_arith.hpp -- device-side branch-free multicomponent arithmetic for gfx950.
//
// A K-component number is the unevaluated sum of K binary64 values (binary32
// for float-float), held in registers as mpn<T, K>.  Everything here is
// straight-line code: no branches, no selects, so a wavefront never diverges.
//
// Sources (T. Kouya, arXiv 2603.14926):
//   Section 2      -- the error-free transformations QuickTwoSum, TwoSum and
//                     the FMA form of TwoProd;
//   Section 2.1    -- DWBFAdd and DWBFMul (double-word, also on binary32);
//   Section 2.2    -- TWBFAdd and TWBFMul (triple-word);
//   Section 2.3    -- QWBFAdd and QDBFMul (quad-word).
// The operation sequences must equal the published ones exactly (results are
// compared bit for bit with an independent CPU implementation), so every
// step below keeps the published order and grouping.  Operation counts per
// call (adds + subs + muls + fmas): DD add 20, mul 9; TD add 57, mul 39;
// QD add 103, mul 106 (Tables 1 and 2).
//
// The library is compiled with -ffp-contract=off and without fast-math; the
// pragma below restates that for this header, so a*b + c is never fused
// except where TwoProd asks for an explicit fma.
#pragma once
#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace mpx {

template <typename T, int K>
struct mpn {
    T c[K];
};

using dd_t = mpn<double, 2>;
using td_t = mpn<double, 3>;
using qd_t = mpn<double, 4>;
using ff_t = mpn<float, 2>;

// ---------------------------------------------------------------- EFTs ----

// s + e == a + b exactly when |a| >= |b|.
template <typename T>
__device__ __forceinline__ void qts(T a, T b, T& s, T& e) {
    const T t = a + b;
    e = b - (t - a);
    s = t;
}

// s + e == a + b exactly for all a, b (6 operations).
template <typename T>
__device__ __forceinline__ void ts(T a, T b, T& s, T& e) {
    const T t = a + b;
    const T v = t - a;
    e = (a - (t - v)) + (b - v);
    s = t;
}

__device__ __forceinline__ double fma_rn(double a, double b, double c) {
    return __builtin_fma(a, b, c);
}
__device__ __forceinline__ float fma_rn(float a, float b, float c) {
    return __builtin_fmaf(a, b, c);
}

// p + e == a * b exactly (one multiply, one fma).
template <typename T>
__device__ __forceinline__ void tp(T a, T b, T& p, T& e) {
    const T t = a * b;
    e = fma_rn(a, b, -t);
    p = t;
}

// ------------------------------------------------------- double-word ----
// Used for DD (T = double) and for float-float (T = float).

template <typename T>
__device__ __forceinline__ mpn<T, 2> bf_add(const mpn<T, 2>& x, const mpn<T, 2>& y) {
    T s0, e0, s1, e1, u, eu;
    ts(x.c[0], y.c[0], s0, e0);
    ts(x.c[1], y.c[1], s1, e1);
    qts(s0, s1, u, eu);
    const T w = (e0 + e1) + eu;
    mpn<T, 2> r;
    qts(u, w, r.c[0], r.c[1]);
    return r;
}

template <typename T>
__device__ __forceinline__ mpn<T, 2> bf_mul(const mpn<T, 2>& x, const mpn<T, 2>& y) {
    T hi, lo;
    tp(x.c[0], y.c[0], hi, lo);
    const T cross = x.c[0] * y.c[1] + x.c[1] * y.c[0];
    mpn<T, 2> r;
    qts(hi, lo + cross, r.c[0], r.c[1]);
    return r;
}

// ------------------------------------------------------- triple-word ----

__device__ __forceinline__ td_t bf_add(const td_t& x, const td_t& y) {
    double a1, b1, c1, d1, e1, f1, a2, c2, d2, e2, a3, d3, b3, c3, c5, d5, b6, c6, b7;
    ts(x.c[0], y.c[0], a1, b1);
    ts(x.c[1], y.c[1], c1, d1);
    ts(x.c[2], y.c[2], e1, f1);
    qts(a1, c1, a2, c2);
    const double b2 = b1 + f1;
    ts(d1, e1, d2, e2);
    qts(a2, d2, a3, d3);
    ts(b2, c2, b3, c3);
    const double c4 = c3 + e2;
    ts(c4, d3, c5, d5);
    ts(b3, c5, b6, c6);
    td_t r;
    qts(a3, b6, r.c[0], b7);
    const double c7 = c6 + d5;
    qts(b7, c7, r.c[1], r.c[2]);
    return r;
}

__device__ __forceinline__ td_t bf_mul(const td_t& x, const td_t& y) {
    double a0, b0, c0, e0, d0, f0, c1, d1, b2, c2, a3, b3, b5, c5, b6;
    tp(x.c[0], y.c[0], a0, b0);
    tp(x.c[0], y.c[1], c0, e0);
    tp(x.c[1], y.c[0], d0, f0);
    const double g0 = x.c[0] * y.c[2];
    const double h0 = x.c[1] * y.c[1];
    const double i0 = x.c[2] * y.c[0];
    ts(c0, d0, c1, d1);
    const double e1 = e0 + f0;
    const double g1 = g0 + i0;
    ts(b0, c1, b2, c2);
    const double g2 = g1 + h0;
    qts(a0, b2, a3, b3);
    const double c3 = c2 + d1;
    const double e3 = e1 + g2;
    const double c4 = c3 + e3;
    qts(b3, c4, b5, c5);
    td_t r;
    qts(a3, b5, r.c[0], b6);
    qts(b6, c5, r.c[1], r.c[2]);
    return r;
}

// --------------------------------------------------------- quad-word ----

__device__ __forceinline__ qd_t bf_add(const qd_t& x, const qd_t& y) {
    double a1, b1, c1, d1, e1, f1, g1, h1, a2, c2, d2, e2, f2, g2, b3, g3, c3, d3, e3, f3;
    double a4, c4, d4, e4, b5, d5, b6, c6, d6, e6, a7, b7, c7, d7, b8, c8, b10, c10, d10, c11;
    ts(x.c[0], y.c[0], a1, b1);
    ts(x.c[1], y.c[1], c1, d1);
    ts(x.c[2], y.c[2], e1, f1);
    ts(x.c[3], y.c[3], g1, h1);
    qts(a1, c1, a2, c2);
    const double b2 = b1 + h1;
    ts(d1, e1, d2, e2);
    ts(f1, g1, f2, g2);
    ts(b2, g2, b3, g3);
    qts(c2, d2, c3, d3);
    ts(e2, f2, e3, f3);
    qts(a2, c3, a4, c4);
    qts(d3, e3, d4, e4);
    ts(b3, d4, b5, d5);
    const double e5 = e4 + f3;
    ts(b5, c4, b6, c6);
    ts(d5, e5, d6, e6);
    qts(a4, b6, a7, b7);
    qts(c6, d6, c7, d7);
    const double e8 = e6 + g3;
    qts(b7, c7, b8, c8);
    const double d9 = d7 + e8;
    qd_t r;
    qts(a7, b8, r.c[0], b10);
    qts(c8, d9, c10, d10);
    qts(b10, c10, r.c[1], c11);
    qts(c11, d10, r.c[2], r.c[3]);
    return r;
}

__device__ __forceinline__ qd_t bf_mul(const qd_t& x, const qd_t& y) {
    double a0, b0, c0, e0, d0, f0, g0, j0, h0, k0, i0, l0;
    double c1, d1, e1, f1, g1, i1, b2, c2, e2, h2, a3, b3, c3, d3, e3, g3;
    double c4, e4, c6, d6, b7, c7, b8, c8, d8, c9;
    tp(x.c[0], y.c[0], a0, b0);
    tp(x.c[0], y.c[1], c0, e0);
    tp(x.c[1], y.c[0], d0, f0);
    tp(x.c[0], y.c[2], g0, j0);
    tp(x.c[1], y.c[1], h0, k0);
    tp(x.c[2], y.c[0], i0, l0);
    const double m0 = x.c[0] * y.c[3];
    const double n0 = x.c[1] * y.c[2];
    const double o0 = x.c[2] * y.c[1];
    const double p0 = x.c[3] * y.c[0];
    ts(c0, d0, c1, d1);
    ts(e0, f0, e1, f1);
    ts(g0, i0, g1, i1);
    const double j1 = j0 + l0;
    const double m1 = m0 + p0;
    const double n1 = n0 + o0;
    ts(b0, c1, b2, c2);
    ts(e1, h0, e2, h2);
    const double f2 = f1 + j1;
    const double i2 = i1 + k0;
    const double m2 = m1 + n1;
    qts(a0, b2, a3, b3);
    qts(c2, d1, c3, d3);
    ts(e2, g1, e3, g3);
    const double f3 = f2 + m2;
    const double h3 = h2 + i2;
    ts(c3, e3, c4, e4);
    const double d4 = d3 + h3;
    const double f4 = f3 + g3;
    const double d5 = d4 + e4;
    ts(c4, d5, c6, d6);
    ts(b3, c6, b7, c7);
    const double d7 = d6 + f4;
    qd_t r;
    qts(a3, b7, r.c[0], b8);
    ts(c7, d7, c8, d8);
    ts(b8, c8, r.c[1], c9);
    qts(c9, d8, r.c[2], r.c[3]);
    return r;
}

// ------------------------------------------------------------ helpers ----

template <typename T, int K>
__device__ __forceinline__ mpn<T, K> mp_zero() {
    mpn<T, K> r;
#pragma unroll
    for (int i = 0; i < K; ++i) r.c[i] = T(0);
    return r;
}

template <typename T, int K>
__device__ __forceinline__ mpn<T, K> mp_from(T v) {
    mpn<T, K> r = mp_zero<T, K>();
    r.c[0] = v;
    return r;
}

template <typename T, int K>
__device__ __forceinline__ mpn<T, K> mp_neg(const mpn<T, K>& x) {
    mpn<T, K> r;
#pragma unroll
    for (int i = 0; i < K; ++i) r.c[i] = -x.c[i];
    return r;
}

// a - b = a + (-b) (Section 2: subtraction is negation of the operand).
template <typename T, int K>
__device__ __forceinline__ mpn<T, K> bf_sub(const mpn<T, K>& a, const mpn<T, K>& b) {
    return bf_add(a, mp_neg(b));
}

// Component-plane access: component c of element idx at base[c*ps + idx].
template <typename T, int K>
__device__ __forceinline__ mpn<T, K> mp_load(const T* __restrict__ base, long long ps,
                                             long long idx) {
    mpn<T, K> r;
#pragma unroll
    for (int i = 0; i < K; ++i) r.c[i] = base[i * ps + idx];
    return r;
}

template <typename T, int K>
__device__ __forceinline__ void mp_store(T* __restrict__ base, long long ps, long long idx,
                                         const mpn<T, K>& v) {
#pragma unroll
    for (int i = 0; i < K; ++i) base[i * ps + idx] = v.c[i];
}

// Lane-to-lane exchange of a whole K-component value (wave64 shuffles).
template <typename T, int K>
__device__ __forceinline__ mpn<T, K> mp_shfl_xor(const mpn<T, K>& v, int mask) {
    mpn<T, K> r;
#pragma unroll
    for (int i = 0; i < K; ++i) r.c[i] = __shfl_xor(v.c[i], mask, 64);
    return r;
}

}  // namespace mpx
