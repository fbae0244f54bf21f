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
// TWBFAdd and TWBFMul (Section 2.2) and QWBFAdd and QDBFMul (Section 2.3).
// Each is a fixed network of error-free transformations: the inputs are
// first turned into exact terms (componentwise TwoSums, or the TwoProds of
// the leading cross products plus rounded products of the last order), and
// those terms are then folded towards the leading word, one order of
// magnitude at a time, with QuickTwoSum wherever the ordering of magnitudes
// is known and TwoSum elsewhere; the lowest terms are added without their
// errors.  Results are compared bit for bit with an independent CPU
// implementation, so the network (which term meets which, in which order,
// with which transformation) is the published one; the names are ours.  A
// name's digit is the order of magnitude it carries (0 = the leading word,
// 1 = about one unit roundoff below it, ...).

__device__ __forceinline__ td_t bf_add(const td_t& x, const td_t& y) {
    // Componentwise exact sums.
    double hi0, lo0, hi1, lo1, hi2, lo2;
    ts(x.c[0], y.c[0], hi0, lo0);
    ts(x.c[1], y.c[1], hi1, lo1);
    ts(x.c[2], y.c[2], hi2, lo2);
    // The leading sum takes in the order-1 head; the order-2 terms meet.
    double lead, spill1;
    qts(hi0, hi1, lead, spill1);
    const double low1 = lo0 + lo2;
    double mid2, err3;
    ts(lo1, hi2, mid2, err3);
    double spill2;
    qts(lead, mid2, lead, spill2);
    // Fold the order-1 terms, then what is left below them.
    double sum1, err2;
    ts(low1, spill1, sum1, err2);
    double sum2, err4;
    ts(err2 + err3, spill2, sum2, err4);
    double next, err5;
    ts(sum1, sum2, next, err5);
    // Renormalise into three words.
    td_t r;
    double carry;
    qts(lead, next, r.c[0], carry);
    qts(carry, err5 + err4, r.c[1], r.c[2]);
    return r;
}

__device__ __forceinline__ td_t bf_mul(const td_t& x, const td_t& y) {
    // Exact products of orders 0 and 1, rounded products of order 2.
    double p0, q1, p1a, q2a, p1b, q2b;
    tp(x.c[0], y.c[0], p0, q1);
    tp(x.c[0], y.c[1], p1a, q2a);
    tp(x.c[1], y.c[0], p1b, q2b);
    const double r2a = x.c[0] * y.c[2];
    const double r2b = x.c[1] * y.c[1];
    const double r2c = x.c[2] * y.c[0];
    // Order 1: the two cross products, then the leading product's error.
    double s1, s1err;
    ts(p1a, p1b, s1, s1err);
    const double errs2 = q2a + q2b;
    const double outer2 = r2a + r2c;
    double t1, t1err;
    ts(q1, s1, t1, t1err);
    const double prods2 = outer2 + r2b;
    double lead, spill;
    qts(p0, t1, lead, spill);
    // Everything of order 2, added without errors.
    const double sum2 = (t1err + s1err) + (errs2 + prods2);
    double w1, w2;
    qts(spill, sum2, w1, w2);
    // Renormalise into three words.
    td_t r;
    double carry;
    qts(lead, w1, r.c[0], carry);
    qts(carry, w2, r.c[1], r.c[2]);
    return r;
}

// --------------------------------------------------------- quad-word ----

__device__ __forceinline__ qd_t bf_add(const qd_t& x, const qd_t& y) {
    // Componentwise exact sums.
    double hi0, lo0, hi1, lo1, hi2, lo2, hi3, lo3;
    ts(x.c[0], y.c[0], hi0, lo0);
    ts(x.c[1], y.c[1], hi1, lo1);
    ts(x.c[2], y.c[2], hi2, lo2);
    ts(x.c[3], y.c[3], hi3, lo3);
    // First pass: each head meets the error of the order above it.
    double lead, spill1;
    qts(hi0, hi1, lead, spill1);
    const double deep = lo0 + lo3;
    double m2, m2err;
    ts(lo1, hi2, m2, m2err);
    double m3, m3err;
    ts(lo2, hi3, m3, m3err);
    double deep1, deep1err;
    ts(deep, m3err, deep1, deep1err);
    double u1, u1err;
    qts(spill1, m2, u1, u1err);
    double u2, u2err;
    ts(m2err, m3, u2, u2err);
    // Second pass.
    double spill2;
    qts(lead, u1, lead, spill2);
    double v2, v2err;
    qts(u1err, u2, v2, v2err);
    double w1, w1err;
    ts(deep1, v2, w1, w1err);
    const double tail3 = v2err + u2err;
    double w2, w2err;
    ts(w1, spill2, w2, w2err);
    double w3, w3err;
    ts(w1err, tail3, w3, w3err);
    // Third pass.
    double z1;
    qts(lead, w2, lead, z1);
    double z2, z2err;
    qts(w2err, w3, z2, z2err);
    const double tail4 = w3err + deep1err;
    double g1, g2;
    qts(z1, z2, g1, g2);
    const double g3 = z2err + tail4;
    // Renormalise into four words.
    qd_t r;
    double c1, c2, c3, c4;
    qts(lead, g1, r.c[0], c1);
    qts(g2, g3, c2, c3);
    qts(c1, c2, r.c[1], c4);
    qts(c4, c3, r.c[2], r.c[3]);
    return r;
}

__device__ __forceinline__ qd_t bf_mul(const qd_t& x, const qd_t& y) {
    // Exact products of orders 0-2 (pNN = x[i]*y[j] rounded, eNN its error),
    // rounded products of order 3.
    double p00, e00, p01, e01, p10, e10, p02, e02, p11, e11, p20, e20;
    tp(x.c[0], y.c[0], p00, e00);
    tp(x.c[0], y.c[1], p01, e01);
    tp(x.c[1], y.c[0], p10, e10);
    tp(x.c[0], y.c[2], p02, e02);
    tp(x.c[1], y.c[1], p11, e11);
    tp(x.c[2], y.c[0], p20, e20);
    const double p03 = x.c[0] * y.c[3];
    const double p12 = x.c[1] * y.c[2];
    const double p21 = x.c[2] * y.c[1];
    const double p30 = x.c[3] * y.c[0];
    // Pair up the terms of equal order.
    double a1, a1err;
    ts(p01, p10, a1, a1err);
    double a2, a2err;
    ts(e01, e10, a2, a2err);
    double b2, b2err;
    ts(p02, p20, b2, b2err);
    const double e3 = e02 + e20;
    const double o3 = p03 + p30;
    const double i3 = p12 + p21;
    // Order 1 meets the leading product's error; order 2 gathers.
    double s1, s1err;
    ts(e00, a1, s1, s1err);
    double s2, s2err;
    ts(a2, p11, s2, s2err);
    const double f3 = a2err + e3;
    const double g3 = b2err + e11;
    const double h3 = o3 + i3;
    double lead, spill1;
    qts(p00, s1, lead, spill1);
    double t2, t2err;
    qts(s1err, a1err, t2, t2err);
    double u2, u2err;
    ts(s2, b2, u2, u2err);
    const double k3 = f3 + h3;
    const double l3 = s2err + g3;
    // Order 2 total, then the order-3 remainder.
    double v2, v2err;
    ts(t2, u2, v2, v2err);
    const double m3 = t2err + l3;
    const double n3 = k3 + u2err;
    const double q3 = m3 + v2err;
    double w2, w3;
    ts(v2, q3, w2, w3);
    double z1, z2;
    ts(spill1, w2, z1, z2);
    const double rest3 = w3 + n3;
    // Renormalise into four words.
    qd_t r;
    double c1, c2, c3, c4;
    qts(lead, z1, r.c[0], c1);
    ts(z2, rest3, c2, c3);
    ts(c1, c2, r.c[1], c4);
    qts(c4, c3, r.c[2], r.c[3]);
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
