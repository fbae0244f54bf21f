// mp_conv.hpp -- device-side conventional ("NoBF") multicomponent arithmetic
// for gfx950, the baseline against which the paper measures its branch-free
// operations, and the compile-time selector that lets one kernel template
// run either arithmetic.
//
// Sources (T. Kouya, arXiv 2603.14926):
//   Section 2.1 -- DWAdd (QD's default "sloppy" addition), DWAccurateAdd and
//                  DWMul.  DWMul performs exactly the operations of DWBFMul
//                  (one addition has its operands swapped), so bf_mul serves
//                  both.
//   Section 2.2 -- TWAdd and TWMul, each ending in TWRenormalize.
//   Section 2.3 -- the quad-word operations, named there as QD's, ending in
//                  QWRenormalize; here they are the four-component forms of
//                  TWAdd / TWMul (the paper states that its TD arithmetic is
//                  QD arithmetic with the fourth component zero).
// The renormalisations are named but not printed in the paper; they follow
// the published two-pass scheme of the QD library (Hida, Li and Bailey):
// QuickTwoSum upward from the least significant term, then downward, emitting
// a component whenever the running sum leaves a non-zero error; after K-1
// components the remainder is added into the last one.  Those data-dependent
// tests are the branches the BF algorithms remove; on a GPU they become
// compares and per-lane selects (or divergent branches).
//
// Two readings: in TWMul the last TwoSum takes t0 (the O(eps^3) error sum)
// where the printed line has q3; the four-component multiplication adds the
// four O(eps^3) partial products, rounded, into that term and passes the
// O(eps^4) remainder as the fifth renormalisation input.
#pragma once
#include "mp_arith.hpp"

#pragma clang fp contract(off)

namespace mpx {

// Arithmetic selector (template argument of the kernels that accept it).
enum : int { AR_BF = 0, AR_NOBF = 1, AR_NOBF_ACC = 2 };

// ------------------------------------------------------- double-word ----

template <typename T>
__device__ __forceinline__ mpn<T, 2> cv_add_sloppy(const mpn<T, 2>& x, const mpn<T, 2>& y) {
    T s, e;
    ts(x.c[0], y.c[0], s, e);
    e = e + (x.c[1] + y.c[1]);
    mpn<T, 2> r;
    qts(s, e, r.c[0], r.c[1]);
    return r;
}

template <typename T>
__device__ __forceinline__ mpn<T, 2> cv_add_accurate(const mpn<T, 2>& x, const mpn<T, 2>& y) {
    T s1, s2, t1, t2;
    ts(x.c[0], y.c[0], s1, s2);
    ts(x.c[1], y.c[1], t1, t2);
    s2 = s2 + t1;
    qts(s1, s2, s1, s2);
    s2 = s2 + t2;
    mpn<T, 2> r;
    qts(s1, s2, r.c[0], r.c[1]);
    return r;
}

// ------------------------------------------------------ renormalise ----

// K+1 roughly ordered terms -> K non-overlapping components.  The loops are
// unrolled; the emission index k is a run-time value, so "component k := s"
// is written as a compare against every position it can take.
template <int K>
__device__ __forceinline__ mpn<double, K> cv_renorm(const double (&x)[K + 1]) {
    double t[K + 1];
    double s = x[K];
#pragma unroll
    for (int i = K - 1; i >= 0; --i) qts(x[i], s, s, t[i + 1]);
    t[0] = s;
    mpn<double, K> r = mp_zero<double, K>();
    int k = 0;
#pragma unroll
    for (int i = 1; i <= K; ++i) {
        if (k == K - 1) {
            s = s + t[i];
        } else {
            double e;
            qts(s, t[i], s, e);
            if (e != 0.0) {
#pragma unroll
                for (int j = 0; j < K - 1; ++j)
                    if (j == k) r.c[j] = s;
                ++k;
                s = e;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (j == k) r.c[j] = s;
    return r;
}

// ------------------------------------------------------- triple-word ----

// TWAdd: the three componentwise TwoSums written out, the error chain,
// "t0 + t1 + t2" left to right, then TWRenormalize.
__device__ __forceinline__ td_t cv_add(const td_t& a, const td_t& b) {
    const double s0 = a.c[0] + b.c[0], s1a = a.c[1] + b.c[1], s2a = a.c[2] + b.c[2];
    const double v0 = s0 - a.c[0], v1 = s1a - a.c[1], v2 = s2a - a.c[2];
    const double w0 = a.c[0] - (s0 - v0), w1 = a.c[1] - (s1a - v1), w2 = a.c[2] - (s2a - v2);
    const double u0 = b.c[0] - v0, u1 = b.c[1] - v1, u2 = b.c[2] - v2;
    double t0 = w0 + u0, t1 = w1 + u1;
    const double t2 = w2 + u2;
    double s1, s2, i1, i2, i3;
    ts(s1a, t0, s1, t0);
    ts(s2a, t0, i1, i2);
    ts(t1, i1, s2, i3);
    ts(i2, i3, t0, t1);
    t0 = (t0 + t1) + t2;
    const double x[4] = {s0, s1, s2, t0};
    return cv_renorm<3>(x);
}

// Partial-product terms shared by TWMul and its four-component form.  On
// return r = {O(1), O(eps), O(eps^2), O(eps^3)} terms and lo = the three
// O(eps^4) pieces (kept only by the four-component form).
__device__ __forceinline__ void cv_mul_terms(const double* a, const double* b, double (&r)[5],
                                             double (&lo)[3]) {
    double p0, q0, p1, q1, p2, q2, p3, q3, p4, q4, p5, q5;
    double i1, i2, i3, s0, t0, s1, t1, e;
    tp(a[0], b[0], p0, q0);
    tp(a[0], b[1], p1, q1);
    tp(a[1], b[0], p2, q2);
    tp(a[0], b[2], p3, q3);
    tp(a[1], b[1], p4, q4);
    tp(a[2], b[0], p5, q5);
    ts(p1, p2, i1, i2); ts(q0, i1, p1, i3); ts(i2, i3, p2, q0);
    ts(p2, q1, i1, i2); ts(q2, i1, p2, i3); ts(i2, i3, q1, q2);
    ts(p3, p4, i1, i2); ts(p5, i1, p3, i3); ts(i2, i3, p4, p5);
    ts(p2, p3, s0, t0);
    ts(q1, p4, s1, t1);
    double s2 = q2 + p5;
    ts(s1, t0, s1, t0);
    s2 = s2 + (t0 + t1);
    ts(q0, q3, q0, q3);
    ts(q4, q5, q4, q5);
    ts(q0, q4, t0, t1);
    t1 = t1 + (q3 + q5);
    ts(t0, s1, t0, e);
    r[0] = p0; r[1] = p1; r[2] = s0; r[3] = t0; r[4] = 0.0;
    lo[0] = s2; lo[1] = t1; lo[2] = e;
}

__device__ __forceinline__ td_t cv_mul(const td_t& a, const td_t& b) {
    double r[5], lo[3];
    cv_mul_terms(a.c, b.c, r, lo);
    const double x[4] = {r[0], r[1], r[2], r[3]};
    return cv_renorm<3>(x);
}

// --------------------------------------------------------- quad-word ----

__device__ __forceinline__ qd_t cv_add(const qd_t& a, const qd_t& b) {
    double s[4], t[4], i1, i2, i3;
#pragma unroll
    for (int i = 0; i < 4; ++i) ts(a.c[i], b.c[i], s[i], t[i]);
    ts(s[1], t[0], s[1], t[0]);
    ts(s[2], t[0], i1, i2); ts(t[1], i1, s[2], i3); ts(i2, i3, t[0], t[1]);
    ts(s[3], t[0], i1, i2); ts(t[2], i1, s[3], i3); t[0] = i2 + i3;
    t[0] = (t[0] + t[1]) + t[3];
    const double x[5] = {s[0], s[1], s[2], s[3], t[0]};
    return cv_renorm<4>(x);
}

__device__ __forceinline__ qd_t cv_mul(const qd_t& a, const qd_t& b) {
    double r[5], lo[3];
    cv_mul_terms(a.c, b.c, r, lo);
    const double p6 = (a.c[0] * b.c[3] + a.c[1] * b.c[2]) + (a.c[2] * b.c[1] + a.c[3] * b.c[0]);
    const double x[5] = {r[0], r[1], r[2], r[3] + p6, lo[0] + (lo[1] + lo[2])};
    return cv_renorm<4>(x);
}

// ------------------------------------------------------------ selector ----

template <int AR, typename T, int K>
__device__ __forceinline__ mpn<T, K> ar_add(const mpn<T, K>& a, const mpn<T, K>& b) {
    if constexpr (AR == AR_BF) return bf_add(a, b);
    else if constexpr (K == 2) {
        if constexpr (AR == AR_NOBF_ACC) return cv_add_accurate(a, b);
        else return cv_add_sloppy(a, b);
    } else return cv_add(a, b);
}

template <int AR, typename T, int K>
__device__ __forceinline__ mpn<T, K> ar_mul(const mpn<T, K>& a, const mpn<T, K>& b) {
    if constexpr (AR == AR_BF || K == 2) return bf_mul(a, b);
    else return cv_mul(a, b);
}

// a - b = a + (-b), as for the BF operations.
template <int AR, typename T, int K>
__device__ __forceinline__ mpn<T, K> ar_sub(const mpn<T, K>& a, const mpn<T, K>& b) {
    return ar_add<AR>(a, mp_neg(b));
}

}  // namespace mpx
