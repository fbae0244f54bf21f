/*
 * mpx_oracle.c -- plain, slow, sequential CPU oracle for branch-free
 * multicomponent (DD / TD / QD, and binary32 float-float) arithmetic.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may call, link or
 * load this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header or table with the HIP
 * library; the two are written independently from the paper.
 *
 * Paper: T. Kouya, "Acceleration of multicomponent multiple-precision
 * arithmetic with branch-free algorithms and SIMD vectorization"
 * (arXiv 2603.14926).  Every function names the passage it follows.
 *
 * Arithmetic model (Section 2, opening paragraphs): IEEE binary64 (binary32
 * for float-float) with round-to-nearest-even, every value a normalised float.
 * Build with  -O2 -ffp-contract=off -fno-fast-math  so that no a*b+c is fused
 * behind our back; the only fused operations are the explicit fma()/fmaf()
 * calls of TwoProd.  All loops run in a fixed sequential order; the optional
 * OpenMP loops parallelise only over independent outputs, so results do not
 * depend on the thread count.
 *
 * Number layout used by the array entry points: a multicomponent number is the
 * unevaluated sum of K doubles; component c of element i of a vector lives at
 * base[c*ps + i] ("component planes"), of a row-major matrix at
 * base[c*ps + row*ld + col].
 *
 * A build with -DMPXO_COUNT counts every floating-point operation by kind
 * (add, sub, mul, fma) so the operation counts printed in Tables 1 and 2 can
 * be checked.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#include <stdlib.h>

/* ------------------------------------------------------------------------ */
/* Operation counting (Tables 1 and 2 count additions, subtractions,         */
/* multiplications and FMAs separately; negating an FMA operand is free).    */
/* ------------------------------------------------------------------------ */
#ifdef MPXO_COUNT
static long long cnt_add, cnt_sub, cnt_mul, cnt_fma;
#define OP_ADD(a, b) (cnt_add++, (a) + (b))
#define OP_SUB(a, b) (cnt_sub++, (a) - (b))
#define OP_MUL(a, b) (cnt_mul++, (a) * (b))
#define OP_FMA(a, b, c) (cnt_fma++, fma((a), (b), (c)))
#define OP_FMAF(a, b, c) (cnt_fma++, fmaf((a), (b), (c)))
void orc_count_reset(void) { cnt_add = cnt_sub = cnt_mul = cnt_fma = 0; }
void orc_count_get(long long out[4]) {
    out[0] = cnt_add; out[1] = cnt_sub; out[2] = cnt_mul; out[3] = cnt_fma;
}
#else
#define OP_ADD(a, b) ((a) + (b))
#define OP_SUB(a, b) ((a) - (b))
#define OP_MUL(a, b) ((a) * (b))
#define OP_FMA(a, b, c) fma((a), (b), (c))
#define OP_FMAF(a, b, c) fmaf((a), (b), (c))
void orc_count_reset(void) {}
void orc_count_get(long long out[4]) { out[0] = out[1] = out[2] = out[3] = -1; }
#endif

#ifdef _OPENMP
#include <omp.h>
void orc_set_threads(int t) { omp_set_num_threads(t); }
int orc_get_threads(void) { return omp_get_max_threads(); }
#else
void orc_set_threads(int t) { (void)t; }
int orc_get_threads(void) { return 1; }
#endif

int orc_counting_build(void) {
#ifdef MPXO_COUNT
    return 1;
#else
    return 0;
#endif
}

/* ------------------------------------------------------------------------ */
/* Error-free transformations (Section 2: QuickTwoSum, TwoSum, TwoProd).     */
/* ------------------------------------------------------------------------ */

/* QuickTwoSum: s = fl(a+b) and its error, exact when |a| >= |b|. */
static void quick_two_sum(double a, double b, double *s, double *e) {
    double sum = OP_ADD(a, b);
    double back = OP_SUB(sum, a);
    *e = OP_SUB(b, back);
    *s = sum;
}

/* TwoSum: s = fl(a+b) and its error, exact for any a, b. */
static void two_sum(double a, double b, double *s, double *e) {
    double sum = OP_ADD(a, b);
    double v = OP_SUB(sum, a);
    double a_err = OP_SUB(a, OP_SUB(sum, v));
    double b_err = OP_SUB(b, v);
    *e = OP_ADD(a_err, b_err);
    *s = sum;
}

/* TwoProd with FMA: p = fl(a*b), e = a*b - p exactly. */
static void two_prod(double a, double b, double *p, double *e) {
    double prod = OP_MUL(a, b);
    *e = OP_FMA(a, b, -prod);
    *p = prod;
}

/* binary32 versions of the same three transformations (DS / float-float). */
static void quick_two_sum_f(float a, float b, float *s, float *e) {
    float sum = OP_ADD(a, b);
    float back = OP_SUB(sum, a);
    *e = OP_SUB(b, back);
    *s = sum;
}
static void two_sum_f(float a, float b, float *s, float *e) {
    float sum = OP_ADD(a, b);
    float v = OP_SUB(sum, a);
    float a_err = OP_SUB(a, OP_SUB(sum, v));
    float b_err = OP_SUB(b, v);
    *e = OP_ADD(a_err, b_err);
    *s = sum;
}
static void two_prod_f(float a, float b, float *p, float *e) {
    float prod = OP_MUL(a, b);
    *e = OP_FMAF(a, b, -prod);
    *p = prod;
}

/* ------------------------------------------------------------------------ */
/* Double-word (Section 2.1): DWBFAdd and DWBFMul (Zhang & Aiken), and the   */
/* QD-default DWMul which is the same operation sequence as DWBFMul once its */
/* final "QuickTwoProd" is read as QuickTwoSum.                              */
/* ------------------------------------------------------------------------ */

/* DWBFAdd: branch-free accurate double-word addition. */
static void dw_bf_add(const double a[2], const double b[2], double c[2]) {
    double g1, g1e, g2, g2e, g3, g3e, g4, g5;
    two_sum(a[0], b[0], &g1, &g1e);
    two_sum(a[1], b[1], &g2, &g2e);
    quick_two_sum(g1, g2, &g3, &g3e);
    g4 = OP_ADD(g1e, g2e);
    g5 = OP_ADD(g4, g3e);
    quick_two_sum(g3, g5, &c[0], &c[1]);
}

/* DWBFMul: all products first, then branch-free error handling. */
static void dw_bf_mul(const double a[2], const double b[2], double c[2]) {
    double p00, pe00, p01, p10, g1, g2;
    two_prod(a[0], b[0], &p00, &pe00);
    p01 = OP_MUL(a[0], b[1]);
    p10 = OP_MUL(a[1], b[0]);
    g1 = OP_ADD(p01, p10);
    g2 = OP_ADD(pe00, g1);
    quick_two_sum(p00, g2, &c[0], &c[1]);
}

/* The same two algorithms on binary32 components (float-float, "DS"). */
static void ff_bf_add(const float a[2], const float b[2], float c[2]) {
    float g1, g1e, g2, g2e, g3, g3e, g4, g5;
    two_sum_f(a[0], b[0], &g1, &g1e);
    two_sum_f(a[1], b[1], &g2, &g2e);
    quick_two_sum_f(g1, g2, &g3, &g3e);
    g4 = OP_ADD(g1e, g2e);
    g5 = OP_ADD(g4, g3e);
    quick_two_sum_f(g3, g5, &c[0], &c[1]);
}
static void ff_bf_mul(const float a[2], const float b[2], float c[2]) {
    float p00, pe00, p01, p10, g1, g2;
    two_prod_f(a[0], b[0], &p00, &pe00);
    p01 = OP_MUL(a[0], b[1]);
    p10 = OP_MUL(a[1], b[0]);
    g1 = OP_ADD(p01, p10);
    g2 = OP_ADD(pe00, g1);
    quick_two_sum_f(p00, g2, &c[0], &c[1]);
}

/* ------------------------------------------------------------------------ */
/* Triple-word (Section 2.2): TWBFAdd and TWBFMul; quad-word (Section 2.3):  */
/* QWBFAdd and QDBFMul.  Each turns its inputs into exact terms (TwoSum of   */
/* each component pair, or TwoProd of the leading cross products and plain   */
/* products of the last order) and folds those terms into the leading word   */
/* in the fixed order the paper gives: QuickTwoSum where the magnitudes are  */
/* known to be ordered, TwoSum elsewhere, plain additions for the lowest     */
/* terms.  The order of the steps is the paper's; the names are ours:        */
/* s[i], t[i] are the componentwise sums and their errors, pIJ / qIJ the     */
/* product x[i]*y[j] rounded and its error, and a trailing digit elsewhere   */
/* is the order of magnitude of the term (0 = the leading word).             */
/* ------------------------------------------------------------------------ */

static void tw_bf_add(const double x[3], const double y[3], double c[3]) {
    double s[3], t[3];
    double top, up1, mid2, low3, up2, acc1, low2, acc2, low4, acc, low5, carry;
    for (int i = 0; i < 3; ++i) two_sum(x[i], y[i], &s[i], &t[i]);
    quick_two_sum(s[0], s[1], &top, &up1);
    double rest1 = OP_ADD(t[0], t[2]);
    two_sum(t[1], s[2], &mid2, &low3);
    quick_two_sum(top, mid2, &top, &up2);
    two_sum(rest1, up1, &acc1, &low2);
    two_sum(OP_ADD(low2, low3), up2, &acc2, &low4);
    two_sum(acc1, acc2, &acc, &low5);
    quick_two_sum(top, acc, &c[0], &carry);
    quick_two_sum(carry, OP_ADD(low5, low4), &c[1], &c[2]);
}

static void tw_bf_mul(const double x[3], const double y[3], double c[3]) {
    double p00, q00, p01, q01, p10, q10;
    double cross1, cross_err, lead1, lead1_err, top, up, hi, lo, carry;
    two_prod(x[0], y[0], &p00, &q00);
    two_prod(x[0], y[1], &p01, &q01);
    two_prod(x[1], y[0], &p10, &q10);
    double p02 = OP_MUL(x[0], y[2]);
    double p11 = OP_MUL(x[1], y[1]);
    double p20 = OP_MUL(x[2], y[0]);
    two_sum(p01, p10, &cross1, &cross_err);
    double qsum2 = OP_ADD(q01, q10);
    double psum2 = OP_ADD(p02, p20);
    two_sum(q00, cross1, &lead1, &lead1_err);
    psum2 = OP_ADD(psum2, p11);
    quick_two_sum(p00, lead1, &top, &up);
    double part_a = OP_ADD(lead1_err, cross_err);
    double part_b = OP_ADD(qsum2, psum2);
    double order2 = OP_ADD(part_a, part_b);
    quick_two_sum(up, order2, &hi, &lo);
    quick_two_sum(top, hi, &c[0], &carry);
    quick_two_sum(carry, lo, &c[1], &c[2]);
}

static void qw_bf_add(const double x[4], const double y[4], double c[4]) {
    double s[4], t[4];
    double top, up1, m2, m2e, m3, m3e, deep, deep_e, u1, u1e, u2, u2e;
    double up2, v2, v2e, w1, w1e, w2, w2e, w3, w3e, up3, z2, z2e, h1, h2;
    double k1, k2, k3, k4;
    for (int i = 0; i < 4; ++i) two_sum(x[i], y[i], &s[i], &t[i]);
    /* first pass: each head meets the error of the order above it */
    quick_two_sum(s[0], s[1], &top, &up1);
    double bottom = OP_ADD(t[0], t[3]);
    two_sum(t[1], s[2], &m2, &m2e);
    two_sum(t[2], s[3], &m3, &m3e);
    two_sum(bottom, m3e, &deep, &deep_e);
    quick_two_sum(up1, m2, &u1, &u1e);
    two_sum(m2e, m3, &u2, &u2e);
    /* second pass */
    quick_two_sum(top, u1, &top, &up2);
    quick_two_sum(u1e, u2, &v2, &v2e);
    two_sum(deep, v2, &w1, &w1e);
    double tail3 = OP_ADD(v2e, u2e);
    two_sum(w1, up2, &w2, &w2e);
    two_sum(w1e, tail3, &w3, &w3e);
    /* third pass */
    quick_two_sum(top, w2, &top, &up3);
    quick_two_sum(w2e, w3, &z2, &z2e);
    double tail4 = OP_ADD(w3e, deep_e);
    quick_two_sum(up3, z2, &h1, &h2);
    double h3 = OP_ADD(z2e, tail4);
    /* renormalise into four words */
    quick_two_sum(top, h1, &c[0], &k1);
    quick_two_sum(h2, h3, &k2, &k3);
    quick_two_sum(k1, k2, &c[1], &k4);
    quick_two_sum(k4, k3, &c[2], &c[3]);
}

static void qd_bf_mul(const double x[4], const double y[4], double c[4]) {
    double p00, q00, p01, q01, p10, q10, p02, q02, p11, q11, p20, q20;
    double sum1, sum1e, qsum2, qsum2e, psum2, psum2e, n1, n1e, n2, n2e, top, up;
    double r2, r2e, g2, g2e, h2, h3, k1, k2, l1, l2, m1, m2;
    two_prod(x[0], y[0], &p00, &q00);
    two_prod(x[0], y[1], &p01, &q01);
    two_prod(x[1], y[0], &p10, &q10);
    two_prod(x[0], y[2], &p02, &q02);
    two_prod(x[1], y[1], &p11, &q11);
    two_prod(x[2], y[0], &p20, &q20);
    double p03 = OP_MUL(x[0], y[3]);
    double p12 = OP_MUL(x[1], y[2]);
    double p21 = OP_MUL(x[2], y[1]);
    double p30 = OP_MUL(x[3], y[0]);
    /* pair up terms of equal order */
    two_sum(p01, p10, &sum1, &sum1e);
    two_sum(q01, q10, &qsum2, &qsum2e);
    two_sum(p02, p20, &psum2, &psum2e);
    double qq3 = OP_ADD(q02, q20);
    double outer3 = OP_ADD(p03, p30);
    double inner3 = OP_ADD(p12, p21);
    /* order 1 meets the leading product's error; order 2 gathers */
    two_sum(q00, sum1, &n1, &n1e);
    two_sum(qsum2, p11, &n2, &n2e);
    double a3 = OP_ADD(qsum2e, qq3);
    double b3 = OP_ADD(psum2e, q11);
    double c3 = OP_ADD(outer3, inner3);
    quick_two_sum(p00, n1, &top, &up);
    quick_two_sum(n1e, sum1e, &r2, &r2e);
    two_sum(n2, psum2, &g2, &g2e);
    double d3 = OP_ADD(a3, c3);
    double e3 = OP_ADD(n2e, b3);
    /* order 2 in total, then the order-3 remainder */
    two_sum(r2, g2, &h2, &h3);
    double f3 = OP_ADD(r2e, e3);
    double g3 = OP_ADD(d3, g2e);
    f3 = OP_ADD(f3, h3);
    two_sum(h2, f3, &k1, &k2);
    two_sum(up, k1, &l1, &l2);
    double rest3 = OP_ADD(k2, g3);
    /* renormalise into four words */
    quick_two_sum(top, l1, &c[0], &m1);
    two_sum(l2, rest3, &k1, &k2);
    two_sum(m1, k1, &c[1], &m2);
    quick_two_sum(m2, k2, &c[2], &c[3]);
}

/* ------------------------------------------------------------------------ */
/* Conventional (not branch-free) operations: the "NoBF" baseline the paper  */
/* measures the BF algorithms against (Sections 2.1-2.3).                    */
/* ------------------------------------------------------------------------ */

/* DWAdd (Section 2.1): QD's default "sloppy" double-word addition; not
 * relatively accurate under cancellation. */
static void dw_add_sloppy(const double a[2], const double b[2], double c[2]) {
    double s, e;
    two_sum(a[0], b[0], &s, &e);
    e = OP_ADD(e, OP_ADD(a[1], b[1]));
    quick_two_sum(s, e, &c[0], &c[1]);
}

/* DWAccurateAdd (Section 2.1). */
static void dw_add_accurate(const double a[2], const double b[2], double c[2]) {
    double s1, s2, t1, t2;
    two_sum(a[0], b[0], &s1, &s2);
    two_sum(a[1], b[1], &t1, &t2);
    s2 = OP_ADD(s2, t1);
    quick_two_sum(s1, s2, &s1, &s2);
    s2 = OP_ADD(s2, t2);
    quick_two_sum(s1, s2, &c[0], &c[1]);
}

/* DWMul (Section 2.1), its final "QuickTwoProd" read as QuickTwoSum. */
static void dw_mul_conv(const double a[2], const double b[2], double c[2]) {
    double p1, p2;
    two_prod(a[0], b[0], &p1, &p2);
    p2 = OP_ADD(p2, OP_ADD(OP_MUL(a[0], b[1]), OP_MUL(a[1], b[0])));
    quick_two_sum(p1, p2, &c[0], &c[1]);
}

/* Renormalisation of K+1 roughly ordered doubles x[] into K components
 * (TWRenormalize for K = 3, QWRenormalize for K = 4; the paper names them
 * and their cost but does not print them).  The two-pass scheme of the QD
 * library's published algorithms (Hida, Li and Bailey): QuickTwoSum from the
 * least significant end upward, then from the top down, emitting a component
 * whenever the running sum leaves a non-zero error.  Once K-1 components are
 * out, what is left is added into the last one.  The data-dependent tests
 * are the branches that the BF algorithms remove. */
static void renormalize(int K, const double *x, double *c) {
    const int n = K + 1;
    double t[5], s, e;
    int k = 0;
    s = x[n - 1];
    for (int i = n - 2; i >= 0; i--) quick_two_sum(x[i], s, &s, &t[i + 1]);
    t[0] = s;
    for (int i = 1; i < n; i++) {
        if (k == K - 1) {
            s = OP_ADD(s, t[i]);
            continue;
        }
        quick_two_sum(s, t[i], &s, &e);
        if (e != 0.0) {
            c[k++] = s;
            s = e;
        }
    }
    c[k++] = s;
    for (; k < K; k++) c[k] = 0.0;
}

/* TWAdd (Section 2.2), as printed: componentwise TwoSums written out, the
 * error chain, then TWRenormalize.  "t0 + t1 + t2" is evaluated left to
 * right. */
static void tw_add_conv(const double a[3], const double b[3], double c[3]) {
    double s0, s1, s2, v0, v1, v2, u0, u1, u2, w0, w1, w2, t0, t1, t2, i1, i2, i3, r[4];
    s0 = OP_ADD(a[0], b[0]); s1 = OP_ADD(a[1], b[1]); s2 = OP_ADD(a[2], b[2]);
    v0 = OP_SUB(s0, a[0]); v1 = OP_SUB(s1, a[1]); v2 = OP_SUB(s2, a[2]);
    u0 = OP_SUB(s0, v0); u1 = OP_SUB(s1, v1); u2 = OP_SUB(s2, v2);
    w0 = OP_SUB(a[0], u0); w1 = OP_SUB(a[1], u1); w2 = OP_SUB(a[2], u2);
    u0 = OP_SUB(b[0], v0); u1 = OP_SUB(b[1], v1); u2 = OP_SUB(b[2], v2);
    t0 = OP_ADD(w0, u0); t1 = OP_ADD(w1, u1); t2 = OP_ADD(w2, u2);
    two_sum(s1, t0, &s1, &t0);
    two_sum(s2, t0, &i1, &i2);
    two_sum(t1, i1, &s2, &i3);
    two_sum(i2, i3, &t0, &t1);
    t0 = OP_ADD(OP_ADD(t0, t1), t2);
    r[0] = s0; r[1] = s1; r[2] = s2; r[3] = t0;
    renormalize(3, r, c);
}

/* The product terms shared by TWMul (Section 2.2) and its four-component
 * form: TwoProd of the O(1), O(eps) and O(eps^2) partial products, three
 * three-term sums, and the O(eps^3) error terms.  On return p0, p1, s0 are
 * the O(1), O(eps), O(eps^2) terms, *t0 the O(eps^3) sum (the printed last
 * TwoSum reads q3 where t0 is meant: read as TwoSum(t0, s1)), and lo[]
 * the three O(eps^4) pieces that only the four-component form keeps. */
static void mul_conv_terms(const double *a, const double *b, double r[4], double lo[3]) {
    double p0, q0, p1, q1, p2, q2, p3, q3, p4, q4, p5, q5;
    double i1, i2, i3, s0, t0, s1, t1, s2, e;
    two_prod(a[0], b[0], &p0, &q0);
    two_prod(a[0], b[1], &p1, &q1);
    two_prod(a[1], b[0], &p2, &q2);
    two_prod(a[0], b[2], &p3, &q3);
    two_prod(a[1], b[1], &p4, &q4);
    two_prod(a[2], b[0], &p5, &q5);
    two_sum(p1, p2, &i1, &i2); two_sum(q0, i1, &p1, &i3); two_sum(i2, i3, &p2, &q0);
    two_sum(p2, q1, &i1, &i2); two_sum(q2, i1, &p2, &i3); two_sum(i2, i3, &q1, &q2);
    two_sum(p3, p4, &i1, &i2); two_sum(p5, i1, &p3, &i3); two_sum(i2, i3, &p4, &p5);
    two_sum(p2, p3, &s0, &t0); two_sum(q1, p4, &s1, &t1); s2 = OP_ADD(q2, p5);
    two_sum(s1, t0, &s1, &t0); s2 = OP_ADD(s2, OP_ADD(t0, t1));
    two_sum(q0, q3, &q0, &q3); two_sum(q4, q5, &q4, &q5); two_sum(q0, q4, &t0, &t1);
    t1 = OP_ADD(t1, OP_ADD(q3, q5));
    two_sum(t0, s1, &t0, &e);
    r[0] = p0; r[1] = p1; r[2] = s0; r[3] = t0;
    lo[0] = s2; lo[1] = t1; lo[2] = e;
}

/* TWMul (Section 2.2): the terms above, then TWRenormalize of
 * (p0, p1, s0, t0); the O(eps^4) pieces are dropped. */
static void tw_mul_conv(const double a[3], const double b[3], double c[3]) {
    double r[4], lo[3];
    mul_conv_terms(a, b, r, lo);
    renormalize(3, r, c);
}

/* Quad-word addition, conventional (Section 2.3 names it; the QD library's
 * published "sloppy" addition): TWAdd with a fourth component -- TwoSum per
 * component, the error chain, QWRenormalize. */
static void qw_add_conv(const double a[4], const double b[4], double c[4]) {
    double s[4], t[4], i1, i2, i3, r[5];
    for (int i = 0; i < 4; i++) two_sum(a[i], b[i], &s[i], &t[i]);
    two_sum(s[1], t[0], &s[1], &t[0]);
    two_sum(s[2], t[0], &i1, &i2); two_sum(t[1], i1, &s[2], &i3); two_sum(i2, i3, &t[0], &t[1]);
    two_sum(s[3], t[0], &i1, &i2); two_sum(t[2], i1, &s[3], &i3); t[0] = OP_ADD(i2, i3);
    t[0] = OP_ADD(OP_ADD(t[0], t[1]), t[3]);
    r[0] = s[0]; r[1] = s[1]; r[2] = s[2]; r[3] = s[3]; r[4] = t[0];
    renormalize(4, r, c);
}

/* Quad-word multiplication, conventional: the TWMul terms plus the four
 * O(eps^3) partial products (rounded, added into the O(eps^3) term) and the
 * O(eps^4) remainder as the fifth input of QWRenormalize. */
static void qw_mul_conv(const double a[4], const double b[4], double c[4]) {
    double r[5], lo[3], p6;
    mul_conv_terms(a, b, r, lo);
    p6 = OP_ADD(OP_ADD(OP_MUL(a[0], b[3]), OP_MUL(a[1], b[2])),
                OP_ADD(OP_MUL(a[2], b[1]), OP_MUL(a[3], b[0])));
    r[3] = OP_ADD(r[3], p6);
    r[4] = OP_ADD(lo[0], OP_ADD(lo[1], lo[2]));
    renormalize(4, r, c);
}

/* Arithmetic used by every K-generic routine below: 0 = branch-free (the
 * paper's BF algorithms), 1 = conventional with the sloppy DWAdd, 2 =
 * conventional with DWAccurateAdd (TD and QD as 1). */
static int g_arith = 0;
void orc_set_arith(int a) { g_arith = a; }
int orc_get_arith(void) { return g_arith; }

void orc_renormalize(int K, const double *x, double *c) { renormalize(K, x, c); }

/* ------------------------------------------------------------------------ */
/* K-generic dispatch: K = 2 (DD), 3 (TD), 4 (QD).                           */
/* ------------------------------------------------------------------------ */

static void mp_add(int K, const double *a, const double *b, double *c) {
    double t[4];
    if (g_arith == 0) {
        if (K == 2) dw_bf_add(a, b, t);
        else if (K == 3) tw_bf_add(a, b, t);
        else qw_bf_add(a, b, t);
    } else {
        if (K == 2) (g_arith == 2 ? dw_add_accurate : dw_add_sloppy)(a, b, t);
        else if (K == 3) tw_add_conv(a, b, t);
        else qw_add_conv(a, b, t);
    }
    memcpy(c, t, sizeof(double) * K);
}
static void mp_mul(int K, const double *a, const double *b, double *c) {
    double t[4];
    if (g_arith == 0) {
        if (K == 2) dw_bf_mul(a, b, t);
        else if (K == 3) tw_bf_mul(a, b, t);
        else qd_bf_mul(a, b, t);
    } else {
        if (K == 2) dw_mul_conv(a, b, t);
        else if (K == 3) tw_mul_conv(a, b, t);
        else qw_mul_conv(a, b, t);
    }
    memcpy(c, t, sizeof(double) * K);
}
static void mp_neg(int K, const double *a, double *c) {
    for (int i = 0; i < K; i++) c[i] = -a[i];
}
/* Subtraction is addition of the negated operand (Section 2). */
static void mp_sub(int K, const double *a, const double *b, double *c) {
    double nb[4];
    mp_neg(K, b, nb);
    mp_add(K, a, nb, c);
}
static void mp_zero(int K, double *c) { for (int i = 0; i < K; i++) c[i] = 0.0; }
static void mp_set_d(int K, double v, double *c) { mp_zero(K, c); c[0] = v; }
static void mp_ldexp(int K, const double *a, int e, double *c) {
    for (int i = 0; i < K; i++) c[i] = ldexp(a[i], e);
}

static void gather(int K, const double *base, int64_t ps, int64_t idx, double *v) {
    for (int c = 0; c < K; c++) v[c] = base[c * ps + idx];
}
static void scatter(int K, double *base, int64_t ps, int64_t idx, const double *v) {
    for (int c = 0; c < K; c++) base[c * ps + idx] = v[c];
}

/* Single-number entry points (used by the exact-arithmetic tests). */
void orc_op1(int K, int op, const double *a, const double *b, double *c) {
    if (op == 0) mp_add(K, a, b, c);
    else mp_mul(K, a, b, c);
}
void orc_ff_op1(int op, const float *a, const float *b, float *c) {
    float t[2];
    if (op == 0) ff_bf_add(a, b, t);
    else ff_bf_mul(a, b, t);
    c[0] = t[0]; c[1] = t[1];
}
void orc_eft(int which, double a, double b, double *s, double *e) {
    if (which == 0) quick_two_sum(a, b, s, e);
    else if (which == 1) two_sum(a, b, s, e);
    else two_prod(a, b, s, e);
}

/* ------------------------------------------------------------------------ */
/* Elementwise add / mul and AXPY (the vector layer driven by the BF ops).   */
/* ------------------------------------------------------------------------ */

void orc_add(int K, int64_t n, const double *x, int64_t psx, const double *y,
             int64_t psy, double *z, int64_t psz) {
    for (int64_t i = 0; i < n; i++) {
        double a[4], b[4], c[4];
        gather(K, x, psx, i, a);
        gather(K, y, psy, i, b);
        mp_add(K, a, b, c);
        scatter(K, z, psz, i, c);
    }
}
void orc_mul(int K, int64_t n, const double *x, int64_t psx, const double *y,
             int64_t psy, double *z, int64_t psz) {
    for (int64_t i = 0; i < n; i++) {
        double a[4], b[4], c[4];
        gather(K, x, psx, i, a);
        gather(K, y, psy, i, b);
        mp_mul(K, a, b, c);
        scatter(K, z, psz, i, c);
    }
}
/* y_i := alpha * x_i + y_i : one BF multiplication, then one BF addition. */
void orc_axpy(int K, int64_t n, const double *alpha, const double *x, int64_t psx,
              double *y, int64_t psy) {
    for (int64_t i = 0; i < n; i++) {
        double a[4], b[4], p[4], c[4];
        gather(K, x, psx, i, a);
        gather(K, y, psy, i, b);
        mp_mul(K, alpha, a, p);
        mp_add(K, p, b, c);
        scatter(K, y, psy, i, c);
    }
}

/* Dot product by its definition: acc = 0; acc := acc + x_i*y_i, i ascending. */
void orc_dot(int K, int64_t n, const double *x, int64_t psx, const double *y,
             int64_t psy, double *r) {
    double acc[4], a[4], b[4], p[4];
    mp_zero(K, acc);
    for (int64_t i = 0; i < n; i++) {
        gather(K, x, psx, i, a);
        gather(K, y, psy, i, b);
        mp_mul(K, a, b, p);
        mp_add(K, acc, p, acc);
    }
    memcpy(r, acc, sizeof(double) * K);
}

/* y := op(A) x with A an m x n row-major matrix; op(A) = A (trans = 0) or
 * A^T (trans = 1).  Each output is a sequential dot product. */
void orc_gemv(int K, int trans, int64_t m, int64_t n, const double *A, int64_t lda,
              int64_t psA, const double *x, int64_t psx, double *y, int64_t psy) {
    int64_t rows = trans ? n : m, len = trans ? m : n;
    for (int64_t r = 0; r < rows; r++) {
        double acc[4], a[4], b[4], p[4];
        mp_zero(K, acc);
        for (int64_t l = 0; l < len; l++) {
            int64_t idx = trans ? (l * lda + r) : (r * lda + l);
            gather(K, A, psA, idx, a);
            gather(K, x, psx, l, b);
            mp_mul(K, a, b, p);
            mp_add(K, acc, p, acc);
        }
        scatter(K, y, psy, r, acc);
    }
}

/* One entry of C = op(A) op(B) by the naive triple loop (Section 3.1): the
 * k index ascends, each step one BF multiplication and one BF addition. */
static void gemm_entry(int K, int tA, int tB, int64_t i, int64_t j, int64_t k,
                       const double *A, int64_t lda, int64_t psA, const double *B,
                       int64_t ldb, int64_t psB, double *acc) {
    double a[4], b[4], p[4];
    mp_zero(K, acc);
    for (int64_t l = 0; l < k; l++) {
        gather(K, A, psA, tA ? (l * lda + i) : (i * lda + l), a);
        gather(K, B, psB, tB ? (j * ldb + l) : (l * ldb + j), b);
        mp_mul(K, a, b, p);
        mp_add(K, acc, p, acc);
    }
}

void orc_gemm(int K, int tA, int tB, int64_t m, int64_t n, int64_t k, const double *A,
              int64_t lda, int64_t psA, const double *B, int64_t ldb, int64_t psB,
              double *C, int64_t ldc, int64_t psC) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; i++) {
        for (int64_t j = 0; j < n; j++) {
            double acc[4];
            gemm_entry(K, tA, tB, i, j, k, A, lda, psA, B, ldb, psB, acc);
            scatter(K, C, psC, i * ldc + j, acc);
        }
    }
}

/* Selected entries (rows[t], cols[t]) of op(A) op(B); out is K x cnt planes. */
void orc_gemm_entries(int K, int tA, int tB, int64_t k, const double *A, int64_t lda,
                      int64_t psA, const double *B, int64_t ldb, int64_t psB,
                      int64_t cnt, const int64_t *rows, const int64_t *cols,
                      double *out) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < cnt; t++) {
        double acc[4];
        gemm_entry(K, tA, tB, rows[t], cols[t], k, A, lda, psA, B, ldb, psB, acc);
        scatter(K, out, cnt, t, acc);
    }
}

/* Complex product by the 3M method (Section 3.2, eq. cgemm_3m):
 *   C1 = Re(A) Re(B),  C2 = Im(A) Im(B),
 *   C3 = (Re(A) + Im(A)) (Re(B) + Im(B)),
 *   Re(C) = C1 - C2,   Im(C) = (C3 - C1) - C2,
 * every real product by the naive triple loop and every sum elementwise with
 * the BF addition.  Matrices are row-major K-plane sets with ld = columns. */
void orc_cgemm_3m(int K, int64_t m, int64_t n, int64_t k, const double *Are,
                  const double *Aim, const double *Bre, const double *Bim, double *Cre,
                  double *Cim) {
    const int64_t psA = m * k, psB = k * n, psC = m * n;
    double *SA = (double *)malloc(sizeof(double) * K * psA);
    double *SB = (double *)malloc(sizeof(double) * K * psB);
    double *C1 = (double *)malloc(sizeof(double) * K * psC);
    double *C2 = (double *)malloc(sizeof(double) * K * psC);
    double *C3 = (double *)malloc(sizeof(double) * K * psC);
    orc_add(K, psA, Are, psA, Aim, psA, SA, psA);
    orc_add(K, psB, Bre, psB, Bim, psB, SB, psB);
    orc_gemm(K, 0, 0, m, n, k, Are, k, psA, Bre, n, psB, C1, n, psC);
    orc_gemm(K, 0, 0, m, n, k, Aim, k, psA, Bim, n, psB, C2, n, psC);
    orc_gemm(K, 0, 0, m, n, k, SA, k, psA, SB, n, psB, C3, n, psC);
    for (int64_t i = 0; i < psC; i++) {
        double c1[4], c2[4], c3[4], t[4], re[4], im[4];
        gather(K, C1, psC, i, c1);
        gather(K, C2, psC, i, c2);
        gather(K, C3, psC, i, c3);
        mp_sub(K, c1, c2, re);
        mp_sub(K, c3, c1, t);
        mp_sub(K, t, c2, im);
        scatter(K, Cre, psC, i, re);
        scatter(K, Cim, psC, i, im);
    }
    free(SA); free(SB); free(C1); free(C2); free(C3);
}

/* ---- float-float (binary32 double-word) versions of the same layer ---- */

void orc_ff_add(int64_t n, const float *x, int64_t psx, const float *y, int64_t psy,
                float *z, int64_t psz) {
    for (int64_t i = 0; i < n; i++) {
        float a[2] = {x[i], x[psx + i]}, b[2] = {y[i], y[psy + i]}, c[2];
        ff_bf_add(a, b, c);
        z[i] = c[0]; z[psz + i] = c[1];
    }
}
void orc_ff_mul(int64_t n, const float *x, int64_t psx, const float *y, int64_t psy,
                float *z, int64_t psz) {
    for (int64_t i = 0; i < n; i++) {
        float a[2] = {x[i], x[psx + i]}, b[2] = {y[i], y[psy + i]}, c[2];
        ff_bf_mul(a, b, c);
        z[i] = c[0]; z[psz + i] = c[1];
    }
}
void orc_ff_axpy(int64_t n, const float *alpha, const float *x, int64_t psx, float *y,
                 int64_t psy) {
    for (int64_t i = 0; i < n; i++) {
        float a[2] = {x[i], x[psx + i]}, b[2] = {y[i], y[psy + i]}, p[2], c[2];
        ff_bf_mul(alpha, a, p);
        ff_bf_add(p, b, c);
        y[i] = c[0]; y[psy + i] = c[1];
    }
}
void orc_ff_dot(int64_t n, const float *x, int64_t psx, const float *y, int64_t psy,
                float *r) {
    float acc[2] = {0.0f, 0.0f};
    for (int64_t i = 0; i < n; i++) {
        float a[2] = {x[i], x[psx + i]}, b[2] = {y[i], y[psy + i]}, p[2];
        ff_bf_mul(a, b, p);
        ff_bf_add(acc, p, acc);
    }
    r[0] = acc[0]; r[1] = acc[1];
}
void orc_ff_gemv(int trans, int64_t m, int64_t n, const float *A, int64_t lda,
                 int64_t psA, const float *x, int64_t psx, float *y, int64_t psy) {
    int64_t rows = trans ? n : m, len = trans ? m : n;
    for (int64_t r = 0; r < rows; r++) {
        float acc[2] = {0.0f, 0.0f};
        for (int64_t l = 0; l < len; l++) {
            int64_t idx = trans ? (l * lda + r) : (r * lda + l);
            float a[2] = {A[idx], A[psA + idx]}, b[2] = {x[l], x[psx + l]}, p[2];
            ff_bf_mul(a, b, p);
            ff_bf_add(acc, p, acc);
        }
        y[r] = acc[0]; y[psy + r] = acc[1];
    }
}
static void ff_gemm_entry(int tA, int tB, int64_t i, int64_t j, int64_t k,
                          const float *A, int64_t lda, int64_t psA, const float *B,
                          int64_t ldb, int64_t psB, float *acc) {
    acc[0] = acc[1] = 0.0f;
    for (int64_t l = 0; l < k; l++) {
        int64_t ia = tA ? (l * lda + i) : (i * lda + l);
        int64_t ib = tB ? (j * ldb + l) : (l * ldb + j);
        float a[2] = {A[ia], A[psA + ia]}, b[2] = {B[ib], B[psB + ib]}, p[2];
        ff_bf_mul(a, b, p);
        ff_bf_add(acc, p, acc);
    }
}
void orc_ff_gemm(int tA, int tB, int64_t m, int64_t n, int64_t k, const float *A,
                 int64_t lda, int64_t psA, const float *B, int64_t ldb, int64_t psB,
                 float *C, int64_t ldc, int64_t psC) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < n; j++) {
            float acc[2];
            ff_gemm_entry(tA, tB, i, j, k, A, lda, psA, B, ldb, psB, acc);
            C[i * ldc + j] = acc[0]; C[psC + i * ldc + j] = acc[1];
        }
}
void orc_ff_gemm_entries(int tA, int tB, int64_t k, const float *A, int64_t lda,
                         int64_t psA, const float *B, int64_t ldb, int64_t psB,
                         int64_t cnt, const int64_t *rows, const int64_t *cols,
                         float *out) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < cnt; t++) {
        float acc[2];
        ff_gemm_entry(tA, tB, rows[t], cols[t], k, A, lda, psA, B, ldb, psB, acc);
        out[t] = acc[0]; out[cnt + t] = acc[1];
    }
}

/* ------------------------------------------------------------------------ */
/* Real polynomial evaluation by Horner's method (Section 4.1) and its       */
/* reverse-mode derivative.                                                  */
/* Coefficients of polynomial b: a_i at coef[c*psc + b*(deg+1) + i].         */
/* ------------------------------------------------------------------------ */

/* p(x) = sum_i a_i x^i:  h = a_deg;  h := h*x + a_i for i = deg-1 .. 0. */
void orc_polyval(int K, int64_t batch, int64_t deg, const double *coef, int64_t psc,
                 const double *x, int64_t psx, double *y, int64_t psy) {
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < batch; b++) {
        const int64_t off = b * (deg + 1);
        double h[4], xv[4], a[4];
        gather(K, x, psx, b, xv);
        gather(K, coef, psc, off + deg, h);
        for (int64_t i = deg - 1; i >= 0; i--) {
            gather(K, coef, psc, off + i, a);
            mp_mul(K, h, xv, h);
            mp_add(K, h, a, h);
        }
        scatter(K, y, psy, b, h);
    }
}

/* Estrin's method (Section 4.1 compares it with Horner): the coefficient list
 * is padded with zeros to N = 2^L >= deg+1 entries; level l replaces the list
 * c by c'_j = c_{2j} + c_{2j+1} X_{l-1} (BF multiply, then BF add) with
 * X_0 = x and X_l = X_{l-1} X_{l-1}, until one entry, p(x), is left. */
void orc_polyval_estrin(int K, int64_t batch, int64_t deg, const double *coef, int64_t psc,
                        const double *x, int64_t psx, double *y, int64_t psy) {
    int64_t N = 1;
    while (N < deg + 1) N *= 2;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < batch; b++) {
        const int64_t off = b * (deg + 1);
        double *c = (double *)calloc((size_t)N * 4, sizeof(double));
        double X[4], t[4];
        for (int64_t i = 0; i <= deg; i++) gather(K, coef, psc, off + i, &c[4 * i]);
        gather(K, x, psx, b, X);
        for (int64_t len = N; len > 1; len /= 2) {
            for (int64_t j = 0; j < len / 2; j++) {
                mp_mul(K, &c[4 * (2 * j + 1)], X, t);
                mp_add(K, &c[4 * (2 * j)], t, &c[4 * j]);
            }
            mp_mul(K, X, X, X);
        }
        scatter(K, y, psy, b, &c[0]);
        free(c);
    }
}

/* Gradients of L = sum_b g_b p_b(x_b):
 *   dL/da_{b,i} = g_b x_b^i, by the adjoint of the Horner recurrence
 *                 (t = g_b; t := t*x_b per step, i ascending);
 *   dL/dx_b     = g_b p_b'(x_b), with p' from the derivative Horner
 *                 recurrence d := d*x + h (before h := h*x + a_i), d = 0 at start.
 * Either output pointer may be NULL. */
void orc_polyval_backward(int K, int64_t batch, int64_t deg, const double *coef,
                          int64_t psc, const double *x, int64_t psx, const double *g,
                          int64_t psg, double *gcoef, int64_t psgc, double *gx,
                          int64_t psgx) {
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < batch; b++) {
        const int64_t off = b * (deg + 1);
        double xv[4], gv[4], t[4];
        gather(K, x, psx, b, xv);
        gather(K, g, psg, b, gv);
        if (gcoef) {
            memcpy(t, gv, sizeof(double) * K);
            scatter(K, gcoef, psgc, off, t);
            for (int64_t i = 1; i <= deg; i++) {
                mp_mul(K, t, xv, t);
                scatter(K, gcoef, psgc, off + i, t);
            }
        }
        if (gx) {
            double h[4], d[4], a[4], r[4];
            mp_zero(K, d);
            gather(K, coef, psc, off + deg, h);
            for (int64_t i = deg - 1; i >= 0; i--) {
                gather(K, coef, psc, off + i, a);
                mp_mul(K, d, xv, d);
                mp_add(K, d, h, d);
                mp_mul(K, h, xv, h);
                mp_add(K, h, a, h);
            }
            mp_mul(K, gv, d, r);
            scatter(K, gx, psgx, b, r);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Complex multicomponent numbers, division via Newton's method (Section 2   */
/* says division is built from addition and multiplication by Newton's      */
/* method; the iteration below is the classical reciprocal iteration).       */
/* A complex number is two K-component numbers re[], im[].                   */
/* ------------------------------------------------------------------------ */

typedef struct { double re[4], im[4]; } cmp;

/* (a+bi)(c+di) = (ac - bd) + (ad + bc) i, four BF products, two BF sums. */
static void cmp_mul(int K, const cmp *x, const cmp *y, cmp *z) {
    double ac[4], bd[4], ad[4], bc[4];
    cmp r;
    mp_mul(K, x->re, y->re, ac);
    mp_mul(K, x->im, y->im, bd);
    mp_mul(K, x->re, y->im, ad);
    mp_mul(K, x->im, y->re, bc);
    mp_sub(K, ac, bd, r.re);
    mp_add(K, ad, bc, r.im);
    *z = r;
}
static void cmp_add(int K, const cmp *x, const cmp *y, cmp *z) {
    mp_add(K, x->re, y->re, z->re);
    mp_add(K, x->im, y->im, z->im);
}
static void cmp_sub(int K, const cmp *x, const cmp *y, cmp *z) {
    mp_sub(K, x->re, y->re, z->re);
    mp_sub(K, x->im, y->im, z->im);
}

/* Newton iterations for the reciprocal (doubling the correct bits each
 * time): y0 = 1/d_0 in binary64; DD needs one step, TD and QD two. */
static int newton_steps(int K) { return K == 2 ? 1 : 2; }
static void mp_recip(int K, const double *d, double *y) {
    double one[4], p[4], e[4], ye[4];
    mp_set_d(K, 1.0, one);
    mp_set_d(K, 1.0 / d[0], y);
    for (int it = 0; it < newton_steps(K); it++) {
        mp_mul(K, d, y, p);
        mp_sub(K, one, p, e);        /* e = 1 - d*y */
        mp_mul(K, y, e, ye);
        mp_add(K, y, ye, y);         /* y = y + y*e */
    }
}
void orc_recip(int K, const double *d, double *y) { mp_recip(K, d, y); }

/* x / y = x * conj(y) * (1 / |y|^2). */
static void cmp_div(int K, const cmp *x, const cmp *y, cmp *z) {
    double rr[4], ii[4], den[4], inv[4], t1[4], t2[4], nr[4], ni[4];
    mp_mul(K, y->re, y->re, rr);
    mp_mul(K, y->im, y->im, ii);
    mp_add(K, rr, ii, den);
    mp_recip(K, den, inv);
    mp_mul(K, x->re, y->re, t1);
    mp_mul(K, x->im, y->im, t2);
    mp_add(K, t1, t2, nr);          /* Re(x conj y) */
    mp_mul(K, x->im, y->re, t1);
    mp_mul(K, x->re, y->im, t2);
    mp_sub(K, t1, t2, ni);          /* Im(x conj y) */
    mp_mul(K, nr, inv, z->re);
    mp_mul(K, ni, inv, z->im);
}
void orc_cdiv(int K, const double *xr, const double *xi, const double *yr,
              const double *yi, double *zr, double *zi) {
    cmp x, y, z;
    memcpy(x.re, xr, 8 * K); memcpy(x.im, xi, 8 * K);
    memcpy(y.re, yr, 8 * K); memcpy(y.im, yi, 8 * K);
    cmp_div(K, &x, &y, &z);
    memcpy(zr, z.re, 8 * K); memcpy(zi, z.im, 8 * K);
}

/* Real-coefficient polynomial at complex arguments (Section 4.1, the second
 * polynomial benchmark).  Horner: h = (a_n, 0); h := h * z + a_i for
 * i = n-1 .. 0, the complex product in the 4M form above and the real
 * coefficient added to the real part only (the imaginary part is left as
 * is).  Coefficient planes as in orc_polyval; z and the result as separate
 * real / imaginary planes. */
void orc_polyval_cplx(int K, int64_t batch, int64_t deg, const double *coef, int64_t psc,
                      const double *xre, const double *xim, int64_t psx, double *yre,
                      double *yim, int64_t psy) {
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < batch; b++) {
        const int64_t off = b * (deg + 1);
        cmp z, h;
        double a[4];
        gather(K, xre, psx, b, z.re);
        gather(K, xim, psx, b, z.im);
        memset(&h, 0, sizeof(h));
        gather(K, coef, psc, off + deg, h.re);
        for (int64_t i = deg - 1; i >= 0; i--) {
            cmp_mul(K, &h, &z, &h);
            gather(K, coef, psc, off + i, a);
            mp_add(K, h.re, a, h.re);
        }
        scatter(K, yre, psy, b, h.re);
        scatter(K, yim, psy, b, h.im);
    }
}

/* Estrin's method at complex arguments: the coefficient list padded with
 * zeros to N = 2^L; the first level pairs real coefficients,
 * c'_j = (a_2j + a_{2j+1} x_re, a_{2j+1} x_im) (a real times a complex
 * number is two products); later levels are complex,
 * c'_j = c_2j + c_{2j+1} X with the 4M product and componentwise sums;
 * X := X^2 (4M) after every level. */
void orc_polyval_cplx_estrin(int K, int64_t batch, int64_t deg, const double *coef,
                             int64_t psc, const double *xre, const double *xim, int64_t psx,
                             double *yre, double *yim, int64_t psy) {
    int64_t N = 1;
    while (N < deg + 1) N *= 2;
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < batch; b++) {
        const int64_t off = b * (deg + 1);
        double *a = (double *)calloc((size_t)N * 4, sizeof(double));
        cmp *c = (cmp *)calloc((size_t)(N > 1 ? N / 2 : 1), sizeof(cmp));
        cmp X, t;
        for (int64_t i = 0; i <= deg; i++) gather(K, coef, psc, off + i, &a[4 * i]);
        gather(K, xre, psx, b, X.re);
        gather(K, xim, psx, b, X.im);
        if (N == 1) {
            memset(&c[0], 0, sizeof(cmp));
            memcpy(c[0].re, a, sizeof(double) * K);
        } else {
            for (int64_t j = 0; j < N / 2; j++) {
                double p[4];
                mp_mul(K, &a[4 * (2 * j + 1)], X.re, p);
                mp_add(K, &a[4 * (2 * j)], p, c[j].re);
                mp_mul(K, &a[4 * (2 * j + 1)], X.im, c[j].im);
            }
            cmp_mul(K, &X, &X, &X);
            for (int64_t len = N / 2; len > 1; len /= 2) {
                for (int64_t j = 0; j < len / 2; j++) {
                    cmp_mul(K, &c[2 * j + 1], &X, &t);
                    cmp_add(K, &c[2 * j], &t, &c[j]);
                }
                cmp_mul(K, &X, &X, &X);
            }
        }
        scatter(K, yre, psy, b, c[0].re);
        scatter(K, yim, psy, b, c[0].im);
        free(a);
        free(c);
    }
}

/* Exact power-of-two rescaling of a complex number so that the larger of its
 * leading components lies in [0.5, 1); the scale goes into *E.  It changes
 * no bits of the represented value beyond the exponent, so it only protects
 * Horner and the root-difference product from binary64 overflow.
 * down_only != 0 rescales only values of magnitude >= 1 (used by Horner, whose
 * additive terms c_k 2^{-E} must never be scaled up into overflow). */
static void cmp_rescale(int K, cmp *z, int64_t *E, int down_only) {
    double m = fmax(fabs(z->re[0]), fabs(z->im[0]));
    if (m == 0.0 || !isfinite(m)) return;
    int e;
    frexp(m, &e);
    if (down_only && e < 1) return;
    for (int c = 0; c < K; c++) {
        z->re[c] = ldexp(z->re[c], -e);
        z->im[c] = ldexp(z->im[c], -e);
    }
    *E += e;
}
static int clamp_exp(int64_t e) {
    return e > 100000 ? 100000 : (e < -100000 ? -100000 : (int)e);
}

/* ------------------------------------------------------------------------ */
/* Durand-Kerner (Weierstrass) simultaneous iteration, Section 4.2.          */
/* ------------------------------------------------------------------------ */

static void load_c(int K, const double *re, const double *im, int64_t ps, int64_t i,
                   cmp *z) {
    gather(K, re, ps, i, z->re);
    gather(K, im, ps, i, z->im);
}
static void store_c(int K, double *re, double *im, int64_t ps, int64_t i,
                    const cmp *z) {
    scatter(K, re, ps, i, z->re);
    scatter(K, im, ps, i, z->im);
}

/* Monic coefficients of q_n = p_n / a_n: c_i = a_i / a_n, i = 0..n-1. */
static void dk_monic(int K, int64_t n, const double *are, const double *aim,
                     int64_t psa, int64_t aoff, cmp *c) {
    cmp an, ai;
    load_c(K, are, aim, psa, aoff + n, &an);
    for (int64_t i = 0; i < n; i++) {
        load_c(K, are, aim, psa, aoff + i, &ai);
        cmp_div(K, &ai, &an, &c[i]);
    }
}

/* Aberth initial values (equation for z_i^(0)): centre -c_{n-1}/n, radius
 * r = max_i |n_nz c_i|^(1/(n-i)), angles 2(i-1)pi/n + 3/(2n).  Evaluated in
 * binary64 on the leading components; lower components start at zero. */
static void dk_aberth(int64_t n, const cmp *c, cmp *z) {
    int64_t nnz = 0;
    for (int64_t i = 0; i < n; i++)
        if (c[i].re[0] != 0.0 || c[i].im[0] != 0.0) nnz++;
    double r = 0.0;
    for (int64_t i = 0; i < n; i++) {
        double mag = hypot(c[i].re[0], c[i].im[0]) * (double)nnz;
        double t = pow(mag, 1.0 / (double)(n - i));
        if (t > r) r = t;
    }
    double cre = -c[n - 1].re[0] / (double)n;
    double cim = -c[n - 1].im[0] / (double)n;
    for (int64_t i = 0; i < n; i++) {
        double th = 2.0 * (double)i * M_PI / (double)n + 3.0 / (2.0 * (double)n);
        memset(&z[i], 0, sizeof(cmp));
        z[i].re[0] = cre + r * cos(th);
        z[i].im[0] = cim + r * sin(th);
    }
}

/* q(z) by Horner on the monic coefficients, kept as value * 2^E with E >= 0:
 * h = 1; h := h*z + c_k 2^{-E}, k = n-1 .. 0, rescaling h down after each step. */
static void dk_horner(int K, int64_t n, const cmp *c, const cmp *z, cmp *h, int64_t *E) {
    memset(h, 0, sizeof(cmp));
    h->re[0] = 1.0;
    *E = 0;
    for (int64_t k = n - 1; k >= 0; k--) {
        cmp t, ck;
        cmp_mul(K, h, z, &t);
        mp_ldexp(K, c[k].re, clamp_exp(-*E), ck.re);
        mp_ldexp(K, c[k].im, clamp_exp(-*E), ck.im);
        cmp_add(K, &t, &ck, h);
        cmp_rescale(K, h, E, 1);
    }
}

/* One Jacobi sweep: every new z_i is computed from the previous iterate:
 *   z_i := z_i - q(z_i) / prod_{j != i} (z_i - z_j), j ascending. */
static void dk_sweep(int K, int64_t n, const cmp *c, const cmp *z, cmp *znew) {
    for (int64_t i = 0; i < n; i++) {
        cmp q, P, d, w;
        int64_t E, F = 0;
        dk_horner(K, n, c, &z[i], &q, &E);
        memset(&P, 0, sizeof(cmp));
        P.re[0] = 1.0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i) continue;
            cmp_sub(K, &z[i], &z[j], &d);
            cmp_mul(K, &P, &d, &P);
            cmp_rescale(K, &P, &F, 0);
        }
        cmp_div(K, &q, &P, &w);
        mp_ldexp(K, w.re, clamp_exp(E - F), w.re);
        mp_ldexp(K, w.im, clamp_exp(E - F), w.im);
        cmp_sub(K, &z[i], &w, &znew[i]);
    }
}

/* Batched driver.  Polynomial b has degree deg[b]; its coefficients a_0..a_n
 * start at coef_off[b], its roots at root_off[b].  flags bit 0: compute the
 * Aberth start values first (otherwise the roots arrays hold the start).
 * status[b] = 0 if all roots are finite after the iterations, 1 otherwise. */
void orc_polyroots(int K, int64_t batch, const int32_t *deg, const int64_t *coef_off,
                   const int64_t *root_off, const double *are, const double *aim,
                   int64_t psc, double *zre, double *zim, int64_t psr, int iters,
                   int flags, int32_t *status) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t b = 0; b < batch; b++) {
        int64_t n = deg[b];
        cmp *c = (cmp *)calloc((size_t)n, sizeof(cmp));
        cmp *z = (cmp *)calloc((size_t)n, sizeof(cmp));
        cmp *zn = (cmp *)calloc((size_t)n, sizeof(cmp));
        dk_monic(K, n, are, aim, psc, coef_off[b], c);
        if (flags & 1) dk_aberth(n, c, z);
        else
            for (int64_t i = 0; i < n; i++) load_c(K, zre, zim, psr, root_off[b] + i, &z[i]);
        for (int it = 0; it < iters; it++) {
            dk_sweep(K, n, c, z, zn);
            cmp *t = z; z = zn; zn = t;
        }
        int bad = 0;
        for (int64_t i = 0; i < n; i++) {
            for (int q = 0; q < K; q++)
                if (!isfinite(z[i].re[q]) || !isfinite(z[i].im[q])) bad = 1;
            store_c(K, zre, zim, psr, root_off[b] + i, &z[i]);
        }
        if (status) status[b] = bad;
        free(c); free(z); free(zn);
    }
}

/* Monic coefficients alone (for tests of the division step). */
void orc_dk_monic(int K, int64_t n, const double *are, const double *aim, int64_t psa,
                  double *cre, double *cim, int64_t psc) {
    cmp *c = (cmp *)calloc((size_t)n, sizeof(cmp));
    dk_monic(K, n, are, aim, psa, 0, c);
    for (int64_t i = 0; i < n; i++) store_c(K, cre, cim, psc, i, &c[i]);
    free(c);
}

/* q(z) at given points (value and binary exponent), for residual tests. */
void orc_dk_horner(int K, int64_t n, const double *cre, const double *cim, int64_t psc,
                   int64_t npts, const double *zr, const double *zi, int64_t psz,
                   double *qr, double *qi, int64_t psq, int64_t *E) {
    cmp *c = (cmp *)calloc((size_t)n, sizeof(cmp));
    for (int64_t i = 0; i < n; i++) load_c(K, cre, cim, psc, i, &c[i]);
    for (int64_t t = 0; t < npts; t++) {
        cmp z, q;
        load_c(K, zr, zi, psz, t, &z);
        dk_horner(K, n, c, &z, &q, &E[t]);
        store_c(K, qr, qi, psq, t, &q);
    }
    free(c);
}

/* ------------------------------------------------------------------------ */
/* Ozaki-style error-free splitting of DD matrices and the slice GEMM.       */
/* The paper only names the Ozaki scheme among its GEMM schemes (Section     */
/* 3.1); the reading implemented here:                                       */
/*  * each k-block b (kblk consecutive k indices) of row i of A gets the     */
/*    exponent e_ib with max over the block of |A_il[0]| < 2^{e_ib} (frexp   */
/*    of the maximum; 0 for an all-zero block); each k-block of column j of  */
/*    B gets f_jb the same way;                                              */
/*  * slice p = 1..s of an element (r1, r2) = (hi, lo) is the integer        */
/*    m_p = rint(r1 * 2^{p*beta - e}), e its block's exponent, then          */
/*    (r1, r2) := TwoSum(r1 - m_p 2^{e - p*beta}, r2): the residual stays    */
/*    exact;                                                                 */
/*  * level g = p + q collects sum_{p+q=g} sum_{l in block} mA_p mB_q in one */
/*    binary64 accumulator, exact because every term is an integer and, with */
/*    |m_1| <= 2^beta, |m_p| <= 2^(beta-1) for p >= 2, every partial sum is  */
/*    at most kblk 2^{2 beta} (1 + max(0, s-2)/4) <= 2^53 (the caller's      */
/*    parameter choice; the tests check it);                                 */
/*  * C_ij = sum over k-blocks b (ascending), levels g = 2..s+1 (ascending)  */
/*    of DWBFAdd(acc, (S_g * 2^{e_ib + f_jb - g*beta}, 0)).                  */
/* ------------------------------------------------------------------------ */

static int exp_of_max(double m) {
    if (m == 0.0) return 0;
    int e;
    frexp(m, &e);
    return e;
}

/* Split one DD value into s integer-valued slices with exponent e. */
static void split_value(double hi, double lo, int e, int s, int beta, double *m) {
    double r1 = hi, r2 = lo;
    for (int p = 1; p <= s; p++) {
        double q = rint(ldexp(r1, p * beta - e));
        double d = r1 - ldexp(q, e - p * beta);
        two_sum(d, r2, &r1, &r2);
        m[p - 1] = q;
    }
}

/* Block exponents and slices of A (m x k, row-major, DD planes): e_row is
 * m x nb (nb = ceil(k / kblk), row-major), slices are s planes of m x k
 * (plane stride m*k). */
void orc_ozaki_split_rows(int64_t m, int64_t k, const double *A, int64_t lda,
                          int64_t psA, int s, int beta, int64_t kblk, int32_t *e_row,
                          double *slices) {
    const int64_t nb = (k + kblk - 1) / kblk;
    for (int64_t i = 0; i < m; i++) {
        for (int64_t b = 0; b < nb; b++) {
            const int64_t l0 = b * kblk, l1 = l0 + kblk < k ? l0 + kblk : k;
            double mx = 0.0;
            for (int64_t l = l0; l < l1; l++) mx = fmax(mx, fabs(A[i * lda + l]));
            int e = exp_of_max(mx);
            e_row[i * nb + b] = e;
            for (int64_t l = l0; l < l1; l++) {
                double sl[64];
                split_value(A[i * lda + l], A[psA + i * lda + l], e, s, beta, sl);
                for (int p = 0; p < s; p++) slices[(int64_t)p * m * k + i * k + l] = sl[p];
            }
        }
    }
}
/* Block exponents and slices of B (k x n, row-major, DD planes): f_col is
 * n x nb (row-major), slices are s planes of k x n. */
void orc_ozaki_split_cols(int64_t k, int64_t n, const double *B, int64_t ldb,
                          int64_t psB, int s, int beta, int64_t kblk, int32_t *f_col,
                          double *slices) {
    const int64_t nb = (k + kblk - 1) / kblk;
    for (int64_t j = 0; j < n; j++) {
        for (int64_t b = 0; b < nb; b++) {
            const int64_t l0 = b * kblk, l1 = l0 + kblk < k ? l0 + kblk : k;
            double mx = 0.0;
            for (int64_t l = l0; l < l1; l++) mx = fmax(mx, fabs(B[l * ldb + j]));
            int f = exp_of_max(mx);
            f_col[j * nb + b] = f;
            for (int64_t l = l0; l < l1; l++) {
                double sl[64];
                split_value(B[l * ldb + j], B[psB + l * ldb + j], f, s, beta, sl);
                for (int p = 0; p < s; p++) slices[(int64_t)p * k * n + l * n + j] = sl[p];
            }
        }
    }
}

/* Entries (rows[t], cols[t]) of the Ozaki DD product, from split operands. */
void orc_ozaki_entries(int64_t m, int64_t n, int64_t k, int s, int beta, int64_t kblk,
                       const int32_t *e_row, const double *sa, const int32_t *f_col,
                       const double *sb, int64_t cnt, const int64_t *rows,
                       const int64_t *cols, double *out) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < cnt; t++) {
        int64_t i = rows[t], j = cols[t];
        const int64_t nb = (k + kblk - 1) / kblk;
        double acc[2] = {0.0, 0.0};
        for (int64_t l0 = 0; l0 < k; l0 += kblk) {
            int64_t l1 = l0 + kblk < k ? l0 + kblk : k;
            const int64_t b = l0 / kblk;
            for (int g = 2; g <= s + 1; g++) {
                double S = 0.0;
                for (int p = 1; p < g; p++) {
                    int q = g - p;
                    if (p > s || q > s) continue;
                    for (int64_t l = l0; l < l1; l++)
                        S += sa[(int64_t)(p - 1) * m * k + i * k + l] *
                             sb[(int64_t)(q - 1) * k * n + l * n + j];
                }
                double term[2] = {ldexp(S, e_row[i * nb + b] + f_col[j * nb + b] - g * beta), 0.0};
                dw_bf_add(acc, term, acc);
            }
        }
        out[t] = acc[0];
        out[cnt + t] = acc[1];
    }
}
