/*
 * mpx.h -- C ABI of libmpx: branch-free multicomponent (DD / TD / QD and
 * binary32 float-float) linear algebra and polynomial kernels for AMD
 * Instinct MI355X (gfx950).
 *
 * Method: T. Kouya, "Acceleration of multicomponent multiple-precision
 * arithmetic with branch-free algorithms and SIMD vectorization",
 * arXiv 2603.14926.  Each entry point names the passage defining its
 * operation.
 *
 * ---------------------------------------------------------------- layout --
 * A K-component number is the unevaluated sum of K binary64 values
 * (Section 2; K = 2 DD, 3 TD, 4 QD) or of two binary32 values (FF, the
 * "DS" double-word of Section 2.1).  Arrays are stored as K component
 * PLANES:  component c of vector element i lives at  base[c*ps + i],  of
 * row-major matrix element (r, col) at  base[c*ps + r*ld + col].  `ps` is
 * the plane stride in elements (>= the plane's extent).  A contiguous torch
 * tensor of shape (K, n) or (K, rows, cols), dtype float64 (float32 for FF),
 * is the canonical container.
 *
 * ------------------------------------------------------------ conventions --
 * All array pointers are DEVICE pointers unless the name ends in _host.
 * All calls are asynchronous on `stream` (a hipStream_t; NULL = the legacy
 * default stream) and return before the work completes.  Argument errors are
 * detected on the host before anything is launched and nothing is written;
 * a failed launch returns MPX_EDEVICE.  No call allocates device memory
 * except the plan constructors (mpx_polyroots_plan, mpx_gemm_batched_plan)
 * and mpx_polyroots_autotune (a scratch copy of the roots), and none
 * synchronises the device except the autotuners.  Sizes whose
 * launch grid would not fit (more than 2^31 - 1 GEMV rows or columns or
 * polynomials in a batch, more than 2^30 GEMM tiles) return MPX_ENOTSUP.
 * The caller
 * owns every buffer; the library keeps no pointer after a call returns
 * (plans keep the buffers they are given, see below).  Inputs are assumed
 * finite and normal (Section 2); NaN / Inf / subnormal handling is
 * unspecified.  Outputs may alias inputs only for mpx_add / mpx_mul (z may
 * equal x or y) and mpx_axpy (y in place).  The dot, GEMV and GEMM family
 * (plain, batched, Strassen, 3M, Ozaki), the polynomial evaluations (Horner,
 * Estrin, complex points, backward) and the root solver reject with
 * MPX_EINVAL an output whose memory range overlaps an input's or another
 * output's, or a workspace overlapping any operand (the root solver: roots
 * overlapping the coefficients or each other, a status array overlapping any
 * of them).  A range runs from a buffer's first element in plane 0 to its
 * last element in plane K - 1, so buffers whose planes interleave inside one
 * allocation count as overlapping.
 *
 * Determinism: every call is bitwise reproducible for the same arguments.
 * Elementwise ops, AXPY, GEMM (plain, batched, Strassen, 3M), Horner,
 * Estrin and the root solver perform, per output, exactly the operation
 * sequence of their sequential definition, so their results do not depend
 * on tile sizes or launch configuration.  Dot
 * and GEMV combine partial sums in a fixed tree whose shape depends only on
 * the problem size.
 */
#ifndef MPX_H
#define MPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Precision tag: the low byte is K, the number of components. */
typedef enum {
    MPX_DD = 2,       /* double-double,    ~106-bit significand */
    MPX_TD = 3,       /* triple-double,    ~159-bit */
    MPX_QD = 4,       /* quadruple-double, ~212-bit */
    MPX_FF = 0x102    /* float-float (binary32 double-word), ~48-bit */
} mpx_prec;

/* Arithmetic flags, OR-ed into MPX_DD / MPX_TD / MPX_QD.  Without a flag the
 * branch-free algorithms of Sections 2.1-2.3 are used.  With a flag the same
 * kernels run the conventional algorithms those sections compare against:
 *   MPX_NOBF      DWAdd (QD's "sloppy" addition) and DWMul for DD; TWAdd /
 *                 TWMul and their four-component forms, each ending in the
 *                 TW / QW renormalisation with data-dependent tests;
 *   MPX_NOBF_ACC  DD only: DWAccurateAdd in place of DWAdd.
 * Accepted by mpx_add, mpx_mul, mpx_axpy, mpx_dot, mpx_gemm (and its variant,
 * variant-count/name and autotune calls), mpx_gemm_strassen, mpx_polyval,
 * mpx_polyval_cplx (Horner) and mpx_polyroots_plan
 * (the plan then runs Durand-Kerner in that arithmetic); every other entry
 * point, and any flag on MPX_FF, returns MPX_EPREC.  Results of the
 * conventional operations are deterministic and meet the same error bounds
 * as the branch-free ones except that the sloppy DD addition is accurate
 * only relative to |a| + |b|, not to |a + b|. */
enum { MPX_NOBF = 0x1000, MPX_NOBF_ACC = 0x2000 };

typedef enum {
    MPX_OK = 0,
    MPX_EINVAL = -1,      /* bad size, stride, pointer or flag */
    MPX_EPREC = -2,       /* unknown precision tag, or not supported by this op */
    MPX_ENOTSUP = -3,     /* argument combination not supported */
    MPX_EWORKSPACE = -4,  /* workspace missing or smaller than mpx_workspace_size */
    MPX_EDEVICE = -5      /* HIP launch or runtime error */
} mpx_status;

int mpx_version(void);
const char *mpx_status_string(int status);

/* ------------------------------------------------------------ elementwise --
 * z_i = x_i + y_i  (DWBFAdd / TWBFAdd / QWBFAdd, Sections 2.1-2.3)
 * z_i = x_i * y_i  (DWBFMul / TWBFMul / QDBFMul)
 * n >= 0 elements; plane strides >= n.  z may alias x or y exactly. */
int mpx_add(int prec, int64_t n, const void *x, int64_t psx, const void *y, int64_t psy,
            void *z, int64_t psz, void *stream);
int mpx_mul(int prec, int64_t n, const void *x, int64_t psx, const void *y, int64_t psy,
            void *z, int64_t psz, void *stream);

/* y_i := alpha * x_i + y_i : one BF multiplication then one BF addition per
 * element (the vector layer the BF operations drive, Section 3).
 * alpha_host: K host values (double, or float for FF) read before return. */
int mpx_axpy(int prec, int64_t n, const void *alpha_host, const void *x, int64_t psx,
             void *y, int64_t psy, void *stream);

/* --------------------------------------------------------------- reductions --
 * Workspace sizes (bytes) for the calls that need one; op codes: */
enum { MPX_OP_DOT = 1, MPX_OP_GEMV = 2, MPX_OP_GEMM = 3, MPX_OP_OZAKI = 4, MPX_OP_CGEMM = 5,
       MPX_OP_STRASSEN = 6 };
/* For MPX_OP_DOT: m = n (vector length).  MPX_OP_GEMV: m, n = matrix shape,
 * k = trans.  MPX_OP_GEMM: 0.  MPX_OP_OZAKI: m, n, k = GEMM shape,
 * extra = number of slices.  MPX_OP_CGEMM: m, n, k = GEMM shape.
 * MPX_OP_STRASSEN: m, n, k = GEMM shape, extra = cutoff (arithmetic flags
 * allowed).  Returns 0 for invalid arguments. */
size_t mpx_workspace_size(int op, int prec, int64_t m, int64_t n, int64_t k, int64_t extra);

/* result[0..K-1] (device, K contiguous values) = sum_i x_i * y_i: the inner
 * product of the basic linear computations the paper accelerates (Section 1
 * and the BF operations of Section 2 inside the linear kernels of Section 3;
 * the paper benchmarks the matrix products built from them and defines no
 * separate inner-product routine, so the plain sum is the definition).
 * Per-thread partial sums are sequential BF multiply-adds; partials are
 * combined with BF additions in a fixed tree.  Error <= n * 2^-b *
 * sum |x_i y_i| with b = 104 / 155 / 208 (FF: 46).  ws: device workspace of
 * at least mpx_workspace_size(MPX_OP_DOT, prec, n, 0, 0, 0) bytes (0 for
 * n <= 256: one block, one launch; beyond, the block partials and a second
 * one-block launch that adds them). */
int mpx_dot(int prec, int64_t n, const void *x, int64_t psx, const void *y, int64_t psy,
            void *result, void *ws, size_t ws_bytes, void *stream);

/* mpx_dot without a workspace, for callers that cannot allocate (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels and result bits as mpx_dot, with the block partials in
 * a static device array of the library (32 KiB per GPU, enough for every n:
 * the dot never has more than 1024 partials; a larger need would return
 * MPX_EWORKSPACE).  No allocation of any kind.  Every call on one GPU shares
 * that array, so calls that overlap in time on one GPU (on different
 * streams, or from different threads) race and must be ordered by the
 * caller.  The array needs no clearing (each call writes every partial it
 * reads).  The stream must belong to the current device. */
int mpx_dot_noalloc(int prec, int64_t n, const void *x, int64_t psx, const void *y, int64_t psy,
                    void *result, void *stream);

/* y = op(A) x, the matrix-vector product of the same basic linear layer
 * (Sections 1 and 3; no separate definition in the paper, so the plain sums
 * are the definition).  A is an m x n row-major matrix with leading
 * dimension lda >= n and plane stride psA >= m*lda; op(A) = A (trans = 0, y
 * has m entries) or A^T (trans = 1, y has n entries).  Same error bound as
 * mpx_dot with the row length in place of n. */
int mpx_gemv(int prec, int trans, int64_t m, int64_t n, const void *A, int64_t lda,
             int64_t psA, const void *x, int64_t psx, void *y, int64_t psy, void *ws,
             size_t ws_bytes, void *stream);

/* C := op(A) op(B), the square-matrix product of Section 3.1 generalised to
 * m x n x k with transposes (no alpha / beta).  op(A) is m x k: A is m x k
 * row-major (transA = 0, lda >= k) or k x m (transA = 1, lda >= m); op(B) is
 * k x n: B is k x n (transB = 0, ldb >= n) or n x k (transB = 1, ldb >= k).
 * Every C_ij is computed as acc = 0; acc = acc + a_il * b_lj for l = 0..k-1
 * in order (the naive triple loop's per-entry sequence), so C is
 * independent of tiling.  C must not alias A or B. */
int mpx_gemm(int prec, int transA, int transB, int64_t m, int64_t n, int64_t k,
             const void *A, int64_t lda, int64_t psA, const void *B, int64_t ldb,
             int64_t psB, void *C, int64_t ldc, int64_t psC, void *stream);

/* Complex C := A B by the 3M method (Section 3.2, eq. cgemm_3m):
 *   C1 = Re(A) Re(B),  C2 = Im(A) Im(B),  C3 = (Re(A) + Im(A)) (Re(B) + Im(B)),
 *   Re(C) = C1 - C2,   Im(C) = (C3 - C1) - C2,
 * each real product by mpx_gemm (sequential k per entry), each sum an
 * elementwise BF addition.  Real and imaginary parts are separate plane sets
 * sharing lda / psA (A, m x k), ldb / psB (B, k x n) and ldc / psC (C, m x n).
 * ws: mpx_workspace_size(MPX_OP_CGEMM, prec, m, n, k, 0) bytes.  C must not
 * alias A or B. */
int mpx_cgemm_3m(int prec, int64_t m, int64_t n, int64_t k, const void *Are, const void *Aim,
                 int64_t lda, int64_t psA, const void *Bre, const void *Bim, int64_t ldb,
                 int64_t psB, void *Cre, void *Cim, int64_t ldc, int64_t psC, void *ws,
                 size_t ws_bytes, void *stream);

/* C := A B (A m x k, B k x n, row-major planes, no transposes) by Strassen's
 * recursion, the scheme Section 3.1 benchmarks (there with cutoff 32):
 *   M1 = (A11+A22)(B11+B22)  M2 = (A21+A22) B11  M3 = A11 (B12-B22)
 *   M4 = A22 (B21-B11)       M5 = (A11+A12) B22  M6 = (A21-A11)(B11+B12)
 *   M7 = (A12-A22)(B21+B22)
 *   C11 = ((M1+M4)-M5)+M7   C12 = M3+M5   C21 = M2+M4   C22 = ((M1-M2)+M3)+M6
 * A product splits while min(m, k, n) >= cutoff (cutoff >= 2); a dimension d
 * splits into ceil(d/2) + floor(d/2), trailing blocks zero-padded to the
 * leading block's shape; leaves are mpx_gemm (sequential k per entry); sums
 * are the multicomponent addition (a difference adds the negation).  DD, TD,
 * QD, with or without the arithmetic flags (not FF).  ws: at least
 * mpx_workspace_size(MPX_OP_STRASSEN, prec, m, n, k, cutoff) bytes (0 when
 * no split happens).  C must not overlap A, B or ws.  More than 8 levels of
 * recursion return MPX_ENOTSUP.  The error bound is norm-wise (Strassen's
 * method is not componentwise accurate). */
int mpx_gemm_strassen(int prec, int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                      int64_t psA, const void *B, int64_t ldb, int64_t psB, void *C, int64_t ldc,
                      int64_t psC, int64_t cutoff, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ batched GEMM --
 * count independent products C_p = A_p B_p (no transposes) of ragged shapes
 * m_p x k_p times k_p x n_p in one persistent launch: workgroups pull
 * (problem, tile) items, longest k first, from a counter and run the tile
 * routine of mpx_gemm, so every entry is bit-identical to mpx_gemm's (the
 * naive triple loop's sequence).  The tilings offered: mpx_gemm's (some
 * with the LDS-prefetching panel loop), 8 x 8 tiles computed by one wave
 * each, and mixed tilings with workgroup tiles over each product's interior
 * and, over its ragged edges, 8 x 8 wave tiles or waves of 64 consecutive
 * entries of each edge strip.  Operands are packed per component
 * plane:
 * A_p starts at element sum_{q<p} m_q k_q, row-major with ld = k_p; B_p at
 * sum_{q<p} k_q n_q (ld = n_p); C_p at sum_{q<p} m_q n_q (ld = n_p); plane
 * strides psA / psB / psC at least the totals.  The plan (host arrays copied
 * at creation; sizes up to 2^20 per dimension; DD, TD, QD or FF) owns a small
 * device schedule: create and destroy it outside graph capture.
 * mpx_gemm_batched launches two kernels (a counter reset and the persistent
 * kernel) on the stream, allocates nothing and may be captured in a HIP
 * graph; calls that overlap on one plan race on its counter.
 * mpx_gemm_batched_autotune times each tiling on the caller's buffers (C is
 * overwritten), after about 100 ms of warm-up calls of the plan's current
 * tiling, in two rounds over all tilings (a tiling's time is its faster
 * round), keeps the fastest in the plan and returns its index (it
 * synchronises the stream).  Errors as for mpx_gemm; the constructor also
 * returns MPX_ENOTSUP when a tiling's work list would pass 2^30 items and
 * MPX_EDEVICE when a host or device allocation fails. */
typedef struct mpx_gemm_plan_s *mpx_gemm_plan;
int mpx_gemm_batched_plan(mpx_gemm_plan *out, int prec, int64_t count, const int64_t *m_host,
                          const int64_t *n_host, const int64_t *k_host);
int mpx_gemm_batched(mpx_gemm_plan plan, const void *A, int64_t psA, const void *B,
                     int64_t psB, void *C, int64_t psC, void *stream);
int mpx_gemm_batched_variant_count(mpx_gemm_plan plan);
int mpx_gemm_batched_set_variant(mpx_gemm_plan plan, int variant);
int mpx_gemm_batched_autotune(mpx_gemm_plan plan, const void *A, int64_t psA, const void *B,
                              int64_t psB, void *C, int64_t psC, int reps, float *best_ms,
                              void *stream);
int mpx_gemm_plan_destroy(mpx_gemm_plan plan);

/* ---------------------------------------------------------- GEMM tuning --
 * The GEMM has several tilings ("variants"): LDS-staged register tiles
 * ("<p>_<TM>x<TN>_k<BK>", "_pf" reading the next step's operands early) and
 * row-wave tilings ("<p>_rw<R>_k<BK>": each wave owns R rows x 64 columns,
 * A through scalar loads, no LDS); the conventional arithmetic has the same
 * tilings under its own prefix (e.g. "dd_nobf_rw2_k4"); all produce the
 * same bits.  mpx_gemm picks one per (precision, transposes, log2 size
 * bucket): a tiling named in the environment variable MPX_GEMM_VARIANT
 * (comma-separated names; the first that belongs to the precision), else
 * the tuned choice for that bucket, else the largest tile that still gives
 * >= 2048 workgroups.  Tuned choices come from mpx_gemm_autotune in this
 * process and, when MPX_TUNE_CACHE names a file, from that file, which every
 * autotune rewrites (lines "<gfx arch> gemm <prec> <tA> <tB> <log2 m> <log2 n>
 * <log2 k> <tiling name>"; lines of other GPUs are kept).  MPX_TUNE=off
 * ignores tuned choices.  The root solver's plans use the same cache for
 * their launch variant ("<arch> dk <prec> <log2 batch> <log2 max degree>
 * <variant>"), with MPX_DK_VARIANT=<index> forcing one. */
int mpx_gemm_variant_count(int prec);
/* The variant mpx_gemm would use for this shape now (>= 0), or a negative
 * status for invalid arguments (m, n >= 1). */
int mpx_gemm_selected_variant(int prec, int transA, int transB, int64_t m, int64_t n, int64_t k);
/* Re-read the tune-cache file named by MPX_TUNE_CACHE (no file: empty),
 * replacing this process's tuned choices. */
int mpx_tune_reload(void);
const char *mpx_gemm_variant_name(int prec, int variant);   /* NULL if out of range */
/* mpx_gemm with an explicit variant; same arguments and errors otherwise. */
int mpx_gemm_variant(int prec, int variant, int transA, int transB, int64_t m, int64_t n,
                     int64_t k, const void *A, int64_t lda, int64_t psA, const void *B,
                     int64_t ldb, int64_t psB, void *C, int64_t ldc, int64_t psC,
                     void *stream);
/* Time every variant `reps` times on the given buffers (C is overwritten)
 * with HIP events on `stream`, after about 100 ms of warm-up calls (the
 * engine clock ramps up over tens of milliseconds of sustained work), in two
 * rounds over all variants (a variant's time is its faster round), skipping
 * the row-wave tilings ("_rw" names) for products with 4096 or more tiles of
 * 32 x 32, where they re-read B far more and run no faster; remember the fastest
 * (the size heuristic's tiling unless another is at least 1 % faster)
 * for this bucket and return its index (>= 0) or a negative status; *best_ms
 * (nullable) receives its mean time per call.  Synchronises `stream`; must not be called under graph
 * capture. */
int mpx_gemm_autotune(int prec, int transA, int transB, int64_t m, int64_t n, int64_t k,
                      const void *A, int64_t lda, int64_t psA, const void *B, int64_t ldb,
                      int64_t psB, void *C, int64_t ldc, int64_t psC, int reps,
                      float *best_ms, void *stream);
void mpx_gemm_autotune_reset(void);

/* ------------------------------------------------------------- Ozaki GEMM --
 * C := A B for DD matrices (K = 2 planes, transposes not supported) by an
 * Ozaki-style error-free split evaluated on the FP64 matrix cores.  The
 * paper lists the Ozaki scheme among its GEMM schemes (Section 3.1) without
 * defining it; the reading implemented:
 *   e_ib: for k-block b (kblk consecutive k indices) of row i of A,
 *        max_{l in b} |A_il[0]| < 2^{e_ib} (0 for a zero block); f_jb likewise
 *        for the k-blocks of the columns of B;
 *   slices: for p = 1..slices, m_p = rint(r1 * 2^{p*beta - e}),
 *        (r1, r2) := TwoSum(r1 - m_p 2^{e - p*beta}, r2), from (hi, lo), e
 *        the exponent of the element's block;
 *   level sums over k-blocks of kblk: S_g = sum_{p+q=g} sum_l mA_p mB_q,
 *        g = 2..slices+1, exact in binary64: |m_1| <= 2^beta and
 *        |m_p| <= 2^(beta-1) (p >= 2) bound |S_g| by
 *        kblk 2^(2 beta) (1 + max(0, slices-2)/4), which must be <= 2^53
 *        (else MPX_EINVAL; e.g. beta = 22 with kblk = 256 allows 6 slices,
 *        beta = 20 with kblk = 256 allows 12);
 *   C_ij = DWBFAdd accumulation (k-blocks ascending, g ascending) of
 *        (S_g 2^{e_ib + f_jb - g beta}, 0) of block b.
 * slices in 1..12, kblk a positive multiple of 16.  The result is
 * independent of the tiling and stage depth (bit-reproducible).  ws:
 * mpx_workspace_size(MPX_OP_OZAKI, MPX_DD, m, n, k, slices) bytes (the slice
 * planes of A and B and the block exponents; the size holds for every kblk). */
int mpx_gemm_ozaki_dd(int64_t m, int64_t n, int64_t k, const double *A, int64_t lda,
                      int64_t psA, const double *B, int64_t ldb, int64_t psB, double *C,
                      int64_t ldc, int64_t psC, int slices, int beta, int64_t kblk, void *ws,
                      size_t ws_bytes, void *stream);
/* Stage depth of the slice GEMM for later calls in this process: 0 = 8, 1 = 16
 * k values per LDS stage (results are identical). */
int mpx_gemm_ozaki_set_variant(int variant);

/* ------------------------------------------------------------ polynomials --
 * Real Horner evaluation (Section 4.1): y_b = p_b(x_b) = sum_i a_{b,i} x_b^i
 * for b < batch, all of degree deg >= 0.  Coefficient a_{b,i} (ascending
 * powers) is column b*(deg+1) + i of the K coefficient planes (psc >=
 * batch*(deg+1)); x, y are (K, batch) planes.  Per polynomial:
 * h = a_deg; h := h*x + a_i for i = deg-1 .. 0.  DD / TD / QD only. */
int mpx_polyval(int prec, int64_t batch, int64_t deg, const void *coef, int64_t psc,
                const void *x, int64_t psx, void *y, int64_t psy, void *stream);

/* The same values by Estrin's method (Section 4.1 compares Horner and
 * Estrin): the coefficient list of each polynomial is padded with zeros to
 * N = 2^L >= deg+1 entries; level l = 1..L replaces it by
 * c'_j = c_{2j} + c_{2j+1} X_{l-1} (BF multiply, then BF add), X_0 = x,
 * X_l = X_{l-1}^2.  One wave per polynomial up to deg 2047, one
 * four-wave workgroup per polynomial for deg 2048..8191 (at most 32
 * coefficients per lane either way); deg >= 8192 gives MPX_ENOTSUP.  Same
 * layout and errors as mpx_polyval. */
int mpx_polyval_estrin(int prec, int64_t batch, int64_t deg, const void *coef, int64_t psc,
                       const void *x, int64_t psx, void *y, int64_t psy, void *stream);

/* Real-coefficient polynomials at complex points (Section 4.1, the second
 * polynomial benchmark): y_b = p_b(x_b) with coef as for mpx_polyval (real
 * planes, batch x (deg+1)) and x, y given as real / imaginary plane sets
 * (xre, xim share psx; yre, yim share psy).  method 0 = Horner,
 * h = (a_n, 0), h := h x + a_i with the 4M complex product and a_i added to
 * the real part only (arithmetic flags accepted); method 1 = Estrin's list
 * halving, whose first level pairs real coefficients,
 * c' = (a_2j + a_2j+1 Re x, a_2j+1 Im x), later levels c' = c_2j + c_2j+1 X
 * with X := X^2 per level (branch-free only; one wave per polynomial up
 * to deg 1023, a four-wave workgroup for deg 1024..4095; deg >= 4096 gives
 * MPX_ENOTSUP).  Bit-identical to the sequential definitions; y must not
 * alias the inputs. */
int mpx_polyval_cplx(int prec, int64_t batch, int64_t deg, const void *coef, int64_t psc,
                     const void *xre, const void *xim, int64_t psx, void *yre, void *yim,
                     int64_t psy, int method, void *stream);

/* Reverse mode of mpx_polyval for L = sum_b gy_b p_b(x_b):
 *   gcoef_{b,i} = gy_b x_b^i  (t_0 = gy_b, t_{i+1} = t_i * x_b: the adjoint of
 *                               the Horner recurrence), same layout as coef;
 *   gx_b        = gy_b p_b'(x_b) (derivative recurrence d := d*x + h before
 *                               each h := h*x + a_i, d = 0 initially).
 * gcoef and gx are nullable (skipped when NULL). */
int mpx_polyval_backward(int prec, int64_t batch, int64_t deg, const void *coef, int64_t psc,
                         const void *x, int64_t psx, const void *gy, int64_t psg, void *gcoef,
                         int64_t psgc, void *gx, int64_t psgx, void *stream);

/* Batched Durand-Kerner (Weierstrass) root finder, Section 4.2:
 *   z_i <- z_i - q(z_i) / prod_{j != i} (z_i - z_j),  q = p / a_n  (monic),
 * all new roots of a sweep from the previous iterate (Jacobi), `iters` sweeps,
 * no early exit, complex K-component arithmetic (4M multiplication, division
 * as x conj(y) / |y|^2 with Newton's reciprocal).  Optional Aberth start
 * (MPX_DK_INIT): centre -c_{n-1}/n, radius r = max_i |n_nz c_i|^(1/(n-i)),
 * angles 2(i-1)pi/n + 3/(2n), evaluated in binary64 (device libm) from the
 * leading components of c_i = a_i/a_n; lower components start at zero.
 * Horner values and the root-difference product are carried with exact
 * power-of-two rescaling (no binary64 overflow at high degree).
 *
 * Layout: polynomial b has degree[b] >= 1; its coefficients a_0..a_n are
 * columns coef_off[b] .. coef_off[b] + n of the K planes of coef_re and
 * coef_im; its roots are columns root_off[b] .. root_off[b] + n - 1 of
 * roots_re / roots_im.  coef_off_host and root_off_host (host arrays of
 * batch + 1 entries, copied by the constructor) give the offsets; both NULL
 * means packed prefix sums (coef_off[0] = 0, coef_off[b+1] = coef_off[b] +
 * degree[b] + 1; root_off likewise with degree[b]).  Given offsets need
 * coef_off[0], root_off[0] >= 0, coef_off[b+1] - coef_off[b] >= degree[b] + 1
 * and root_off[b+1] - root_off[b] >= degree[b] (so polynomials never share a
 * column; gaps are allowed and left untouched), and at most 2^40 columns;
 * the planes then span coef_off[batch] and root_off[batch] columns.  Only
 * one of the two NULL is MPX_EINVAL.  roots_* hold the start values on entry
 * (unless MPX_DK_INIT) and the iterate on return; passing them back resumes
 * the iteration exactly.
 * status[b] (nullable) = 0 if all roots of b are finite, 1 otherwise (e.g.
 * coincident start values).
 *
 * A plan is created outside graph capture; it allocates its device
 * schedules (polynomials in descending-degree order for load balance, the
 * packed 4-wave jobs, and the lane-packed jobs of every lane-packed variant)
 * and working buffers (monic coefficients, second iterate) and frees them in
 * mpx_plan_destroy.  The constructor returns MPX_EINVAL for a degree below 1,
 * invalid offsets or unknown flags, MPX_ENOTSUP when a schedule's int
 * indices would overflow (about 2^24 items of 64 roots), MPX_EDEVICE when a
 * host or device allocation fails.  With
 * MPX_DK_GRAPH and a non-NULL stream, mpx_polyroots captures its launches
 * into a HIP graph on first use and replays it while buffers and stream stay
 * the same; on a stream the caller is already capturing it launches
 * directly, so the caller's graph records the launches.  One persistent
 * launch processes the whole batch.  Calls on one plan must not overlap. */
typedef struct mpx_plan_s *mpx_plan;
enum { MPX_DK_INIT = 1, MPX_DK_GRAPH = 2 };
int mpx_polyroots_plan(mpx_plan *out, int prec, int64_t batch, const int32_t *degree_host,
                       const int64_t *coef_off_host, const int64_t *root_off_host, int iters,
                       uint32_t flags);
int mpx_polyroots(mpx_plan plan, const void *coef_re, const void *coef_im, int64_t psc,
                  void *roots_re, void *roots_im, int64_t psr, int32_t *status, void *stream);
int mpx_plan_destroy(mpx_plan plan);
/* Launch-shape variants: roots per lane, resident waves per CU, and the
 * schedule, which is one of
 *   - one wave per polynomial;
 *   - packed: 4-wave jobs built by the plan, each holding whole polynomials
 *     whose 64-root chunks are spread over the waves to balance their loads;
 *   - lane-packed: 4-, 8-, 12- or 16-wave jobs whose roots are laid out lane
 *     by lane over 64-lane items, so roots of several polynomials share a
 *     wave and small polynomials fill lanes a larger one leaves idle; the
 *     jobs go to workgroups through a shared counter, heaviest first, or by
 *     a static assignment the plan computes from the jobs' step counts (each
 *     workgroup sweeps its own list).
 * Results do not depend on the variant.  A new plan uses lane-packed 16-wave
 * jobs (four waves per SIMD) on the static assignment, or the variant the
 * tune cache holds for its (precision, batch, largest degree) bucket, or
 * MPX_DK_VARIANT (see the GEMM tuning notes).  The autotuner runs each for
 * iters_probe sweeps on a private copy of the given start roots, after
 * about 100 ms of warm-up runs of the plan's current variant, in two
 * rounds over all variants (a variant's time is its faster round), switches
 * the plan to the fastest only when it beats the plan's current variant by
 * at least 3 %, and returns the index kept (or a negative status), which it
 * also records in the tune cache.  Synchronises; allocates. */
int mpx_polyroots_variant_count(void);
int mpx_polyroots_set_variant(mpx_plan plan, int variant);
int mpx_polyroots_get_variant(mpx_plan plan);   /* the plan's current variant */
int mpx_polyroots_autotune(mpx_plan plan, const void *coef_re, const void *coef_im, int64_t psc,
                           const void *roots_re, const void *roots_im, int64_t psr,
                           int iters_probe, float *best_ms, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MPX_H */
