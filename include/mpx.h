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
 * except mpx_polyroots_plan, and none synchronises the device.  The caller
 * owns every buffer; the library keeps no pointer after a call returns
 * (plans keep the buffers they are given, see below).  Inputs are assumed
 * finite and normal (Section 2); NaN / Inf / subnormal handling is
 * unspecified.  Outputs may alias inputs only for mpx_add / mpx_mul (z may
 * equal x or y) and mpx_axpy (y in place).
 *
 * Determinism: every call is bitwise reproducible for the same arguments.
 * Elementwise ops, AXPY, GEMM, Horner and the root solver perform, per
 * output, exactly the operation sequence of the sequential definition, so
 * their results do not depend on tile sizes or launch configuration.  Dot
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
enum { MPX_OP_DOT = 1, MPX_OP_GEMV = 2, MPX_OP_GEMM = 3, MPX_OP_OZAKI = 4 };
/* For MPX_OP_DOT: m = n (vector length).  MPX_OP_GEMV: m, n = matrix shape,
 * k = trans.  MPX_OP_GEMM: 0.  MPX_OP_OZAKI: m, n, k = GEMM shape,
 * extra = number of slices.  Returns 0 for invalid arguments. */
size_t mpx_workspace_size(int op, int prec, int64_t m, int64_t n, int64_t k, int64_t extra);

/* result[0..K-1] (device, K contiguous values) = sum_i x_i * y_i.
 * Per-thread partial sums are sequential BF multiply-adds; partials are
 * combined with BF additions in a fixed tree.  Error <= n * 2^-b *
 * sum |x_i y_i| with b = 104 / 155 / 208 (FF: 46).  ws: device workspace of
 * at least mpx_workspace_size(MPX_OP_DOT, prec, n, 0, 0, 0) bytes. */
int mpx_dot(int prec, int64_t n, const void *x, int64_t psx, const void *y, int64_t psy,
            void *result, void *ws, size_t ws_bytes, void *stream);

/* y = op(A) x, A an m x n row-major matrix with leading dimension lda >= n
 * and plane stride psA >= m*lda; op(A) = A (trans = 0, y has m entries) or
 * A^T (trans = 1, y has n entries).  Same error bound as mpx_dot with the
 * row length in place of n. */
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

/* ---------------------------------------------------------- GEMM tuning --
 * The GEMM has several register/LDS tilings ("variants"); all produce the
 * same bits.  mpx_gemm picks one per (precision, transposes, log2 size
 * bucket): the autotuned choice if mpx_gemm_autotune ran for that bucket in
 * this process, else the largest tile that still gives >= 2048 workgroups. */
int mpx_gemm_variant_count(int prec);
const char *mpx_gemm_variant_name(int prec, int variant);   /* NULL if out of range */
/* mpx_gemm with an explicit variant; same arguments and errors otherwise. */
int mpx_gemm_variant(int prec, int variant, int transA, int transB, int64_t m, int64_t n,
                     int64_t k, const void *A, int64_t lda, int64_t psA, const void *B,
                     int64_t ldb, int64_t psB, void *C, int64_t ldc, int64_t psC,
                     void *stream);
/* Time every variant `reps` times on the given buffers (C is overwritten)
 * with HIP events on `stream`, remember the fastest for this bucket and
 * return its index (>= 0) or a negative status; *best_ms (nullable) receives
 * its mean time.  Synchronises `stream`; must not be called under graph
 * capture. */
int mpx_gemm_autotune(int prec, int transA, int transB, int64_t m, int64_t n, int64_t k,
                      const void *A, int64_t lda, int64_t psA, const void *B, int64_t ldb,
                      int64_t psB, void *C, int64_t ldc, int64_t psC, int reps,
                      float *best_ms, void *stream);
void mpx_gemm_autotune_reset(void);

#ifdef __cplusplus
}
#endif

#endif /* MPX_H */
