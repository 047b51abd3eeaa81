/*
 * cholinv.h -- C-ABI of libcholinv, the MI355X (gfx950) implementation of the
 * reduced-operation inversion of Hermitian positive-definite matrices from
 * Krishnamoorthy & Menon, "Matrix Inversion Using Cholesky Decomposition"
 * (arXiv:1111.4144).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are dense and row major: element (i, j) of a matrix with leading
 *   dimension ld sits at index i*ld + j (elements, not bytes).  The paper
 *   prefers the upper factor R because its rows are contiguous (Section II).
 * - Complex elements are interleaved (re, im) pairs of float (CI_C64) or
 *   double (CI_C128).  Real types are CI_F32 and CI_F64.
 * - Every matrix pointer is DEVICE memory owned by the caller; it must stay
 *   valid until the work queued on `stream` has finished.  `stream` is a
 *   hipStream_t passed as void* (NULL = the default stream).  Options structs
 *   and n_host-style arguments are HOST memory, read before the call returns.
 * - Inputs must be Hermitian (real: symmetric) positive definite.  Only the
 *   upper triangle (i <= j) of an input A is read; its strict lower triangle
 *   may hold anything, NaN included.  The imaginary part of a diagonal entry is
 *   ignored.
 * - Calls are asynchronous: they enqueue kernels on `stream` and return (a
 *   batch too large for one dispatch grid, whose size counts work-items in 32
 *   bits, is queued as several launches in order).  The library never
 *   synchronises the stream and never allocates device memory on
 *   the call path; scratch space is the caller's `work` buffer, sized by
 *   chol_workspace_size().
 *
 * Errors
 * ------
 * The return value reports argument and launch errors at once:
 *     0                    success (work queued)
 *    -k  (1 <= k < 100)    argument number k (1-based) is invalid
 *    CI_ERR_UNSUPPORTED    valid arguments but a combination the library lacks
 *    CI_ERR_WORKSPACE      work_bytes smaller than chol_workspace_size()
 *    CI_ERR_NOALLOC_LIMIT  uneven batch above CI_NOALLOC_MAX_BATCH
 *                          (allocation-free entry point only)
 *    CI_ERR_LAUNCH - e     a HIP launch failed with hipError_t e
 * Numerical failure is never a return code.  `info` (device int32, one per
 * matrix, may be NULL) receives 0, or the 1-based index i of the first pivot
 * whose value is not a finite positive number: the radicand of eq. (3) for
 * Cholesky, d_i of eq. (10) for LDL.  A NaN anywhere in the upper triangle
 * reaches some pivot, so it is reported there.  The X of a failed matrix is
 * filled with NaN.
 */
#ifndef CHOLINV_H
#define CHOLINV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element types. */
enum { CI_F32 = 0, CI_F64 = 1, CI_C64 = 2, CI_C128 = 3 };

/* Factorisation used by the inversion: Cholesky A = R^*R (Section II, eqs.
 * 3-4; inversion Section IV.A) or LDL A = R^*DR (Section II.A, eqs. 10-11;
 * inversion Section IV.B). */
enum { CI_METHOD_CHOL = 0, CI_METHOD_LDL = 1 };

/* Arithmetic.
 * CI_PLAIN: everything in the element type (FP64 for CI_F64/CI_C128, FP32 for
 *   CI_F32/CI_C64).
 * CI_MIXED: element type must be CI_F32 or CI_C64.  The bulk of the work is
 *   FP32; the pivot sums and square roots / reciprocals of eq. (3) or eq. (10)
 *   are FP64; then ns_steps Newton-Schulz steps X <- X + X(I - AX) follow,
 *   with the residual I - AX in FP64 (A and X upcast exactly) and the update
 *   in FP32. */
enum { CI_PLAIN = 0, CI_MIXED = 1 };

typedef struct {
    int32_t method;     /* CI_METHOD_CHOL or CI_METHOD_LDL                    */
    int32_t precision;  /* CI_PLAIN or CI_MIXED                               */
    int32_t ns_steps;   /* Newton-Schulz steps, 0..3 (CI_MIXED only)          */
    int32_t fill_lower; /* 1: also write x_ji = conj(x_ij) (the Hermitian half
                           "where needed", Section IV.A); 0: the strict lower
                           triangle of X is left untouched                    */
} ci_opts;

#define CI_ERR_UNSUPPORTED (-2000)
#define CI_ERR_WORKSPACE   (-2001)
#define CI_ERR_NOALLOC_LIMIT (-2002)
#define CI_ERR_LAUNCH      (-1000)

/* Largest order handled by the batched small-matrix kernels (one matrix per
 * lane or per lane group, held on chip).  Larger orders use the blocked
 * single-matrix path of chol_inverse. */
#define CI_SMALL_NMAX 64

/*
 * chol_factor -- Cholesky factorisation in place, Section II eqs. (3)-(4).
 *   dtype     CI_F32 / CI_F64 / CI_C64 / CI_C128
 *   batch     number of matrices (>= 0)
 *   n         order, 0 <= n <= CI_SMALL_NMAX when batch > 1; any n >= 0 when
 *             batch == 1 (blocked path for n > CI_SMALL_NMAX)
 *   a         device, batch matrices; matrix b starts at a + b*stride
 *   lda       leading dimension, >= n
 *   stride    elements between matrices, >= lda*n (ignored when batch == 1)
 *   info      device int32[batch] or NULL
 *   work, work_bytes  scratch (size from chol_workspace_size(CI_FN_FACTOR,..))
 * On return the upper triangle of each A holds R (real positive diagonal);
 * the strict lower triangle is untouched.  Precision: CI_PLAIN semantics.
 * The blocked path (batch == 1, n > CI_SMALL_NMAX) needs lda == n and a real
 * type (else CI_ERR_UNSUPPORTED).
 */
int chol_factor(int dtype, int64_t batch, int64_t n, void* a, int64_t lda, int64_t stride,
                int32_t* info, void* work, size_t work_bytes, void* stream);

/*
 * ldl_factor -- LDL factorisation in place, Section II.A eqs. (10)-(11).
 *   Same arguments as chol_factor plus
 *   d         device, real array (float for CI_F32/CI_C64, double otherwise)
 *             of batch*n; matrix b's pivots at d + b*n
 * On return the strict upper triangle of each A holds the unit upper R (its
 * unit diagonal is implied; the diagonal of A is left as it was).  info
 * reports the first pivot d_i that is zero or not finite (no positivity is
 * required for the factorisation alone).  Only batched orders
 * n <= CI_SMALL_NMAX are supported.
 */
int ldl_factor(int dtype, int64_t batch, int64_t n, void* a, int64_t lda, int64_t stride,
               void* d, int32_t* info, void* stream);

/*
 * chol_solve -- X_b = A_b^{-1} Y_b for a batch of small systems, from the
 * factor written by chol_factor (Cholesky: R^* b = y then R x = b, Section II
 * eqs. 5-7) or ldl_factor (LDL: R^* c = y, b_i = c_i/d_i, R x = b, Section
 * II.A eqs. 12-14); 2 x n^2/2 multiplies per right-hand side.
 *   dtype      CI_F32 / CI_F64 / CI_C64 / CI_C128
 *   method     CI_METHOD_CHOL or CI_METHOD_LDL
 *   batch      number of systems (>= 0)
 *   n          order, 0 <= n <= CI_SMALL_NMAX
 *   nrhs       right-hand sides per system (>= 0)
 *   r, ldr, stride_r  device, the factors: the upper triangle of matrix b at
 *              r + b*stride_r holds R (CHOL: with its real positive diagonal;
 *              LDL: the strict upper part of the unit R, whose diagonal is
 *              implied).  Nothing below the diagonal is read.
 *   d          device, LDL pivots as ldl_factor wrote them (float for
 *              CI_F32/CI_C64, double otherwise; matrix b's at d + b*n);
 *              ignored for CHOL (may be NULL)
 *   b, ldb, stride_b  device, right-hand sides: an n x nrhs row-major block
 *              per system, element (i, c) of system b at b + b*stride_b +
 *              i*ldb + c; column c is one right-hand side
 *   x, ldx, stride_x  device, solutions in the same layout; x may equal b
 *              (in place) when ldx == ldb and stride_x == stride_b, and must
 *              not overlap it otherwise
 * Strides are ignored when batch == 1.  A zero or non-finite pivot gives
 * non-finite solutions (the factorisation's info reports it); no info is
 * written here.  Precision: the element type throughout.
 */
int chol_solve(int dtype, int method, int64_t batch, int64_t n, int64_t nrhs, const void* r,
               int64_t ldr, int64_t stride_r, const void* d, const void* b, int64_t ldb,
               int64_t stride_b, void* x, int64_t ldx, int64_t stride_x, void* stream);

/*
 * chol_inverse -- X = A^{-1} of one matrix of any order by the proposed method
 * (Section IV): factorisation, then one back-substitution R X = S against the
 * known upper triangle S = diag(1/r_ii) (eq. 24) or diag(1/d_i) (eq. 29) of
 * the skipped first solve, computing only the upper half of X.
 *   a, lda    device input (not modified)
 *   x, ldx    device output; x may equal a only for CI_PLAIN with
 *             n <= CI_SMALL_NMAX and lda == ldx
 *   opts      host options (NULL = Cholesky, plain, no refinement, fill)
 *   work      device scratch of work_bytes >= chol_workspace_size(CI_FN_INVERSE, ...)
 *   info      device int32[1] or NULL
 * For n > CI_SMALL_NMAX the blocked path runs: right-looking blocked Cholesky
 * with MFMA trailing updates (mixed precision: FP64 pivot accumulators), then
 * the inverse of R by block columns and the upper half of X = R^{-1} R^{-T}
 * as one MFMA product (the same n^3/2 multiplies as Section IV, reading
 * "zero-skipping triangular inverse"; the block form of the Section IV
 * recurrence itself is large-order configuration 4, see the tuner below),
 * then the Newton-Schulz steps as an FP64
 * and an FP32 MFMA product.  There only CI_METHOD_CHOL and real types
 * (CI_F32, CI_F64) are supported (else CI_ERR_UNSUPPORTED), x must not equal
 * a, and X is always written in full (fill_lower is ignored).
 */
int chol_inverse(int dtype, int64_t n, const void* a, int64_t lda, void* x, int64_t ldx,
                 const ci_opts* opts, void* work, size_t work_bytes, int32_t* info,
                 void* stream);

/*
 * chol_inverse_batched -- X_b = A_b^{-1} for a batch of small matrices
 * (Section IV), one matrix per lane or per lane group, in one launch.
 *   batch       number of matrices
 *   n_uniform   > 0: every matrix has this order (<= CI_SMALL_NMAX); matrix b
 *               is at a + b*stride_a and x + b*stride_x, leading dimension n
 *               0: variable orders (packed): n_dev[b] is the order of matrix b
 *               and offsets_dev[b] its first element in both a and x; each
 *               matrix is dense with leading dimension n_dev[b].  n_max is an
 *               upper bound of the orders (host value, <= CI_SMALL_NMAX).
 *   n_dev, offsets_dev  device int32[batch] / int64[batch] (varlen only)
 *   work        device scratch (varlen: the bucketed work list lives here)
 * Every matrix of a varlen batch is processed by the kernel of its size
 * bucket: after a small device-side bucketing prologue (largest orders
 * first), one persistent launch takes the orders 33..64 and one the rest;
 * nothing synchronises with the host, so the call is capturable in a HIP
 * graph.  Varlen batches support the real types (CI_F32, CI_F64; others give
 * CI_ERR_UNSUPPORTED); a matrix whose order is outside 0..n_max gets
 * info[b] = -1 and its X is left untouched; order 0 gives info[b] = 0.
 * For uniform batches of order <= 16 the kernel is the one recorded by
 * chol_autotune for (dtype, precision, method, order), if any.
 */
int chol_inverse_batched(int dtype, int64_t batch, int64_t n_uniform, const int32_t* n_dev,
                         const int64_t* offsets_dev, int64_t n_max, const void* a,
                         int64_t stride_a, void* x, int64_t stride_x, const ci_opts* opts,
                         void* work, size_t work_bytes, int32_t* info, void* stream);

/*
 * chol_inverse_batched_noalloc -- chol_inverse_batched for callers that cannot
 * allocate or pass device memory for scratch: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments and
 * results as chol_inverse_batched without work/work_bytes.  An uneven batch
 * (n_uniform == 0) keeps its bucketing plan and sorted work list in a scratch
 * array that the library holds in device memory, one per GPU, for the life of
 * the process (CI_NOALLOC_MAX_BATCH * 4 bytes plus about 1.3 KiB); uniform
 * batches need no scratch.  The call allocates nothing (no hipMalloc, no
 * hipFree), does not synchronise and clears the plan with a kernel, so it may
 * be captured; the first call on a device must not be captured (it looks up
 * that device's array).  The device is the current one, and `stream` must
 * belong to it.
 *   batch       uneven batches: at most CI_NOALLOC_MAX_BATCH, else
 *               CI_ERR_NOALLOC_LIMIT (checked before any other argument)
 * Calls on one GPU share its array: two uneven-batch calls whose work may
 * overlap in time on that GPU (different streams, or concurrent host
 * threads) race on it and give undefined results; calls queued in order on
 * one stream are safe.
 */
#define CI_NOALLOC_MAX_BATCH 2097152
int chol_inverse_batched_noalloc(int dtype, int64_t batch, int64_t n_uniform,
                                 const int32_t* n_dev, const int64_t* offsets_dev, int64_t n_max,
                                 const void* a, int64_t stride_a, void* x, int64_t stride_x,
                                 const ci_opts* opts, int32_t* info, void* stream);

/*
 * chol_inverse_nonherm -- D_b^{-1} for a batch of general (not Hermitian)
 * nonsingular square matrices by the route of Section III.C: A = D D^* is
 * Hermitian positive definite, so D^{-1} = D^* A^{-1}.  Three steps on
 * `stream`: A = D D^* (upper triangle) into the workspace, X_A = A^{-1} by
 * the batched Section IV inversion (opts: method, precision, ns_steps;
 * fill_lower is ignored), then D^{-1} = D^* X_A into x.  The condition number
 * of A is the square of that of D, so the accuracy is that of an inversion
 * at kappa(D)^2.
 *   batch      number of matrices
 *   n          order, 0 <= n <= CI_SMALL_NMAX
 *   d, stride  device input, matrix b at d + b*stride, leading dimension n
 *              (stride >= n*n; ignored when batch == 1); not modified
 *   x          device output, same layout as d; must not overlap d
 *   work       device scratch of work_bytes >= chol_workspace_size(
 *              CI_FN_NONHERM, dtype, batch, n, opts) (two dense batches)
 *   info       device int32[batch] or NULL: the first failing pivot of the
 *              factorisation of D D^* (a singular D), whose output is NaN
 */
int chol_inverse_nonherm(int dtype, int64_t batch, int64_t n, const void* d, int64_t stride,
                         void* x, const ci_opts* opts, void* work, size_t work_bytes,
                         int32_t* info, void* stream);

/*
 * chol_inverse_backward -- adjoint of X = A^{-1} for the real loss
 * L = Re<G, X> restricted to Hermitian A:  gA = -X Gh X, Gh = (G + G^H)/2.
 * It reuses the forward's X (full Hermitian, e.g. written with fill_lower = 1)
 * instead of recomputing the inverse.  gA is Hermitian and written in full.
 *   x, g, ga    device, batch matrices of order n (<= CI_SMALL_NMAX; CI_C128
 *               only up to 32, larger orders give CI_ERR_UNSUPPORTED: three
 *               64 x 64 complex128 matrices do not fit one workgroup's LDS),
 *               leading dimension n, matrix b at ptr + b*stride
 */
int chol_inverse_backward(int dtype, int64_t batch, int64_t n, const void* x, const void* g,
                          void* ga, int64_t stride, void* stream);

/*
 * chol_inverse_q15 -- the proposed inversion in fixed point, for batches of
 * complex Hermitian positive-definite matrices of order n <= CI_Q15_NMAX
 * (Cholesky, eqs. 3-4; Section IV.A back-substitution; mirror).  The paper
 * evaluates its method by fixed-point simulation without naming a format;
 * this one is:
 *   - input entries are int16 (re, im) pairs q standing for q / 2^15 (scale
 *     each matrix by a power of two beforehand; the inverse scales back by
 *     the inverse power); only the upper triangle is read, the imaginary part
 *     of the diagonal is ignored;
 *   - R is held in Q15 and saturates at +-32767; every sum of products is an
 *     int64 with 30 fractional bits; r_ii = floor(sqrt(radicand)) exactly;
 *     off-diagonal entries divide by r_ii with rounding to nearest, halves
 *     away from zero (as every rounding here);
 *   - X is formed as X 2^F in int64, F = 2 floor(log2 min r_ii) -
 *     ceil(log2 n), saturating at +-(2^40 - 1);
 *   - the output is int16 (re, im) mantissas x with X = x 2^xexp (xexp per
 *     matrix, the smallest shift that fits), written in full with x_ji =
 *     conj(x_ij).
 *   batch        number of matrices
 *   n            order, 0 <= n <= CI_Q15_NMAX
 *   a, stride    device int16, matrix b at a + 2*b*stride (stride in complex
 *                entries, >= n*n; ignored when batch == 1), leading dimension n
 *   x            device int16 output, same layout; must not equal a
 *   xexp         device int32[batch], required
 *   sat          device int32[batch] or NULL: saturation events per matrix
 *   info         device int32[batch] or NULL: 0, or the 1-based row whose
 *                radicand is <= 0 (then x = 0 and xexp = 0)
 * Results are exact integers: they do not depend on the device or the launch.
 */
#define CI_Q15_NMAX 16
int chol_inverse_q15(int64_t batch, int64_t n, const int16_t* a, int64_t stride, int16_t* x,
                     int32_t* xexp, int32_t* sat, int32_t* info, void* stream);

/*
 * chol_inverse_compare -- the existing methods the paper compares against,
 * for batches of small matrices (orders <= CI_COMPARE_NMAX), arithmetic in the
 * element type, one lane per matrix (straightforward kernels for accuracy and
 * timing comparisons, not tuned):
 *   CI_III_A  Section III.A, equation solving: A x_i = e_i (eq. 15) for the
 *             upper half of each column, after a Cholesky (method
 *             CI_METHOD_CHOL) or LDL (CI_METHOD_LDL) factorisation
 *   CI_III_B  Section III.B, triangular operations: M = R^{-1} (eq. 18), then
 *             the upper half of X = M M^* (eq. 19); Cholesky only
 *   CI_IV_SAME  the proposed Section IV back-substitution (Cholesky or LDL)
 *             in this same framework (same factor code, LDS layout and
 *             arithmetic), the reference point the other two are compared
 *             with: the three differ only by their route from R to X
 *   a, stride  device input, matrix b at a + b*stride (stride >= n*n;
 *              ignored when batch == 1), leading dimension n; upper triangle
 *              read
 *   x          device output, same layout, written in full (mirrored); must
 *              not equal a
 *   info       device int32[batch] or NULL: first failing 1-based pivot (not
 *              a finite positive number); the X of a failed matrix is NaN
 */
#define CI_COMPARE_NMAX 16
enum { CI_III_A = 0, CI_III_B = 1, CI_IV_SAME = 2 };
int chol_inverse_compare(int dtype, int variant, int method, int64_t batch, int64_t n,
                         const void* a, int64_t stride, void* x, int32_t* info, void* stream);

/*
 * chol_inverse_q15_compare -- the Section III methods (variant CI_III_A,
 * equation solving, eq. 15; CI_III_B, triangular operations, eqs. 17-19) in
 * the fixed-point format of chol_inverse_q15, Cholesky only: the same Q15
 * factor, the same Y = X 2^F and the same int16 output with one exponent per
 * matrix; only the route from R to Y differs.  The forward solution of III.A
 * (one column at a time) and M = R^{-1} of III.B are held as (.) 2^G in int64,
 * G = floor(log2 min r_ii) + 13 - ceil(ceil(log2 n) / 2), saturating at
 * +-(2^29 - 1) (counted in sat); every division is the same rounded integer
 * division.  For side-by-side accuracy comparisons of the three methods on
 * the same quantized inputs.
 *   variant      CI_III_A or CI_III_B (argument 1)
 *   the other arguments as chol_inverse_q15 (numbered from 2)
 * Results are exact integers: they do not depend on the device or the launch.
 */
int chol_inverse_q15_compare(int variant, int64_t batch, int64_t n, const int16_t* a,
                             int64_t stride, int16_t* x, int32_t* xexp, int32_t* sat,
                             int32_t* info, void* stream);

/* Which entry point a workspace query is for. */
enum { CI_FN_FACTOR = 0, CI_FN_INVERSE = 1, CI_FN_BATCHED = 2, CI_FN_NONHERM = 3 };

/* Bytes of device scratch the named entry point needs for these arguments
 * (0 when none).  For CI_FN_BATCHED pass n = n_uniform (0 for varlen). */
size_t chol_workspace_size(int fn, int dtype, int64_t batch, int64_t n, const ci_opts* opts);

/* Human-readable text for a return code (static storage). */
const char* chol_status_string(int code);

/* Library version string (static storage). */
const char* chol_version(void);

/* ---- autotuner of the small-order engines --------------------------------
 * For orders up to 16 several kernels can invert a uniform batch (engines:
 * 1 one lane per matrix, direct loads; 2 the same with LDS staging; 3 with
 * persistent staging; 4 sixteen-lane groups; 5 sixteen-lane groups with the
 * Newton-Schulz step on MFMA, mixed precision only; 6 four-lane groups with
 * sixteen matrices per wave, orders 9..16, CI_F32 / CI_C64, the refinement
 * on MFMA, the built-in choice for CI_C64 orders 9..16 and for CI_F32 orders
 * 9..16 in mixed precision; 7 eight-lane groups for CI_F64 / CI_C128 in plain
 * precision, one column per lane up to order 8 and two above).  The choice
 * depends on
 * the device, so it is measured, not fixed.
 *
 * chol_autotune times every candidate engine of (dtype, opts) for each order
 * n_lo..n_hi (1 <= n_lo <= n_hi <= 16; n_lo == n_hi > CI_SMALL_NMAX tunes a
 * large order instead, see below) on a synthetic batch of `batch`
 * diagonally dominant matrices on `stream`, and records the fastest (ties
 * within 1% go to the lower engine number).  Later chol_inverse /
 * chol_inverse_batched calls with the same dtype, precision and method use the
 * record.  cache_path (may be NULL): a text file; entries for this device
 * (architecture name and compute-unit count) are loaded instead of measured,
 * and new measurements are appended.  This is a set-up call: it allocates and
 * frees device memory (two batches and an info array) and synchronises the
 * stream; it must not run during stream capture.  The record is process-wide
 * and thread-safe.
 * Returns the number of orders measured (>= 0), -k for an invalid argument k,
 * or CI_ERR_LAUNCH - hipError_t on a HIP failure. */
int chol_autotune(int dtype, const ci_opts* opts, int n_lo, int n_hi, int64_t batch,
                  const char* cache_path, void* stream);

/* The recorded engine for (dtype, opts precision/method, order n); 0 when
 * the built-in choice applies.  n > CI_SMALL_NMAX: the large-order
 * configuration recorded for n's power-of-two bucket (large orders, below);
 * n = 0: the uneven-batch bucket edge (see chol_autotune_varlen).
 * Negative for an invalid argument. */
int chol_tuned_engine(int dtype, const ci_opts* opts, int n);

/* Record `engine` (one of the candidates above for this dtype, precision and
 * order, or 0 for the built-in choice) for (dtype, opts precision/method,
 * order n, 1..16) without measuring, e.g. a choice read from a tuning file or
 * one a test wants to exercise.  n > CI_SMALL_NMAX records a large-order
 * configuration 0..5 for n's bucket; n = 0 records the uneven-batch bucket
 * edge (0, 17, 25 or 33).  Returns 0, or -k for an invalid argument k (-4:
 * the engine cannot invert this combination). */
int chol_tune_set(int dtype, const ci_opts* opts, int n, int engine);

/* ---- large orders (n > CI_SMALL_NMAX, real types, Cholesky) -------------
 * chol_autotune with n_lo == n_hi == n > CI_SMALL_NMAX times the large-order
 * configurations on a synthetic symmetric positive-definite matrix of order
 * n and records the fastest for n's power-of-two bucket (batch is ignored;
 * the cache file and the tie rule are those above).  Configurations:
 *   0 diagonal blocks sub-blocked on MFMA, blocked triangular inverse and
 *     X = M M^T, split-K products aiming at 512 workgroups (built-in)
 *   1, 2 the same aiming at 256 / 1024 workgroups
 *   3 diagonal blocks by the row-by-row Crout recurrence
 *   4 the Section IV recurrence in block form for the inverse
 *   5 configuration 0 with the long unsplit products (at least 256 tiles,
 *     K >= 512) on 256 x 128 workgroup tiles instead of 128 x 128
 * Returns 1 when it measured, 0 when the cache had the answer.  Later
 * chol_inverse / chol_factor calls of that bucket use the record. */

/* ---- uneven batches ----------------------------------------------------------
 * chol_autotune_varlen times the uneven-batch path on the caller's own batch
 * (arguments as chol_inverse_batched with n_uniform = 0; x is overwritten
 * with the inverses) for three edges of its last size bucket, whose orders
 * are inverted by four waves per matrix: 33 (built-in), 25 and 17, and
 * records the fastest for (dtype, precision, method).  Real types only.
 * Returns the chosen edge, or a negative code. */
int chol_autotune_varlen(int dtype, const ci_opts* opts, int64_t batch, const int32_t* n_dev,
                         const int64_t* offsets_dev, int64_t n_max, const void* a, void* x,
                         void* work, size_t work_bytes, void* stream);

/* Forget every recorded choice. */
void chol_autotune_clear(void);

#ifdef __cplusplus
}
#endif

#endif /* CHOLINV_H */
