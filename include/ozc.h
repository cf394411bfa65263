/*
 * ozc - complex matrix multiplication emulated on INT8 matrix cores by the
 * Ozaki-II scheme (Chinese-remainder reconstruction), for AMD MI355X (gfx950).
 *
 * Method: Uchino, Ma, Imamura, Ozaki, Gutsche, "Emulation of Complex Matrix
 * Multiplication based on the Chinese Remainder Theorem" (arXiv 2512.08321).
 * The operation is the BLAS zgemm / cgemm one,
 *
 *     C := alpha * op(A) * op(B) + beta * C,
 *
 * with op(A) m x k, op(B) k x n, C m x n, all column-major with interleaved
 * (re, im) complex elements.  The paper states the product C = AB for
 * A in C^{m x k}, B in C^{k x n} (Section III); alpha, beta and op() are the
 * BLAS calling convention of the routines the paper's library replaces
 * (Section III-D).
 *
 * Pipeline (Algorithm 1, Section III):
 *   1. per-row / per-column power-of-two scaling exponents mu_i, nu_j, shared
 *      by the real and imaginary parts (Section III-B), fast mode (Cauchy-
 *      Schwarz bound) or accurate mode (bound from an extra INT8 product);
 *   2. truncation a' = trunc(a 2^mu) and symmetric INT8 residues modulo N
 *      pairwise-coprime moduli p_l <= 256 (Algorithm 1 Steps I, IV, V-i/ii);
 *   3. per modulus, the complex INT8 product with INT32 accumulation, either
 *      Karatsuba with 3 products (equation (10)) or the expanded form with 4
 *      products (equation (7)), reduced to INT8 residues E'_l (Step V-iii/iv);
 *   4. C' = mod(sum_l (P/p_l) q_l E'_l, P) (Step V-v/vi), reconstructed
 *      exactly in integer arithmetic, rounded to nearest-even, then
 *      C = ldexp(C', -(mu_i + nu_j)) (Step VI) and alpha/beta.
 * The uniqueness condition 2 sum_h |a'_ih| |b'_hj| < P (equation (4)) holds by
 * construction of the exponents, so C' equals the exact integer product of
 * the truncated inputs.
 *
 * Every call is asynchronous on the handle's stream: it enqueues HIP kernels
 * and returns; no host synchronisation happens inside ozc_zgemm/ozc_cgemm.
 * A handle is not thread safe: use one handle per host thread.
 * All matrix pointers are device pointers; alpha/beta are host pointers.
 * No function aborts: every error is reported through the returned status.
 */
#ifndef OZC_H
#define OZC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ozc_context *ozc_handle_t;

typedef enum {
    OZC_STATUS_SUCCESS = 0,
    OZC_STATUS_INVALID_VALUE = 1,   /* an argument is out of range (BLAS-style checks)   */
    OZC_STATUS_NOT_SUPPORTED = 2,   /* e.g. k above OZC_MAX_K in ozc_inspect or a batch    */
    OZC_STATUS_ALLOC_FAILED = 3,    /* device allocation of the workspace failed          */
    OZC_STATUS_HIP_ERROR = 4,       /* a HIP runtime call or kernel launch failed          */
    OZC_STATUS_NONFINITE = 5,       /* reported by ozc_last_info: an input was inf or NaN  */
    OZC_STATUS_INVALID_HANDLE = 6,
    OZC_STATUS_VERIFY_FAILED = 7    /* the Freivalds check still failed at the largest N */
} ozc_status_t;

typedef enum { OZC_OP_N = 0, OZC_OP_T = 1, OZC_OP_C = 2 } ozc_op_t;

/* Scaling-vector rule (Section III-B). */
typedef enum { OZC_MODE_FAST = 0, OZC_MODE_ACCURATE = 1 } ozc_mode_t;

/* Complex INT8 product per modulus (Section III-A): Karatsuba (eq. (10), 3
 * products, 6mnk INT8 operations) or the expanded real form (eq. (7), 4
 * products, 8mnk operations).  Both give bit-identical results. */
typedef enum { OZC_ALGO_KARATSUBA = 0, OZC_ALGO_4M = 1 } ozc_algo_t;

#define OZC_MIN_MODULI 2
#define OZC_MAX_MODULI 24
/* INT8 products accumulate exactly in INT32 while k <= 2^17 (Section II). */
#define OZC_MAX_K 131072

/* Exponent sentinels reported by ozc_inspect for rows/columns without scaling. */
#define OZC_EXP_ZERO ((int16_t)-32768)    /* all-zero row (or vanishing accurate bound) */
#define OZC_EXP_NONFINITE ((int16_t)32767) /* the row/column holds an inf or NaN        */

/* Create a handle bound to HIP device `device` (made current for the call).
 * The handle owns its moduli tables and, unless ozc_set_workspace is used, a
 * device workspace that grows on demand.  Stream: the null stream until
 * ozc_set_stream.  Errors: INVALID_VALUE (handle NULL / bad device),
 * HIP_ERROR, ALLOC_FAILED. */
ozc_status_t ozc_create(ozc_handle_t *handle, int device);

/* Free the handle and the workspace it owns (synchronises its stream first). */
ozc_status_t ozc_destroy(ozc_handle_t handle);

/* Stream (a hipStream_t, passed as void*) on which later calls enqueue work. */
ozc_status_t ozc_set_stream(ozc_handle_t handle, void *stream);

/* Number of moduli N in [OZC_MIN_MODULI, OZC_MAX_MODULI] (Algorithm 1 input
 * N; moduli are the first N of 256, 255, 253, 251, 247, 241, ... , the
 * greedy descending pairwise-coprime integers <= 256), scaling mode and
 * product algorithm for the following calls.  Default: N = 14, fast,
 * Karatsuba.  num_moduli == 0 selects the learned choice (see "moduli-count
 * predictor" below) for ozc_zgemm and ozc_zgemm_vbatched; complex64 calls then
 * use N = 9.  ozc_inspect and ozc_workspace_size keep the last fixed N.
 * Errors: INVALID_VALUE. */
ozc_status_t ozc_set_config(ozc_handle_t handle, int num_moduli, ozc_mode_t mode,
                            ozc_algo_t algo);

/* Device workspace in bytes that ozc_zgemm/ozc_cgemm need for this shape
 * under the current configuration (element size does not matter). */
ozc_status_t ozc_workspace_size(ozc_handle_t handle, ozc_op_t transa, ozc_op_t transb,
                                int64_t m, int64_t n, int64_t k, size_t *bytes);

/* Use caller-owned device memory as workspace (ptr == NULL returns to the
 * handle's own growing workspace).  The caller keeps ownership and must keep
 * it alive while calls using it are in flight.  A later call whose shape
 * needs more than `bytes` fails with ALLOC_FAILED. */
ozc_status_t ozc_set_workspace(ozc_handle_t handle, void *ptr, size_t bytes);

/* C := alpha op(A) op(B) + beta C, complex128 (double2) elements.
 * A: lda >= max(1, m) if transa == N, else >= max(1, k); B: ldb >= max(1, k)
 * if transb == N, else >= max(1, n); ldc >= max(1, m).  m, n, k >= 0.
 * The INT32 accumulation of the products is exact for k <= OZC_MAX_K; a
 * larger k is split into ceil(k / OZC_MAX_K) near-equal chunks, each
 * emulated with its own scaling exponents and accumulated into C (beta = 1
 * after the first chunk).  m == 0 or n == 0: no work.
 * alpha == 0 or k == 0: C := beta C without reading A or B.  beta == 0: C
 * is not read.  Rows of op(A) / columns of op(B) holding inf or NaN give NaN
 * output entries and set the status that ozc_last_info reports.
 * Result (alpha = 1, beta = 0): out_ij = ldexp(RNE(C'_ij), -(mu_i + nu_j)),
 * with C' the exact integer reconstruction.  General alpha/beta, in this
 * order: x_r = fma(a_r, c_r, -(a_i c_i)); x_i = fma(a_r, c_i, a_i c_r);
 * beta == 0: out = x; else out_r = fma(b_r, C_r, fma(-b_i, C_i, x_r)),
 * out_i = fma(b_r, C_i, fma(b_i, C_r, x_i)). */
ozc_status_t ozc_zgemm(ozc_handle_t handle, ozc_op_t transa, ozc_op_t transb, int64_t m,
                       int64_t n, int64_t k, const double alpha[2], const void *A,
                       int64_t lda, const void *B, int64_t ldb, const double beta[2],
                       void *C, int64_t ldc);

/* As ozc_zgemm for complex64 (float2) elements: inputs are promoted exactly
 * to double, the result above is computed in double with alpha/beta
 * promoted, and rounded once more to float (round to nearest even). */
ozc_status_t ozc_cgemm(ozc_handle_t handle, ozc_op_t transa, ozc_op_t transb, int64_t m,
                       int64_t n, int64_t k, const float alpha[2], const void *A,
                       int64_t lda, const void *B, int64_t ldb, const float beta[2],
                       void *C, int64_t ldc);

/* The emulated product op(A) op(B) of complex128 operands as a double-double pair
 * C_hi + C_lo, for results beyond double precision.  The reconstruction is exact, so
 * the only rounding of ozc_zgemm's result is its final conversion to double; here,
 * per real and imaginary part, C_hi = ldexp(RNE(C'), -(mu_i + nu_j)) (the entry
 * ozc_zgemm computes with alpha = 1, beta = 0) and C_lo = ldexp(RNE(C' - RNE(C')),
 * -(mu_i + nu_j)), so C_hi + C_lo is the exact integer product of the truncated
 * inputs, scaled, to within 2^-106 relative (exactly when |C'| < 2^106), a second
 * rounding only in the subnormal range.  The accuracy is then limited by the
 * truncation of the scaled inputs, which more moduli reduce (at 24 moduli about
 * 2^-90 of the row maxima).  Operands, checks, configuration and errors as
 * ozc_zgemm; C_hi and C_lo: m x n, leading dimension ldc, not read; k == 0 gives
 * zeros; k above OZC_MAX_K: NOT_SUPPORTED.  The Freivalds check and the learned
 * moduli count are not run (the handle's fixed N is used).  Asynchronous. */
ozc_status_t ozc_zgemm_dd(ozc_handle_t handle, ozc_op_t transa, ozc_op_t transb, int64_t m,
                          int64_t n, int64_t k, const void *A, int64_t lda, const void *B,
                          int64_t ldb, void *C_hi, void *C_lo, int64_t ldc);

/* Real products, C := alpha op(A) op(B) + beta C for float64 (dgemm) and float32
 * (sgemm) matrices: Algorithm 1 as the paper states it for real A and B
 * (Section II), with the scaling rules of Section III-B applied to rows of k
 * reals and one INT8 product per modulus (2 N m n k INT8 operations),
 * E'_l = mod(A'_l B'_l, p_l), exact reconstruction as for complex products.
 * Same layout, argument checks, k-chunking, quick returns and non-finite
 * handling as ozc_zgemm; op C is op T.  alpha, beta: host pointers to one
 * value.  Result: c_ij = ldexp(RNE(C'_ij), -(mu_i + nu_j)); x = alpha c (one
 * rounding); out = x if beta == 0, else fma(beta, C_ij, x).  sgemm promotes the
 * inputs exactly to double, computes this in double and rounds once to float.
 * Uses the handle's fixed moduli count and scaling mode (the product-form
 * setting does not apply); the Freivalds check and the learned moduli count are
 * not run for real products. */
ozc_status_t ozc_dgemm(ozc_handle_t handle, ozc_op_t transa, ozc_op_t transb, int64_t m,
                       int64_t n, int64_t k, const double *alpha, const void *A, int64_t lda,
                       const void *B, int64_t ldb, const double *beta, void *C, int64_t ldc);
ozc_status_t ozc_sgemm(ozc_handle_t handle, ozc_op_t transa, ozc_op_t transb, int64_t m,
                       int64_t n, int64_t k, const float *alpha, const void *A, int64_t lda,
                       const void *B, int64_t ldb, const float *beta, void *C, int64_t ldc);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): ozc_zgemm with the workspace
 * taken from a fixed array of OZC_NOALLOC_WORKSPACE bytes that the library holds
 * in device memory, one per device, from the first ozc_create on that device until
 * the process ends.  Same arguments, semantics and results (bit for bit) as
 * ozc_zgemm with the handle's fixed moduli count, mode and algorithm; the call
 * allocates nothing and enqueues only kernels on the handle's stream.
 * Errors: those of ozc_zgemm's argument checks; NOT_SUPPORTED, before any work,
 * when the shape needs more workspace than the array holds (ozc_workspace_size
 * above OZC_NOALLOC_WORKSPACE: e.g. m = n = k = 700 at 14 moduli, Karatsuba, fits)
 * or when the handle has the Freivalds check or the learned moduli count
 * configured (both need buffers of their own); HIP_ERROR when the array's device
 * address could not be looked up.  Phase timing is not recorded.  Every call on a
 * device shares that device's array and leaves its contents behind (nothing in it
 * is assumed zero at entry): calls that overlap in time on one device, from any
 * handle or stream, race and give wrong results. */
#define OZC_NOALLOC_WORKSPACE ((size_t)64 << 20)
ozc_status_t ozc_zgemm_noalloc(ozc_handle_t handle, ozc_op_t transa, ozc_op_t transb,
                               int64_t m, int64_t n, int64_t k, const double alpha[2],
                               const void *A, int64_t lda, const void *B, int64_t ldb,
                               const double beta[2], void *C, int64_t ldc);

/* Intermediates of the pipeline for alpha = 1, beta = 0, for verification.
 * `single` = element kind of A, B and C: 0 complex128, 1 complex64, 2 float64,
 * 3 float32 (2 and 3 as ozc_dgemm / ozc_sgemm).  Output buffers are device
 * memory owned by the caller; any of them may be NULL.  Layouts (dense):
 *   mu     int16[m]   nu int16[n]   (exponents or the OZC_EXP_* sentinels)
 *   resA   int8[N][planes][m][k]    residues of the rows of op(A)
 *   resB   int8[N][planes][n][k]    residues of the columns of op(B)
 *          planes: Karatsuba 3 (re, im, re+im reduced), 4M 2 (re, im), real 1
 *   prods  int32[N][nprod][n][m]    raw INT32 products per modulus, each
 *          plane column-major: Karatsuba (D, E, F) = (RR, II, SS); 4M (RR, II, RI, IR);
 *          real 1 (A'_l B'_l)
 *   eprime int8[N][eplanes][n][m]   E'_R, E'_I per modulus (real: E'), column-major
 *   C      m x n output (ldc) as ozc_zgemm/ozc_cgemm/ozc_dgemm/ozc_sgemm would write it.
 * Same validity rules and errors as ozc_zgemm. */
ozc_status_t ozc_inspect(ozc_handle_t handle, int single, ozc_op_t transa, ozc_op_t transb,
                         int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                         const void *B, int64_t ldb, int16_t *mu, int16_t *nu, int8_t *resA,
                         int8_t *resB, int32_t *prods, int8_t *eprime, void *C, int64_t ldc);

typedef struct {
    int num_moduli;      /* N used by the last call                                  */
    int mode;            /* ozc_mode_t                                               */
    int algo;            /* ozc_algo_t                                               */
    int nonfinite;       /* 1 if the last call met an inf/NaN input                  */
    int64_t m, n, k;     /* shape of the last call (batched: sums over the problems)  */
    size_t workspace;    /* bytes of workspace the last call used                    */
    double int8_ops;     /* INT8 MFMA operations of the residue products (2 per MAC)  */
    int verified;        /* 1 if the last call ran the Freivalds check                */
    int escalations;     /* reruns with more moduli after a failed check             */
    int64_t verify_failed_rows; /* rows over tolerance in the final check             */
    double verify_ratio; /* max_i |residual_i| / tolerance_i of the final check       */
} ozc_info_t;

/* Freivalds verification (an addition of this library, not in the paper).
 * When enabled, every ozc_zgemm/ozc_cgemm call checks its result with one
 * random sign vector x (x_j = +-1 from SplitMix64(seed, j)):
 *   w = C x,  z = op(A) (op(B) x),  v = C_in x  (v only when beta != 0),
 *   accepted iff for every row i
 *   |w_i - alpha z_i - beta v_i| <= rel (|alpha| (|A||B||x|)_i + |beta| (|C_in||x|)_i)
 *                                    + g (|C||x| + |alpha| |A||B||x| + |beta| |C_in||x|)_i
 * with the three products accumulated in double-double arithmetic and
 * g = 4 (n + k + 4) 2^-104 covering that evaluation, so that tolerances well
 * below double precision (e.g. a 1e-15 target) can be checked.  rel <= 0
 * selects 4 k 2^-53 for ZGEMM and 4 k 2^-24 for CGEMM.  On failure, with
 * escalate != 0, the call reruns with N + 2 moduli (at most OZC_MAX_MODULI;
 * C_in is saved first when beta != 0) and finally returns
 * OZC_STATUS_VERIFY_FAILED with C holding the last result.  A verified call
 * synchronises the stream.  Extra device memory: O(m + n + k) vectors, plus
 * m x n elements when beta != 0.  Batches (ozc_zgemm_vbatched) check every
 * problem the same way, all checks in one set of launches with the same sums
 * as a single call's check, and rerun the failing problems as a smaller batch
 * with two more moduli each; ozc_last_info then reports the rerun rounds, the
 * failing rows and the largest ratio over all problems. */
ozc_status_t ozc_set_verify(ozc_handle_t handle, int enable, double rel, int escalate,
                            uint64_t seed);

/* Test hook that corrupts the pipeline on purpose so that the check above can
 * be exercised: 0 none; 1 flip one byte of E' (modulus 1, entry (0,0)) on the
 * first attempt of each call only; 2 raise the exponent of row 0 of op(A) by
 * 12 on every attempt (breaks the uniqueness condition (4) for that row). */
ozc_status_t ozc_debug_inject(ozc_handle_t handle, int fault);

/* Phase timing.  While enabled, every ozc_zgemm/ozc_cgemm call records HIP
 * events on the handle's stream around its phases (scaling statistics and
 * exponents; residue split; INT8 residue products; CRT reconstruction and
 * output).  ozc_profile_read synchronises the stream, returns the sums over
 * all calls since the previous read (or since enabling) and resets them. */
typedef struct {
    int calls;
    double scale_ms;     /* Step III: statistics, bound product, exponents        */
    double split_ms;     /* Steps IV, V-i/ii: truncation and residues             */
    double gemm_ms;      /* Step V-iii/iv: INT8 products with the reduce epilogue */
    double crt_ms;       /* Steps V-v, V-vi, VI                                   */
    double total_ms;     /* first to last event of each call                      */
} ozc_profile_t;

ozc_status_t ozc_set_profiling(ozc_handle_t handle, int enable);
ozc_status_t ozc_profile_read(ozc_handle_t handle, ozc_profile_t *out);

/* ------------------------------------------------------------------ batches
 * Many independent problems of uneven shapes (an addition of this library;
 * the paper treats one product at a time).  Problem p computes
 *   C_p = alpha_p op(A_p) op(B_p) + beta_p C_p
 * with exactly the semantics and the bit-exact results of ozc_zgemm /
 * ozc_cgemm on the same arguments (fixed moduli order, Section II), using
 * the handle's moduli count and algorithm.  Arguments are host arrays of
 * `count` entries: transa, transb, m, n, k, lda, ldb, ldc; A, B, C hold device
 * pointers; alpha and beta hold 2 * count values (re, im of problem p at
 * 2p, 2p + 1).  Every problem is validated as ozc_zgemm does; the first
 * invalid one makes the call return INVALID_VALUE before any work starts.
 * Problems with m == 0 or n == 0 are skipped; k == 0 or alpha == 0 give
 * C_p = beta_p C_p.
 *
 * The whole batch runs as one launch per phase (statistics, exponents,
 * residue split, products, reconstruction); the products run in a
 * persistent kernel that takes (problem, moduli group, tile) items from
 * device work queues (one per XCD, neighbouring tiles on one XCD), largest k
 * first.  The launch sequence is recorded once
 * into a HIP graph per distinct argument list (pointers included) and
 * replayed when the same list comes again.  The batch owns a workspace of its
 * own (kept until the handle is destroyed or a larger batch needs more).
 * With the learned moduli count configured (N = 0), one statistics pass over
 * all problems and one forward pass of the predictor choose N per problem (one
 * synchronisation), and the batch runs as one launch sequence in which every
 * problem uses its own N; ozc_last_info reports the largest.  Up to 8
 * recorded sequences are kept.  Both scaling modes: in accurate mode the
 * magnitudes and the bound products of all problems run as batched launches
 * too (the bound products in a persistent kernel over their 128 x 128
 * tiles).  Problems must not overlap in C.  Asynchronous on the handle's
 * stream unless the Freivalds check is enabled (see ozc_set_verify: the
 * call then synchronises); non-finite inputs are reported by ozc_last_info
 * as for a single call. */
ozc_status_t ozc_zgemm_vbatched(ozc_handle_t handle, int count, const ozc_op_t *transa,
                                const ozc_op_t *transb, const int64_t *m, const int64_t *n,
                                const int64_t *k, const double *alpha, const void *const *A,
                                const int64_t *lda, const void *const *B, const int64_t *ldb,
                                const double *beta, void *const *C, const int64_t *ldc);
ozc_status_t ozc_cgemm_vbatched(ozc_handle_t handle, int count, const ozc_op_t *transa,
                                const ozc_op_t *transb, const int64_t *m, const int64_t *n,
                                const int64_t *k, const float *alpha, const void *const *A,
                                const int64_t *lda, const void *const *B, const int64_t *ldb,
                                const float *beta, void *const *C, const int64_t *ldc);

/* Schedule of the batched products. */
typedef struct {
    int tile_threshold;  /* problems with min(m, n) >= this use 256 x 256 output tiles,
                            the others 128 x 128 (default 1024)                          */
    int moduli_group;    /* moduli computed one after another per work item (>= 1;
                            default 1)                                                   */
    int use_graph;       /* record and replay HIP graphs (default 1)                     */
} ozc_batch_policy_t;
ozc_status_t ozc_set_batch_policy(ozc_handle_t handle, const ozc_batch_policy_t *policy);
ozc_status_t ozc_get_batch_policy(ozc_handle_t handle, ozc_batch_policy_t *policy);

/* Autotuner: for the given batch, times the product phase under candidate
 * schedules (tile thresholds 256, 512, 1024, 2048 and never, times moduli
 * groups 1, 2, 4 and N; the preparation phases run once per threshold),
 * keeps the fastest as the handle's batch policy and returns it in *chosen
 * (may be NULL).  C is neither read nor written.  Synchronises the stream.
 * `single` selects complex64 operands. */
ozc_status_t ozc_batch_tune(ozc_handle_t handle, int single, int count, const ozc_op_t *transa,
                            const ozc_op_t *transb, const int64_t *m, const int64_t *n,
                            const int64_t *k, const void *const *A, const int64_t *lda,
                            const void *const *B, const int64_t *ldb,
                            ozc_batch_policy_t *chosen);

/* ------------------------------------------------------------------ moduli-count predictor
 * (an addition of this library; the paper fixes N by hand).  A perceptron
 * OZC_MLP_FEATURES -> OZC_MLP_HIDDEN -> OZC_MLP_HIDDEN -> OZC_MLP_CLASSES (ReLU,
 * FP32) maps cheap statistics of op(A) and op(B) to a class c, N = OZC_MLP_MIN_N
 * + c (the last class stands for "more than 24" and gives 24).  With N = 0
 * configured, every ozc_zgemm call computes the statistics, predicts N (this
 * synchronises the stream), adds the margin and runs with it; with the
 * Freivalds check enabled, a failure escalates N as usual.  Until parameters
 * are set or trained, the fixed fallback count is used.
 *
 * Parameter vector (OZC_MLP_PARAMS floats): W1 (H x F, row-major), b1 (H), W2
 * (H x H), b2 (H), W3 (C x H), b3 (C), mu (F), sd (F); inputs are standardised
 * as (x - mu) / sd before the first layer. */
#define OZC_MLP_FEATURES 20
#define OZC_MLP_HIDDEN 64
#define OZC_MLP_CLASSES 20
#define OZC_MLP_MIN_N 6
#define OZC_MLP_PARAMS (OZC_MLP_HIDDEN * OZC_MLP_FEATURES + OZC_MLP_HIDDEN + \
                        OZC_MLP_HIDDEN * OZC_MLP_HIDDEN + OZC_MLP_HIDDEN + \
                        OZC_MLP_CLASSES * OZC_MLP_HIDDEN + OZC_MLP_CLASSES + 2 * OZC_MLP_FEATURES)

/* Statistics of op(A) (m x k) and op(B) (k x n) into `features` (device, 20
 * floats), taken from the integer sums of the fast-mode scaling step (Section
 * III-B): for a row (the 2k reals of a row of op(A) or a column of op(B)) with
 * e = floor(log2 max |x|), sigma = sum ceil(|x| 2^(20-e))^2 and tau = sum
 * ceil(|x| 2^(20-e)), l2 = 0.5 log2 sigma - 20 and l1 = log2 tau - 20.
 * Features: log2 m, log2 n, log2 k; min, max, mean, std of l2 and of l1 over the
 * nonzero finite rows of op(A); the same over the columns of op(B); the
 * fraction of zero reals.  k above OZC_MAX_K: the statistics of the first
 * k-chunk of the call (log2 k is that chunk's).  m, n, k >= 1.  Asynchronous.
 * A call with the learned moduli count computes these in its own scaling pass
 * and reuses that pass's maxima and sums for the product itself. */
ozc_status_t ozc_features(ozc_handle_t handle, int single, ozc_op_t transa, ozc_op_t transb,
                          int64_t m, int64_t n, int64_t k, const void *A, int64_t lda,
                          const void *B, int64_t ldb, float *features);

/* Host copies of the parameter vector (count must be OZC_MLP_PARAMS; every
 * sd entry > 0).  get fails with INVALID_VALUE before parameters exist. */
ozc_status_t ozc_mlp_set_params(ozc_handle_t handle, const float *params, int count);
ozc_status_t ozc_mlp_get_params(ozc_handle_t handle, float *params, int count);

/* Logits (device, rows x OZC_MLP_CLASSES) for feature rows X (device, rows x
 * OZC_MLP_FEATURES).  Asynchronous. */
ozc_status_t ozc_mlp_forward(ozc_handle_t handle, const float *X, int rows, float *logits);

/* Classes (device int, rows) of feature rows X (device, rows x OZC_MLP_FEATURES): the
 * argmax of the logits ozc_mlp_forward computes (lowest class on ties), in one fused
 * launch that runs the same operations in the same order (the launch the per-call
 * prediction uses).  Asynchronous. */
ozc_status_t ozc_mlp_predict(ozc_handle_t handle, const float *X, int rows, int *classes);

/* Gradient (device, OZC_MLP_PARAMS floats; zero for mu, sd) of the mean softmax
 * cross-entropy over rows X with labels y (device int, classes) at the current
 * parameters; *loss (host, may be NULL) receives the loss (synchronises). */
ozc_status_t ozc_mlp_grad(ozc_handle_t handle, const float *X, const int *y, int rows,
                          float *grad, float *loss);

/* Train with Adam (beta1 0.9, beta2 0.999, eps 1e-8, rate lr) for `epochs`
 * passes over (X, y) (device) in mini-batches of `batch` rows, shuffled per
 * epoch with SplitMix64(seed) draws (a batch >= rows keeps the row order).
 * init != 0 (or no parameters yet): mu, sd from the data, He-uniform weights
 * from SplitMix64(seed), zero biases.  epoch_loss (host, epochs floats, may be
 * NULL) receives the mean batch loss per epoch.  Synchronises. */
ozc_status_t ozc_mlp_train(ozc_handle_t handle, const float *X, const int *y, int rows,
                           int epochs, int batch, float lr, uint64_t seed, int init,
                           float *epoch_loss);

/* Store / restore the predictor's parameters (mu, sd and the weights of the
 * three layers) in a file at `path` (host string), so that a network trained
 * once serves later processes.  File layout, little-endian: the 8 bytes
 * "OZCMLP01"; int32 F, H, C, MIN_N, count (the OZC_MLP_* values and
 * OZC_MLP_PARAMS); count float32 parameters in the order ozc_mlp_get_params
 * returns them; the 64-bit FNV-1a hash of those parameter bytes.
 * save: INVALID_VALUE before parameters exist or when the file cannot be
 * written (synchronises).  load: INVALID_VALUE when the file cannot be read,
 * is shorter or longer than that layout, names other dimensions, fails the
 * hash, or holds an sd entry <= 0; the handle's parameters are replaced only
 * by a file that passes every check. */
ozc_status_t ozc_mlp_save(ozc_handle_t handle, const char *path);
ozc_status_t ozc_mlp_load(ozc_handle_t handle, const char *path);

/* Fallback N (used without parameters; default 18) and a margin added to every
 * prediction (default 0, at most 8). */
ozc_status_t ozc_set_auto_moduli(ozc_handle_t handle, int fallback, int margin);

/* The N the predictor would choose for this product (synchronises). */
ozc_status_t ozc_predict_moduli(ozc_handle_t handle, int single, ozc_op_t transa,
                                ozc_op_t transb, int64_t m, int64_t n, int64_t k, const void *A,
                                int64_t lda, const void *B, int64_t ldb, int *num_moduli);

/* Synchronises the handle's stream and reports on the last call.  Returns
 * NONFINITE when the last call met inf/NaN input (info still filled). */
ozc_status_t ozc_last_info(ozc_handle_t handle, ozc_info_t *info);

/* Static text for a status code. */
const char *ozc_status_string(ozc_status_t status);

#ifdef __cplusplus
}
#endif

#endif /* OZC_H */
