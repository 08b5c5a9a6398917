/*
 * sap.h - C ABI of the MI355X (gfx950) sketch-and-precondition least-squares
 * library.
 *
 * The library solves the overdetermined least-squares problem
 *     min_x || b - A x ||,   A in R^{m x n}, m >> n          (paper eq. 1.1)
 * with the sketch-and-precondition method of Alg. 1: sample a sparse sign
 * sketch S (Def. 2.2; rejection sampling of Sec. 3.1.2 / Alg. 3), form
 * Y = S [A b], take the Householder QR of Y, use M = R^-1 as a right
 * preconditioner and x0 = M (Q^T S b) as the initial guess, then run
 * preconditioned LSQR (Alg. 2).
 *
 * Conventions shared by every call:
 *   - Pointers named as device pointers must point to device memory of the
 *     context's GPU.  All of them are owned by the caller; the library never
 *     frees or retains them beyond the call (sap_submit: until sap_poll
 *     reports a terminal status).  The library owns only its internal
 *     workspace, bounded by the context's HBM budget.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls enqueue their kernels on it; a call returns when the documented
 *     result is available unless it says it is asynchronous.
 *   - Matrices: A is row-major m x n with leading dimension lda >= n
 *     (element (i, j) at A[i*lda + j]).  Y and R are column-major
 *     (element (r, c) at Y[r + c*ldy]).
 *   - Errors: every call returns a sap_status; no exception crosses the ABI.
 *     On SAP_EINVAL / SAP_ENOMEM outputs are untouched.  sap_last_error()
 *     gives a human-readable reason for the calling thread's last failure
 *     on that context.
 *   - Threads: one caller per context at a time, except the served-form
 *     calls (sap_submit / sap_poll / sap_cancel / sap_serve_stats), which
 *     are thread-safe and may run beside one other blocking call.
 */
#ifndef SAP_H
#define SAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sap_status {
    SAP_OK = 0,
    SAP_EINVAL = 1,          /* invalid argument (shape, pointer, dtype, non-finite b or A) */
    SAP_ENOMEM = 2,          /* workspace would exceed the context's HBM budget */
    SAP_RANK_DEFICIENT = 3,  /* min |R_kk| <= d * 2^-53 * max |R_kk| */
    SAP_NOT_CONVERGED = 4,   /* maxiter reached; x holds the last iterate */
    SAP_PENDING = 5,         /* served request not finished yet */
    SAP_EDEVICE = 6,         /* HIP runtime error or device-side failure */
    SAP_ECANCELED = 7        /* served request cancelled */
} sap_status;

typedef enum sap_dtype { SAP_F64 = 0, SAP_F32 = 1, SAP_BF16 = 2 } sap_dtype;

/* Precision forms of sap_solve.  FP64: A and every step in double.
 * MIXED_FP32: A stored in FP32 (the problem is the FP32 matrix, whose
 * elements are exact in FP64).  The sketch apply and the LSQR passes read the
 * FP32 A and widen each element, so the sketch, the QR, the products and
 * accumulations, u, the preconditioner and the recurrences are FP64.  The
 * passes, which dominate the run time, move half the bytes of the FP64 form
 * and reach the same FP64 stopping test, with no refinement loop.  (An FP32
 * sketch is available through sps_apply; it perturbs the preconditioner of an
 * ill-conditioned A enough to cost extra iterations, so sap_solve does not
 * use it.) */
/* MIXED_FP32_REFINE: A stored in FP32; iterative refinement: each outer
 * step forms r = b - A x with FP64 accumulation, solves min ||r - A delta||
 * by preconditioned LSQR whose products, accumulations and u are FP32, until
 * that problem's normal-equation residual has dropped by 1e-6 or reached FP32
 * resolution, and sets x += delta.  It stops with SAP_OK when
 * ||delta|| <= tol ||x|| (tol is the target relative error of x, e.g. 1e-8;
 * the error left is much smaller than that last correction), and with
 * SAP_NOT_CONVERGED when a correction is no smaller than the previous one
 * (the FP32 representation of r, about 2^-24 ||r|| / sigma_min(A) in x, is
 * reached) or after max_refine steps.  The sketch, QR and preconditioner are
 * FP64 as in MIXED_FP32, which reaches the FP64 stopping test and is usually
 * faster. */
/* MIXED_BF16SA: A stored in FP32; the sketch is applied to a BF16 copy of A
 * (round to nearest even, made by the library in its workspace: m * n * 2
 * more bytes, counted in t_apply_ms) with FP64 accumulation, since the
 * preconditioner only has to be approximate (Sec. 3.2: LSQR on A R^-1
 * converges to the solution for any invertible R); the iterations are those
 * of MIXED_FP32_REFINE, with the same tol semantics.  BF16 keeps 8 bits of
 * each entry: a relative perturbation of up to 2^-9 per entry of A.  Where
 * A's ill-conditioning is column scaling (which commutes with entrywise
 * relative rounding) the convergence rate stays that of the sketch, but the
 * sketch-and-solve initial guess is then only ~2^-9 accurate, which costs
 * extra iterations on near-consistent problems; otherwise the preconditioner
 * itself degrades. */
typedef enum sap_mode {
    SAP_MODE_FP64 = 0,
    SAP_MODE_MIXED_FP32 = 1,
    SAP_MODE_MIXED_FP32_REFINE = 2,
    SAP_MODE_MIXED_BF16SA = 3
} sap_mode;

typedef struct sap_ctx sap_ctx;

/* Create a context on HIP device `device` whose internal workspace may use at
 * most `hbm_budget` bytes (0 = 90% of the device's free memory).
 * Errors: SAP_EINVAL (bad device / null out), SAP_EDEVICE. */
sap_status sap_create(sap_ctx **out, int device, size_t hbm_budget);
void sap_destroy(sap_ctx *ctx);
const char *sap_last_error(const sap_ctx *ctx);
const char *sap_status_string(sap_status s);

/* ------------------------------------------------------------------------
 * Sparse sign sketch (Def. 2.2; generation by rejection sampling, Sec. 3.1.2
 * and Alg. 3).  S is d x m; column i holds exactly zeta nonzeros, at the
 * distinct rows idx[i*zeta + 0 .. zeta-1] (strictly ascending), with value
 * +1/sqrt(zeta) where bit k of sign[i] is 1 and -1/sqrt(zeta) where it is 0
 * (bit k belongs to the k-th smallest row).  Bits >= zeta of sign[i] are 0.
 *
 * Random stream: Philox4x64-10 with key (seed, stream).  Draw j of redraw
 * round r of column i is Lemire's bounded integer in [0, d) taken from word
 * (j mod 4) of Philox(counter = (i, r, floor(j/4), k)), k = 0, 1, ... until
 * accepted; the sign word is word 0 of Philox(counter = (i, 2^64-1, 0, 0)).
 * Round 0 draws zeta values; each later round redraws, on the sorted column,
 * every position j whose value equals that of position j+1.
 * ---------------------------------------------------------------------- */
typedef struct sps_sketch {
    int64_t m;        /* columns of S (rows of A), >= 1 */
    int32_t d;        /* rows of S (embedding dimension), 1 <= d < 2^31 */
    int32_t zeta;     /* nonzeros per column, 1 <= zeta <= min(d, 64) */
    uint64_t seed;    /* Philox key word 0 */
    uint64_t stream;  /* Philox key word 1 (0 for single solves) */
    int32_t *idx;     /* device, m*zeta int32 (row i of idx = column i of S) */
    uint64_t *sign;   /* device, m words */
} sps_sketch;

/* Fill S->idx and S->sign.  Asynchronous on `stream`.
 * Errors: SAP_EINVAL if zeta < 1, zeta > 64, zeta > d, m < 1, d < 1 or a
 * pointer is NULL. */
sap_status sps_generate(sap_ctx *ctx, const sps_sketch *S, void *stream);

/* Y = S [A b]  (the sketching step of Alg. 1; b is sketched as column n of Y so that
 * Q^T S b comes out of the same factorisation).  A: device, row-major m x n,
 * lda >= n, dtype a_type in {F64, F32, BF16}.  b: device, m doubles, or NULL
 * (then Y has n columns).  Y: device, column-major d x (n + (b != NULL)),
 * ldy >= d, dtype y_type in {F64, F32}; it is overwritten.  Accumulation is
 * in y_type; the 1/sqrt(zeta) scale is applied once after summation.
 * Asynchronous on `stream`.  Errors: SAP_EINVAL (shapes, dtypes, NULL),
 * SAP_ENOMEM (partial-sum workspace). */
sap_status sps_apply(sap_ctx *ctx, const sps_sketch *S, const void *A, int64_t lda,
                     sap_dtype a_type, const double *b, int32_t n, void *Y, int64_t ldy,
                     sap_dtype y_type, void *stream);

/* sps_apply without any allocation, for callers that cannot allocate device
 * memory (code being captured into a HIP graph, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments, result and errors as sps_apply;
 * its partial sums live in a static device buffer of 128 MiB that the
 * library holds on every GPU it runs on until the process ends (looked up
 * once at sap_create).  It calls no hipMalloc, hipFree or other allocating
 * routine.  Errors: those of sps_apply, and SAP_ENOMEM when this apply
 * needs more than the static buffer (sap_last_error gives the size needed;
 * the 2^20 x 1000, d = 4000 apply needs 64 MB).  Every call on a GPU uses
 * that GPU's one buffer: calls that overlap in time on one GPU (on
 * different streams, or from different contexts) race and must be
 * serialised by the caller.  Asynchronous on `stream`. */
sap_status sps_apply_noalloc(sap_ctx *ctx, const sps_sketch *S, const void *A, int64_t lda, sap_dtype a_type,
                             const double *b, int32_t n, void *Y, int64_t ldy, sap_dtype y_type, void *stream);

/* Householder QR of Y (the factorization step of Alg. 1), in place, FP64.
 * Y: device, column-major rows x cols (ldy >= rows), rows >= cols.  On return
 * the upper triangle holds R and the strict lower part the Householder
 * vectors v_k (unit leading entry implicit); tau (device, cols doubles)
 * holds the reflector scalars, H_k = I - tau_k v_k v_k^T, with the LAPACK
 * dlarfg sign convention R_kk = -sign(alpha_k) ||x_k||.
 * Asynchronous on `stream`.  Errors: SAP_EINVAL, SAP_ENOMEM. */
sap_status sap_qr(sap_ctx *ctx, double *Y, int64_t ldy, int32_t rows, int32_t cols,
                  double *tau, void *stream);

/* Triangular solve with the preconditioner factor (M = R^-1 applied without
 * forming the inverse).  R: device, upper triangle of a column-major n x n
 * array with leading dimension ldr (entries below the diagonal are ignored).
 * trans = 0 solves R x = rhs; trans = 1 solves R^T x = rhs.  rhs and x are
 * device arrays of n doubles (they may alias).  Asynchronous.
 * Errors: SAP_EINVAL. */
sap_status sap_trsv(sap_ctx *ctx, const double *R, int64_t ldr, int32_t n, int32_t trans,
                    const double *rhs, double *x, void *stream);

/* ------------------------------------------------------------------------
 * Least-squares problems and solver parameters.
 * ---------------------------------------------------------------------- */
typedef struct sap_problem {
    int64_t m;          /* rows of A, m >= n + 1 */
    int32_t n;          /* columns of A, n >= 1 */
    const void *A;      /* device, row-major m x n, lda >= n */
    int64_t lda;
    sap_dtype a_type;   /* F64 for SAP_MODE_FP64, F32 for the mixed modes */
    const double *b;    /* device, m doubles */
} sap_problem;

typedef struct sap_params {
    int32_t d;          /* embedding dimension, n + 1 <= d (paper: d = O(n));
                           0 = choose (Sec. 4.3): sap_solve takes sap_choose_d's
                           pick, the batched and served forms eq. (4.2)'s d
                           (cost ratio 1) capped at their d limit */
    int32_t zeta;       /* sketch nonzeros per column, 1..min(d, 64) */
    uint64_t seed;      /* sketch seed (stream word is 0 for sap_solve) */
    double tol;         /* LSQR stopping tolerance (see below), e.g. 1e-12 */
    int32_t maxiter;    /* LSQR iteration cap (summed over refinements) */
    int32_t mode;       /* sap_mode */
    int32_t max_refine; /* MIXED_FP32_REFINE: outer steps cap (0 = 10) */
    int32_t fixed_iters; /* 0: stop on the test below.  > 0: run exactly this
                           many iterations (fewer only on breakdown) and report
                           SAP_OK; < 0: run the eq. (4.1) count for tol,
                           ceil(2 log(tol) / log(n/d)) (the fixed-count mode of
                           Sec. 4.2).  FP64 and MIXED_FP32 modes only. */
} sap_params;

typedef struct sap_info {
    int32_t status;      /* final sap_status of the solve */
    int32_t iters;       /* LSQR iterations (summed over refinements) */
    int32_t refinements; /* MIXED_FP32_REFINE: residual refinement steps */
    double resid_est;    /* estimate of ||b - A x|| */
    double normar_est;   /* estimate of ||(A M)^T (b - A x)|| */
    double t_generate_ms, t_apply_ms, t_qr_ms, t_iterate_ms; /* phase times */
    double t_queue_ms;   /* served form: submit -> admission */
    double t_total_ms;   /* served form: submit -> finished */
    int32_t d_used;      /* the embedding dimension the solve used */
    int32_t pad_;
} sap_info;

/* Solve min ||b - A x|| by Alg. 1 with a sparse sign sketch and LSQR (Alg. 2)
 * on A R^-1.  x: device, n doubles (output).  info: host pointer (nullable).
 * Stopping (the paper leaves the test open; reading after Paige & Saunders,
 * with ||A M|| ~ 1 by Lemma 2.4): stop after iteration t when
 * alpha_{t+1} |c_t| <= tol, or phibar_{t+1} <= tol ||b||, or on breakdown
 * (beta or alpha exactly 0).  Blocking: returns when x is written.
 * Errors: SAP_EINVAL (shapes, dtype/mode mismatch, non-finite b, non-finite A
 * found through a non-finite diagonal of the sketch's R),
 * SAP_ENOMEM, SAP_RANK_DEFICIENT (x untouched), SAP_NOT_CONVERGED (x holds
 * the last iterate), SAP_EDEVICE. */
sap_status sap_solve(sap_ctx *ctx, const sap_problem *prob, const sap_params *params, double *x,
                     sap_info *info, void *stream);

/* Gradient descent with heavy-ball momentum (App. D.3) as the iterative
 * method of Alg. 1, in place of LSQR: x_{t+1} = x_t + alpha g + beta (x_t -
 * x_{t-1}) with g = M M^T A^T (b - A x_t), one fused pass over A a step.
 * alpha > 0 takes (alpha, beta) as given (0 <= beta < 1); alpha <= 0 takes
 * the appendix's pair for the distortion estimate eta = eta_scale sqrt(n/d)
 * (eta_scale <= 0 means 1; the appendix mentions sqrt(1.1) for robustness):
 * alpha = (1 - eta^2)^2 and beta = eta^2, or with gradient_descent = 1
 * alpha = (1 - eta^2)^2 / (1 + eta^2) and beta = 0. */
typedef struct sap_hbm_params {
    double alpha;
    double beta;
    double eta_scale;
    int32_t gradient_descent;
    int32_t pad_;
} sap_hbm_params;

/* Alg. 1 with the momentum method of sap_hbm_params in place of LSQR: the
 * sketch, QR and x0 of sap_solve, then steps from x0.  params as for
 * sap_solve (d = 0 chooses d; fixed_iters runs a set number of steps); modes
 * FP64 and MIXED_FP32.  Stopping (the appendix leaves the test open;
 * reading, the counterpart of the LSQR test): stop at x_t, t >= 1, when
 * ||r_t|| = 0, ||M^T A^T r_t|| <= tol ||r_t|| or ||r_t|| <= tol ||b||, with
 * r_t = b - A x_t; at most maxiter steps.  info: iters = steps taken,
 * resid_est = ||r_t||, normar_est = ||M^T A^T r_t|| of the returned x.
 * The step direction is formed from r_t (the appendix writes it as
 * v - M M^T A^T A x_t with v = M M^T A^T b, the same vector in exact
 * arithmetic).  Blocking.  Errors as for sap_solve, and SAP_EINVAL for a
 * derived eta >= 1 or beta outside [0, 1). */
sap_status sap_solve_hbm(sap_ctx *ctx, const sap_problem *prob, const sap_params *params,
                         const sap_hbm_params *hbm, double *x, sap_info *info, void *stream);

/* The s-step form of App. D.4.2 in place of LSQR: the sketch, QR and x0 of
 * sap_solve, then blocks of s Krylov steps of the preconditioned normal
 * equations Z y = f, Z = (A M)^T (A M), M = R^-1.  Each block, from the
 * current x: r = b - A x and r0 = M^T A^T r (one pass over A); the stopping
 * test of sap_solve_hbm on (||r||, ||r0||) after at least one block; the
 * Chebyshev basis u_k = T_k((Z - c I)/h) r0, k < s, on the interval
 * [(1 - eta)^2, (1 + eta)^2] the embedding bound gives for Z's spectrum
 * (c, h its centre and half-width, eta = eta_scale sqrt(n/d), eta_scale 0
 * meaning 1), built without inner products, one pass over A per step; then
 * x += M U c with (U^T Z U) c = U^T r0, the CG iterate over x + M K_s(Z, r0)
 * in closed form (the Gram system is solved by Cholesky and truncated where
 * the basis turns numerically dependent).  s + 1 passes per block; blocks
 * run while fewer than maxiter steps are made (maxiter rounds up to whole
 * blocks).  params as for sap_solve (d = 0 chooses d; fixed_iters runs that
 * many steps, rounded up to whole blocks); modes FP64 and MIXED_FP32.
 * info: iters = steps made (s per block), resid_est = ||r||, normar_est =
 * ||r0|| at the last test.  The test measures the true residual, whose
 * normal-equation part has a rounding floor near u ||b||: tol far below
 * that relative to ||r|| is not reached on inconsistent problems.
 * Blocking.  Errors as for sap_solve, and SAP_EINVAL for s outside [1, 16]
 * or a derived eta >= 1. */
typedef struct sap_sstep_params {
    int32_t s;          /* Krylov steps per block, 1..16 */
    int32_t pad_;
    double eta_scale;   /* eta = eta_scale sqrt(n/d); 0 means 1 */
} sap_sstep_params;

sap_status sap_solve_sstep(sap_ctx *ctx, const sap_problem *prob, const sap_params *params,
                           const sap_sstep_params *ss, double *x, sap_info *info, void *stream);

/* Preconditioned LSQR alone (Alg. 2) on A M with M = R^-1 for a given R
 * (device, upper triangle of column-major n x n, leading dimension ldr) and
 * initial guess x0 (device, n doubles; may alias x).  A may be F64 or F32
 * (FP32 storage, FP64 arithmetic as in SAP_MODE_MIXED_FP32).  Blocking.  Same stopping rule and errors as
 * sap_solve. */
sap_status sap_lsqr(sap_ctx *ctx, const sap_problem *prob, const double *R, int64_t ldr,
                    const double *x0, double tol, int32_t maxiter, double *x, sap_info *info,
                    void *stream);

/* ------------------------------------------------------------------------
 * Sparse A (Sec. 3 applies the sketch to sparse matrices; Table 1 holds
 * sparse problems).  CSR form, all arrays on the device, owned by the
 * caller: row i holds the entries indptr[i] .. indptr[i+1]-1, with columns
 * indices[e] in [0, n) and values values[e] (F64, or F32 for the MIXED_FP32
 * mode); entries with a column outside [0, n) are ignored.  Limits: n <=
 * 8192, m < 2^31.
 * ---------------------------------------------------------------------- */
typedef struct sap_csr {
    int64_t m;               /* rows */
    int32_t n;               /* columns */
    int64_t nnz;             /* stored entries (= indptr[m]) */
    const int64_t *indptr;   /* device, m + 1 */
    const int32_t *indices;  /* device, nnz */
    const void *values;      /* device, nnz of v_type */
    sap_dtype v_type;        /* F64 or F32 */
} sap_csr;

/* Y = S [A b] for a CSR A (the sketching step of Alg. 1), Y column-major FP64
 * d x (n + (b != NULL)), ldy >= d, d < 20000, in O(zeta (nnz + m)) work:
 * the stored entries only.  The CSR arrays are checked on the device:
 * indptr[0] = 0, indptr[m] = nnz, indptr non-decreasing, every column index
 * in [0, n); column indices need not be sorted within a row.  The work is
 * planned on the device; the call blocks only to read the check's result.
 * Errors: SAP_EINVAL (shapes, the sketch's m differs from A's, a CSR array
 * that fails the check: Y is then undefined), SAP_ENOMEM. */
sap_status sps_apply_csr(sap_ctx *ctx, const sps_sketch *S, const sap_csr *A, const double *b, double *Y,
                         int64_t ldy, void *stream);

/* Alg. 1 and Alg. 2 for a CSR A: the sketch applied to the stored entries
 * (sps_apply_csr), the QR and x0 as in sap_solve, and LSQR whose pass
 * computes A p and A^T u from the stored entries in one sweep.  params as
 * for sap_solve; modes FP64 (F64 values) and MIXED_FP32 (F32 values, FP64
 * arithmetic); d = 0 takes eq. (4.2)'s d (cost ratio 1) within d <= 16384;
 * fixed_iters as for sap_solve.  b: device, m doubles.  Blocking.  Errors as
 * for sap_solve. */
sap_status sap_solve_csr(sap_ctx *ctx, const sap_csr *A, const double *b, const sap_params *params, double *x,
                         sap_info *info, void *stream);

/* Many independent problems solved together (the batched form): each phase of
 * Alg. 1 is one launch over all problems, and the LSQR iterations of all
 * problems advance together (replayed from a captured hipGraph) until every
 * problem has met its own stopping test or its maxiter.  probs, params, x and
 * info are host arrays of `count` entries; x[k] is a device pointer to n_k
 * doubles.  All problems share one A dtype (F32 or F64); each has its own m,
 * n, d, zeta, seed, tol, maxiter, mode and max_refine.  The sketch of
 * problem k uses Philox stream word k.  The sketch apply accumulates in FP64.
 * Modes: SAP_MODE_FP64 and SAP_MODE_MIXED_FP32 run every pass in FP64
 * arithmetic over A in its storage type, to the stopping test of sap_solve;
 * SAP_MODE_MIXED_FP32_REFINE (FP32 A) is the refinement form of sap_solve
 * (FP32 inner passes and u, FP64 residual at each restart, tol = target
 * relative correction, max_refine as there), with its outer loop kept on
 * the device so that the problem advances with the batch; info[k].refinements
 * counts its inner solves.  SAP_MODE_MIXED_BF16SA gives SAP_EINVAL.
 * Limits: 1 <= count <= 65535 (the problems index a grid dimension), n <= 1024,
 * d <= 4096 (a strip of the sketch lives in LDS), m < 2^31.  Blocking.  Returns SAP_OK when every
 * problem converged, SAP_NOT_CONVERGED when some did not or were rank
 * deficient (per-problem status in info[k].status); SAP_EINVAL, SAP_ENOMEM,
 * SAP_EDEVICE as for sap_solve. */
sap_status sap_solve_batch(sap_ctx *ctx, int32_t count, const sap_problem *probs, const sap_params *params,
                           double *const *x, sap_info *info, void *stream);

/* ------------------------------------------------------------------------
 * Served form (continuous batching).  A scheduler thread owned by the
 * context admits submitted problems first in, first out whenever their
 * workspace fits in a device arena reserved for serving, and advances all
 * admitted problems together: each round runs the setup phases of Alg. 1
 * (sketch, apply, QR, x0) for the problems admitted since the last round as
 * one batch, then a few LSQR iterations (Alg. 2) of every active problem as
 * one batch; a problem retires at the end of the round in which it meets its
 * stopping test (same test as sap_solve) or its maxiter, and its memory goes
 * back to the arena.  A problem's sketch is the one sap_solve draws for the
 * same seed, and its result does not depend on what else is in flight
 * beyond the rounding order of the sketch accumulation.  Limits and modes
 * as for sap_solve_batch (a request in the refinement form retires when its
 * outer loop stops); all problems of one context share one A dtype.
 * ---------------------------------------------------------------------- */

/* Start serving with an arena of arena_bytes of device memory (0: half the
 * context's HBM budget, at most 64 GiB) and at most max_active problems in
 * flight (1..4096).  Optional: the first sap_submit starts serving with the
 * defaults (arena 0, max_active 1024).  Errors: SAP_EINVAL (already serving,
 * bad max_active), SAP_ENOMEM. */
sap_status sap_serve_start(sap_ctx *ctx, size_t arena_bytes, int32_t max_active);

/* Queue one problem.  prob->A, prob->b (device) and x (device, n doubles,
 * the output) must stay valid and unmodified until sap_poll reports a
 * terminal status for the ticket.  The inputs count as written once the
 * work already queued on `stream` has run (the scheduler waits on an event
 * recorded there).  Non-blocking; *ticket identifies the request.  Errors:
 * SAP_EINVAL (shapes, parameters, dtype differing from earlier requests),
 * SAP_ENOMEM (the problem can never fit in the arena), SAP_EDEVICE (serving
 * stopped after a device error). */
sap_status sap_submit(sap_ctx *ctx, const sap_problem *prob, const sap_params *params, double *x, uint64_t *ticket,
                      void *stream);

/* State of a request.  wait != 0 blocks until it is finished; x is complete
 * on the device when a terminal status is returned.  Returns
 * SAP_PENDING while queued or running; otherwise the request's final status
 * (SAP_OK, SAP_NOT_CONVERGED, SAP_RANK_DEFICIENT, SAP_ECANCELED,
 * SAP_EDEVICE), fills *info (nullable; t_queue_ms and t_total_ms are the
 * host-clock queueing time and submit-to-finish latency) and forgets the
 * ticket: polling it again gives SAP_EINVAL. */
sap_status sap_poll(sap_ctx *ctx, uint64_t ticket, sap_info *info, int32_t wait);

/* Ask a request to stop: a queued one is dropped, a running one retires at
 * the end of the current round (x then holds its last iterate).  Its poll
 * status becomes SAP_ECANCELED.  Errors: SAP_EINVAL (unknown ticket). */
sap_status sap_cancel(sap_ctx *ctx, uint64_t ticket);

/* Serving counters, 7 int64 values: submitted, completed, active, queued,
 * rejected, arena bytes in use, arena bytes. */
sap_status sap_serve_stats(sap_ctx *ctx, int64_t *stats);

/* ------------------------------------------------------------------------
 * Embedding dimension (Sec. 4.3).  Host-only: no device work, no context,
 * callable before sap_create and without a GPU.
 *
 * sap_embedding_dim: the d of eq. (4.2), d = n exp(W(-r m log(eps) / n^2))
 * with W the principal branch of the Lambert W function: the d at which the
 * iteration work (log eps / log(n/d)) m n, weighted by r = cost_ratio, equals
 * the QR work d n^2.  cost_ratio is the time per unit of iteration work
 * (one m x n pass over A) divided by the time per unit of QR work; the
 * paper's form is 1.  The real d is rounded up and clamped to
 * [n + 1, min(m, INT32_MAX)].  *d receives the result.
 * Errors: SAP_EINVAL (d null, n < 1, m <= n, eps outside (0, 1), cost_ratio
 * not finite and positive, or the argument of W not finite); *d is then
 * untouched.
 * ---------------------------------------------------------------------- */
sap_status sap_embedding_dim(int64_t m, int32_t n, double eps, double cost_ratio, int32_t *d);
/* sap_iteration_estimate: the iterations after which the rate estimate of
 * eq. (4.1), (n/d)^(t/2), reaches eps: t = ceil(2 log eps / log(n/d)).
 * Errors: SAP_EINVAL (iters null, n < 1, d <= n, eps outside (0, 1)). */
sap_status sap_iteration_estimate(int32_t n, int32_t d, double eps, int32_t *iters);

/* Machine-aware embedding dimension for one problem (device work and a
 * context, unlike the two calls above; Sec. 4.3 weighs the QR
 * against the iterations; here every phase is timed on this GPU).  Among the
 * candidates d = k n (k = 1.25, 1.5, 2, 2.5, 3, 4, 5, 6, 8, 10, 12) and
 * eq. (4.2)'s d, clipped to [n + 1, min(m, 16384)], it returns the one that
 * minimises apply(d) + qr(d) + (t(d) + 1) (a m + f): t(d) the eq. (4.1)
 * iteration estimate for eps, apply(d) the sketch apply timed on the first
 * min(m, 65536) rows of the caller's A and scaled to m, qr(d) the QR of that
 * d x (n + 1) sketch, and a m + f the cost of one LSQR iteration fitted from
 * iterations timed on that slab and on half of it.  The timings are taken
 * once per context for each (n, dtype, zeta, candidate d) and cached; the
 * first call for a width costs roughly a few QRs.  Problems with m < 4096
 * get eq. (4.2)'s d.  Blocking on `stream`; uses the context workspace.
 * Errors: SAP_EINVAL (problem, zeta, eps outside (0, 1)), SAP_ENOMEM,
 * SAP_EDEVICE. */
sap_status sap_choose_d(sap_ctx *ctx, const sap_problem *prob, int32_t zeta, double eps, int32_t *d,
                        void *stream);


/* ------------------------------------------------------------------------
 * Kernel timing (measurement support).  When enabled, the library brackets
 * every launch of its two bandwidth-bound kernels with HIP events on the
 * stream it launches them on, and accumulates their durations:
 *   kernel 0 = the fused LSQR pass over A (u <- c (A p) + c' u, q = A^T u),
 *   kernel 1 = the sketch apply (S [A b] accumulation, plus its slice
 *              reduction when there is one).
 * Events are resolved at the end of each blocking call (sap_solve,
 * sap_lsqr) or by sap_profile_read.  Disabled by default.
 * ---------------------------------------------------------------------- */
sap_status sap_profile_enable(sap_ctx *ctx, int enable);
/* Reset (reset != 0) or read the totals: launches and summed milliseconds. */
sap_status sap_profile_read(sap_ctx *ctx, int32_t kernel, int64_t *launches, double *total_ms, int reset);

#ifdef __cplusplus
}
#endif

#endif /* SAP_H */
