/*
 * Plain CPU oracle for sketch-and-precondition least squares with sparse sign
 * sketches (Chen, Epperly, et al., arXiv 2506.03070).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, calls or
 * includes this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * constant generator with the HIP path.
 *
 * Everything is double precision, single-threaded and written in the order of
 * the paper's definitions so that it can be checked against the paper by eye:
 *
 *   - Philox4x64-10 counter-based RNG (Salmon, Moraes, Dror, Shaw, SC'11).
 *     The paper does not name its generator (Alg. 3 draws with a library
 *     randint), so the stream layout below is this project's reading.
 *   - Lemire's multiply-shift bounded integer with rejection (ACM TOMACS 2019)
 *     for exactly uniform draws in [0, d).
 *   - Rejection-sampled column generation (Sec. 3.1.2 and Alg. 3): draw zeta
 *     rows with replacement, sort, redraw the first entry of every equal
 *     neighbour pair, repeat until distinct.  Signs +-1/sqrt(zeta) (Alg. 3),
 *     attached to the sorted positions.
 *   - Sketch apply Y = S [A b] (the sketching step of Alg. 1), dense and
 *     sparse route.
 *   - Unblocked Householder QR with the LAPACK dlarfg sign convention
 *     (the factorization step of Alg. 1).
 *   - Back / forward substitution with R and R^T (the preconditioner M = R^-1
 *     of Alg. 1 applied by triangular solves).
 *   - Preconditioned LSQR exactly as Alg. 2 (Paige & Saunders 1982).
 *   - The whole of Alg. 1, and a direct Householder solve of [A b] for tiny
 *     problems.
 *   - The same for a sparse A in CSR form: products, sketch apply, LSQR and
 *     Alg. 1 on the stored entries, in the order of the dense routes.
 *   - Gradient descent with heavy-ball momentum (App. D.3) in place of LSQR,
 *     with the step size and momentum the appendix derives from the
 *     distortion estimate.
 *   - The s-step form of App. D.4.2: blocks of s Krylov steps, each the CG
 *     iterate over the block's Krylov space in closed form, from a
 *     Chebyshev basis (no inner products while it is built).
 *
 * Parity pins for each function live in the CPU test suite.
 */
#define _POSIX_C_SOURCE 199309L
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

typedef unsigned __int128 orc_u128;

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (SC'11, Sec. 5): two 64x64->128 multiplies per round, key    */
/* bumped by the Weyl constants between rounds.                               */
/* ------------------------------------------------------------------------ */
#define ORC_PHILOX_M0 0xD2E7470EE14C6C93ULL
#define ORC_PHILOX_M1 0xCA5A826395121157ULL
#define ORC_PHILOX_W0 0x9E3779B97F4A7C15ULL
#define ORC_PHILOX_W1 0xBB67AE8584CAA73BULL

void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += ORC_PHILOX_W0;
            k1 += ORC_PHILOX_W1;
        }
        orc_u128 prod0 = (orc_u128)ORC_PHILOX_M0 * x0;
        orc_u128 prod1 = (orc_u128)ORC_PHILOX_M1 * x2;
        uint64_t y0 = (uint64_t)(prod1 >> 64) ^ x1 ^ k0;
        uint64_t y1 = (uint64_t)prod1;
        uint64_t y2 = (uint64_t)(prod0 >> 64) ^ x3 ^ k1;
        uint64_t y3 = (uint64_t)prod0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Stream layout (project reading; the paper leaves the generator open):
 *   key     = (seed, stream)
 *   w(i,r,j,k) = word (j mod 4) of Philox(key, counter = (i, r, floor(j/4), k))
 *   column i's sign word = word 0 of Philox(key, counter = (i, 2^64-1, 0, 0))   */
uint64_t orc_word(uint64_t seed, uint64_t stream, uint64_t i, uint64_t r, uint64_t j, uint64_t k)
{
    uint64_t ctr[4] = {i, r, j / 4, k};
    uint64_t key[2] = {seed, stream};
    uint64_t out[4];
    orc_philox4x64_10(ctr, key, out);
    return out[j % 4];
}

uint64_t orc_sign_word(uint64_t seed, uint64_t stream, uint64_t i)
{
    uint64_t ctr[4] = {i, ~(uint64_t)0, 0, 0};
    uint64_t key[2] = {seed, stream};
    uint64_t out[4];
    orc_philox4x64_10(ctr, key, out);
    return out[0];
}

/* One step of Lemire's method: returns 1 and writes floor(w*d / 2^64) when the
 * low half of w*d is at least (2^64 - d) mod d, else returns 0 (reject). */
int orc_lemire_step(uint64_t w, uint64_t d, uint64_t *value)
{
    orc_u128 prod = (orc_u128)w * d;
    uint64_t low = (uint64_t)prod;
    uint64_t threshold = (0 - d) % d; /* (2^64 - d) mod d */
    if (low < threshold)
        return 0;
    *value = (uint64_t)(prod >> 64);
    return 1;
}

/* U(i,r,j): exactly uniform in [0,d) from the words w(i,r,j,k), k = 0,1,... */
uint64_t orc_bounded(uint64_t seed, uint64_t stream, uint64_t i, uint64_t r, uint64_t j, uint64_t d)
{
    uint64_t value = 0;
    for (uint64_t k = 0;; ++k) {
        if (orc_lemire_step(orc_word(seed, stream, i, r, j, k), d, &value))
            return value;
    }
}

static void orc_sort_ascending(int64_t *c, int n)
{
    /* insertion sort: the columns hold at most 64 entries */
    for (int a = 1; a < n; ++a) {
        int64_t key = c[a];
        int b = a - 1;
        while (b >= 0 && c[b] > key) {
            c[b + 1] = c[b];
            --b;
        }
        c[b + 1] = key;
    }
}

#define ORC_MAX_ZETA 64
#define ORC_MAX_ROUNDS (1 << 16)

/* Column i of the sparse sign sketch (Sec. 3.1.2 steps (i)-(iv); Alg. 3).
 * Writes zeta ascending distinct rows and the sign word masked to zeta bits.
 * Returns the number of redraw rounds used, or -1 on invalid arguments or if
 * the round cap is hit (which needs zeta close to d and astronomically bad
 * luck).  Redraw rule: on the sorted column, every position j with
 * c[j] == c[j+1] (found before any replacement) is redrawn from U(i, r, j). */
int orc_sketch_column(uint64_t seed, uint64_t stream, uint64_t i, int32_t d, int32_t zeta,
                      int32_t *idx_out, uint64_t *sign_out)
{
    if (zeta < 1 || zeta > ORC_MAX_ZETA || d < zeta)
        return -1;
    int64_t c[ORC_MAX_ZETA];
    int dup[ORC_MAX_ZETA];
    for (int j = 0; j < zeta; ++j)
        c[j] = (int64_t)orc_bounded(seed, stream, i, 0, (uint64_t)j, (uint64_t)d);
    orc_sort_ascending(c, zeta);
    int rounds = 0;
    for (uint64_t r = 1;; ++r) {
        int any = 0;
        for (int j = 0; j + 1 < zeta; ++j) {
            dup[j] = (c[j] == c[j + 1]);
            any |= dup[j];
        }
        if (!any)
            break;
        if (r >= ORC_MAX_ROUNDS)
            return -1;
        for (int j = 0; j + 1 < zeta; ++j)
            if (dup[j])
                c[j] = (int64_t)orc_bounded(seed, stream, i, r, (uint64_t)j, (uint64_t)d);
        orc_sort_ascending(c, zeta);
        rounds = (int)r;
    }
    for (int j = 0; j < zeta; ++j)
        idx_out[j] = (int32_t)c[j];
    uint64_t mask = (zeta == 64) ? ~(uint64_t)0 : (((uint64_t)1 << zeta) - 1);
    *sign_out = orc_sign_word(seed, stream, i) & mask;
    return rounds;
}

/* The whole sketch: idx is m x zeta (row i = column i of S), sign has m words.
 * rounds_out (nullable) receives the per-column round counts.  Returns 0, or
 * -1 on invalid arguments. */
int orc_sketch(uint64_t seed, uint64_t stream, int64_t m, int32_t d, int32_t zeta,
               int32_t *idx, uint64_t *sign, int32_t *rounds_out)
{
    for (int64_t i = 0; i < m; ++i) {
        int rr = orc_sketch_column(seed, stream, (uint64_t)i, d, zeta, idx + i * zeta, sign + i);
        if (rr < 0)
            return -1;
        if (rounds_out)
            rounds_out[i] = rr;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sketch apply Y = h * sum_i sum_k s_ik e_{idx[i][k]} [A b](i, :)            */
/* h = 1/sqrt(zeta) (Alg. 3 values), s_ik = +1 if bit k of sign[i] else -1.   */
/* A is row-major m x n (lda), b has m entries (nullable: then only n columns */
/* are formed), Y is column-major d x ncols (ldy).                            */
/* ------------------------------------------------------------------------ */

/* Sparse route: accumulate with i ascending, k ascending; scale once at the
 * end.  cols (nullable) restricts the work to a list of ncols_sel columns of
 * [A b]; column c of the selection goes to Y column c. */
void orc_apply_sparse(int64_t m, int32_t d, int32_t zeta, const int32_t *idx, const uint64_t *sign,
                      const double *A, int64_t lda, const double *b, int32_t n, double h,
                      double *Y, int64_t ldy, const int32_t *cols, int32_t ncols_sel)
{
    int32_t ncols = cols ? ncols_sel : (b ? n + 1 : n);
    for (int32_t cc = 0; cc < ncols; ++cc)
        for (int32_t r = 0; r < d; ++r)
            Y[r + (int64_t)cc * ldy] = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        for (int32_t cc = 0; cc < ncols; ++cc) {
            int32_t c = cols ? cols[cc] : cc;
            double a = (c < n) ? A[i * lda + c] : b[i];
            for (int k = 0; k < zeta; ++k) {
                int32_t r = idx[i * zeta + k];
                double s = ((sign[i] >> k) & 1) ? 1.0 : -1.0;
                Y[r + (int64_t)cc * ldy] += s * a;
            }
        }
    }
    for (int32_t cc = 0; cc < ncols; ++cc)
        for (int32_t r = 0; r < d; ++r)
            Y[r + (int64_t)cc * ldy] *= h;
}

/* Dense route: build the +-1 pattern of S (d x m) explicitly, triple loop,
 * then scale by h.  For small m only. */
void orc_apply_dense(int64_t m, int32_t d, int32_t zeta, const int32_t *idx, const uint64_t *sign,
                     const double *A, int64_t lda, const double *b, int32_t n, double h,
                     double *Y, int64_t ldy)
{
    int32_t ncols = b ? n + 1 : n;
    double *S = (double *)calloc((size_t)d * (size_t)m, sizeof(double));
    for (int64_t i = 0; i < m; ++i)
        for (int k = 0; k < zeta; ++k)
            S[(int64_t)idx[i * zeta + k] * m + i] = ((sign[i] >> k) & 1) ? 1.0 : -1.0;
    for (int32_t r = 0; r < d; ++r) {
        for (int32_t c = 0; c < ncols; ++c) {
            double acc = 0.0;
            for (int64_t i = 0; i < m; ++i) {
                double a = (c < n) ? A[i * lda + c] : b[i];
                acc += S[(int64_t)r * m + i] * a;
            }
            Y[r + (int64_t)c * ldy] = h * acc;
        }
    }
    free(S);
}

/* ------------------------------------------------------------------------ */
/* Householder QR (Golub & Van Loan, Alg. 5.2.1) with the LAPACK dlarfg sign  */
/* convention: beta = -sign(alpha) * ||(alpha, x)||, tau = (beta - alpha) /    */
/* beta, v = (1, x / (alpha - beta)).  In place on Y (rows x cols, ldy):      */
/* R in the upper triangle, v below the diagonal, tau[k] per reflector.       */
/* ------------------------------------------------------------------------ */
void orc_householder_qr(double *Y, int64_t ldy, int32_t rows, int32_t cols, double *tau)
{
    int32_t kmax = rows < cols ? rows : cols;
    for (int32_t k = 0; k < kmax; ++k) {
        double *col = Y + (int64_t)k * ldy;
        double alpha = col[k];
        double ss = 0.0;
        for (int32_t i = k + 1; i < rows; ++i)
            ss += col[i] * col[i];
        if (ss == 0.0) {
            tau[k] = 0.0; /* H = I */
            continue;
        }
        double norm = sqrt(alpha * alpha + ss);
        double beta = (alpha >= 0.0) ? -norm : norm;
        tau[k] = (beta - alpha) / beta;
        double scale = 1.0 / (alpha - beta);
        for (int32_t i = k + 1; i < rows; ++i)
            col[i] *= scale;
        col[k] = beta;
        for (int32_t j = k + 1; j < cols; ++j) {
            double *cj = Y + (int64_t)j * ldy;
            double w = cj[k];
            for (int32_t i = k + 1; i < rows; ++i)
                w += col[i] * cj[i];
            cj[k] -= tau[k] * w;
            for (int32_t i = k + 1; i < rows; ++i)
                cj[i] -= tau[k] * w * col[i];
        }
    }
}

/* Solve R x = rhs, R upper triangular n x n stored column-major in the upper
 * triangle of (R, ldr).  Row k: x_k = (rhs_k - sum_{j>k} R[k,j] x_j) / R[k,k],
 * inner sum with j ascending. */
void orc_backsub(const double *R, int64_t ldr, int32_t n, const double *rhs, double *x)
{
    for (int32_t k = n - 1; k >= 0; --k) {
        double acc = rhs[k];
        for (int32_t j = k + 1; j < n; ++j)
            acc -= R[k + (int64_t)j * ldr] * x[j];
        x[k] = acc / R[k + (int64_t)k * ldr];
    }
}

/* Solve R^T y = rhs (forward substitution with the lower triangular R^T). */
void orc_forwardsub_t(const double *R, int64_t ldr, int32_t n, const double *rhs, double *y)
{
    for (int32_t k = 0; k < n; ++k) {
        double acc = rhs[k];
        for (int32_t j = 0; j < k; ++j)
            acc -= R[j + (int64_t)k * ldr] * y[j];
        y[k] = acc / R[k + (int64_t)k * ldr];
    }
}

/* y = A x (row dots, columns ascending) and y = A^T u (rows ascending). */
void orc_matvec(int64_t m, int32_t n, const double *A, int64_t lda, const double *x, double *y)
{
    for (int64_t i = 0; i < m; ++i) {
        double acc = 0.0;
        for (int32_t c = 0; c < n; ++c)
            acc += A[i * lda + c] * x[c];
        y[i] = acc;
    }
}

void orc_matvec_t(int64_t m, int32_t n, const double *A, int64_t lda, const double *u, double *y)
{
    for (int32_t c = 0; c < n; ++c)
        y[c] = 0.0;
    for (int64_t i = 0; i < m; ++i)
        for (int32_t c = 0; c < n; ++c)
            y[c] += A[i * lda + c] * u[i];
}

static double orc_nrm2(int64_t n, const double *x)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += x[i] * x[i];
    return sqrt(s);
}

/* LSQR result record shared with the Python wrapper. */
typedef struct orc_lsqr_info {
    int32_t iters;     /* iterations taken */
    int32_t converged; /* 1 when a stopping test fired before maxiter */
    double resid_est;  /* phibar_{t+1} = ||b - A x_t|| estimate */
    double normar_est; /* phibar_{t+1} alpha_{t+1} |c_t| = ||(AM)^T r_t|| estimate */
} orc_lsqr_info;

/* Preconditioned LSQR, Alg. 2, on the operator A M with M = R^-1 applied by
 * triangular solves.  history (nullable, maxiter+1 rows of n) receives x_0,
 * x_1, ... for iterate-level comparisons.
 *
 * Stopping (the paper only says "test for convergence"; reading after Paige &
 * Saunders with ||AM|| ~ 1 from Lemma 2.4): stop after iteration t when
 *   alpha_{t+1} |c_t| <= tol          (relative normal-equation residual), or
 *   phibar_{t+1} <= tol * ||b||       (compatible system), or
 *   beta_{t+1} == 0 or alpha_{t+1} == 0 (breakdown: x_t is exact).
 * maxiter <= 0 runs no iteration and returns x0. */
/* The operator A of the least-squares problem: y = A x (m entries) and
 * y = A^T u (n entries), for a dense or a CSR matrix. */
typedef struct orc_op {
    void (*av)(const void *ctx, const double *x, double *y);
    void (*atv)(const void *ctx, const double *u, double *y);
    const void *ctx;
} orc_op;

static void orc_lsqr_op(int64_t m, int32_t n, const orc_op *op, const double *b,
                        const double *R, int64_t ldr, const double *x0, double tol, int32_t maxiter,
                        double *x, double *history, orc_lsqr_info *info)
{
    double *u = (double *)malloc(sizeof(double) * (size_t)m);
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    double *p = (double *)malloc(sizeof(double) * (size_t)n);
    double *t1 = (double *)malloc(sizeof(double) * (size_t)n);
    double *t2 = (double *)malloc(sizeof(double) * (size_t)n);

    memcpy(x, x0, sizeof(double) * (size_t)n);
    if (history)
        memcpy(history, x0, sizeof(double) * (size_t)n);
    info->iters = 0;
    info->converged = 0;
    double normb = orc_nrm2(m, b);

    /* beta_1 u_1 = b - A x_0 */
    op->av(op->ctx, x0, u);
    for (int64_t i = 0; i < m; ++i)
        u[i] = b[i] - u[i];
    double beta = orc_nrm2(m, u);
    info->resid_est = beta;
    info->normar_est = 0.0;
    if (beta == 0.0 || maxiter <= 0) {
        info->converged = (beta == 0.0);
        goto done;
    }
    for (int64_t i = 0; i < m; ++i)
        u[i] /= beta;
    /* alpha_1 v_1 = M^T A^T u_1 */
    op->atv(op->ctx, u, t1);
    orc_forwardsub_t(R, ldr, n, t1, t2);
    double alpha = orc_nrm2(n, t2);
    info->normar_est = alpha * beta;
    if (alpha == 0.0) {
        info->converged = 1;
        goto done;
    }
    for (int32_t c = 0; c < n; ++c)
        v[c] = t2[c] / alpha;
    /* w_1 = M v_1 */
    orc_backsub(R, ldr, n, v, w);
    memcpy(p, w, sizeof(double) * (size_t)n);
    double phibar = beta, rhobar = alpha;

    {
        double *Ap = (double *)malloc(sizeof(double) * (size_t)m);
        for (int32_t t = 1; t <= maxiter; ++t) {
            /* u_hat = A M v_t - alpha_t u_t ; beta_{t+1} = ||u_hat|| */
            op->av(op->ctx, p, Ap);
            for (int64_t i = 0; i < m; ++i)
                Ap[i] -= alpha * u[i];
            beta = orc_nrm2(m, Ap);
            double alpha_next = 0.0;
            if (beta != 0.0) {
                for (int64_t i = 0; i < m; ++i)
                    u[i] = Ap[i] / beta;
                /* v_hat = M^T A^T u_{t+1} - beta_{t+1} v_t ; alpha_{t+1} = ||v_hat|| */
                op->atv(op->ctx, u, t1);
                orc_forwardsub_t(R, ldr, n, t1, t2);
                for (int32_t c = 0; c < n; ++c)
                    t2[c] -= beta * v[c];
                alpha_next = orc_nrm2(n, t2);
                if (alpha_next != 0.0)
                    for (int32_t c = 0; c < n; ++c)
                        v[c] = t2[c] / alpha_next;
            }
            /* plane rotation */
            double rho = sqrt(rhobar * rhobar + beta * beta);
            double cs = rhobar / rho;
            double sn = beta / rho;
            double theta = sn * alpha_next;
            rhobar = -cs * alpha_next;
            double phi = cs * phibar;
            phibar = sn * phibar;
            /* x_t = x_{t-1} + (phi_t / rho_t) w_t */
            for (int32_t c = 0; c < n; ++c)
                x[c] += (phi / rho) * w[c];
            /* w_{t+1} = M v_{t+1} - (theta_{t+1} / rho_t) w_t */
            if (alpha_next != 0.0 && beta != 0.0) {
                orc_backsub(R, ldr, n, v, p);
                for (int32_t c = 0; c < n; ++c)
                    w[c] = p[c] - (theta / rho) * w[c];
            }
            alpha = alpha_next;
            info->iters = t;
            info->resid_est = phibar;
            info->normar_est = phibar * alpha * fabs(cs);
            if (history)
                memcpy(history + (int64_t)t * n, x, sizeof(double) * (size_t)n);
            if (beta == 0.0 || alpha == 0.0 || alpha * fabs(cs) <= tol || phibar <= tol * normb) {
                info->converged = 1;
                break;
            }
        }
        free(Ap);
    }
done:
    free(u); free(v); free(w); free(p); free(t1); free(t2);
}

/* Dense row-major A (lda). */
typedef struct orc_dense { int64_t m; int32_t n; const double *A; int64_t lda; } orc_dense;
static void orc_dense_av(const void *ctx, const double *x, double *y)
{
    const orc_dense *D = (const orc_dense *)ctx;
    orc_matvec(D->m, D->n, D->A, D->lda, x, y);
}
static void orc_dense_atv(const void *ctx, const double *u, double *y)
{
    const orc_dense *D = (const orc_dense *)ctx;
    orc_matvec_t(D->m, D->n, D->A, D->lda, u, y);
}

void orc_lsqr(int64_t m, int32_t n, const double *A, int64_t lda, const double *b,
              const double *R, int64_t ldr, const double *x0, double tol, int32_t maxiter,
              double *x, double *history, orc_lsqr_info *info)
{
    orc_dense D = {m, n, A, lda};
    orc_op op = {orc_dense_av, orc_dense_atv, &D};
    orc_lsqr_op(m, n, &op, b, R, ldr, x0, tol, maxiter, x, history, info);
}

/* ------------------------------------------------------------------------ */
/* Sparse A in CSR form (Sec. 3 applies the sketch to sparse matrices; Table */
/* 1 holds sparse problems): row i holds entries indptr[i] .. indptr[i+1]-1  */
/* with columns indices[] ascending and values[].  Every sum below runs in   */
/* the order of the dense routes (rows ascending, columns ascending), only   */
/* skipping the zeros, so each CSR result equals the dense result on the     */
/* densified matrix bit for bit.                                              */
/* ------------------------------------------------------------------------ */
void orc_matvec_csr(int64_t m, const int64_t *indptr, const int32_t *indices, const double *values,
                    const double *x, double *y)
{
    for (int64_t i = 0; i < m; ++i) {
        double acc = 0.0;
        for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e)
            acc += values[e] * x[indices[e]];
        y[i] = acc;
    }
}

void orc_matvec_t_csr(int64_t m, int32_t n, const int64_t *indptr, const int32_t *indices,
                      const double *values, const double *u, double *y)
{
    for (int32_t c = 0; c < n; ++c)
        y[c] = 0.0;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e)
            y[indices[e]] += values[e] * u[i];
}

/* Sketch apply of [A b] with A in CSR: Y[r, c] gets s_ik a_ic for every
 * stored entry (i, c) and every k with idx[i][k] = r, rows ascending; column
 * n of Y is S b.  Scaled by h once at the end. */
void orc_apply_csr(int64_t m, int32_t d, int32_t zeta, const int32_t *idx, const uint64_t *sign,
                   const int64_t *indptr, const int32_t *indices, const double *values, const double *b,
                   int32_t n, double h, double *Y, int64_t ldy)
{
    int32_t ncols = b ? n + 1 : n;
    for (int32_t c = 0; c < ncols; ++c)
        for (int32_t r = 0; r < d; ++r)
            Y[r + (int64_t)c * ldy] = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e) {
            int32_t c = indices[e];
            for (int k = 0; k < zeta; ++k) {
                double s = ((sign[i] >> k) & 1) ? 1.0 : -1.0;
                Y[idx[i * zeta + k] + (int64_t)c * ldy] += s * values[e];
            }
        }
        if (b)
            for (int k = 0; k < zeta; ++k) {
                double s = ((sign[i] >> k) & 1) ? 1.0 : -1.0;
                Y[idx[i * zeta + k] + (int64_t)n * ldy] += s * b[i];
            }
    }
    for (int32_t c = 0; c < ncols; ++c)
        for (int32_t r = 0; r < d; ++r)
            Y[r + (int64_t)c * ldy] *= h;
}

typedef struct orc_csr { int64_t m; int32_t n; const int64_t *indptr; const int32_t *indices; const double *values; } orc_csr;
static void orc_csr_av(const void *ctx, const double *x, double *y)
{
    const orc_csr *C = (const orc_csr *)ctx;
    orc_matvec_csr(C->m, C->indptr, C->indices, C->values, x, y);
}
static void orc_csr_atv(const void *ctx, const double *u, double *y)
{
    const orc_csr *C = (const orc_csr *)ctx;
    orc_matvec_t_csr(C->m, C->n, C->indptr, C->indices, C->values, u, y);
}

void orc_lsqr_csr(int64_t m, int32_t n, const int64_t *indptr, const int32_t *indices, const double *values,
                  const double *b, const double *R, int64_t ldr, const double *x0, double tol, int32_t maxiter,
                  double *x, double *history, orc_lsqr_info *info)
{
    orc_csr C = {m, n, indptr, indices, values};
    orc_op op = {orc_csr_av, orc_csr_atv, &C};
    orc_lsqr_op(m, n, &op, b, R, ldr, x0, tol, maxiter, x, history, info);
}

/* ------------------------------------------------------------------------ */
/* Gradient descent with heavy-ball momentum (App. D.3) in place of LSQR.    */
/* ------------------------------------------------------------------------ */
/* Step size and momentum of App. D.3 for a distortion estimate
 * eta = c sqrt(n/d) (the paper's example takes c = 1 and mentions a larger c
 * for robustness): heavy ball alpha = (1 - eta^2)^2, beta = eta^2; gradient
 * descent (gd = 1) alpha = (1 - eta^2)^2 / (1 + eta^2), beta = 0.
 * Returns 1 (and leaves the outputs alone) when eta is not in [0, 1). */
int orc_hbm_params(int32_t n, int32_t d, double c, int32_t gd, double *alpha, double *beta)
{
    if (n < 1 || d < 1 || !(c > 0.0))
        return 1;
    double eta = c * sqrt((double)n / (double)d);
    if (!(eta < 1.0))
        return 1;
    double e2 = eta * eta;
    if (gd) {
        *alpha = (1.0 - e2) * (1.0 - e2) / (1.0 + e2);
        *beta = 0.0;
    } else {
        *alpha = (1.0 - e2) * (1.0 - e2);
        *beta = e2;
    }
    return 0;
}

/* M M^T y = R^-1 R^-T y (two triangular solves), into out; tmp holds n. */
static void orc_mmt(const double *R, int64_t ldr, int32_t n, const double *y, double *tmp, double *out)
{
    orc_forwardsub_t(R, ldr, n, y, tmp);
    orc_backsub(R, ldr, n, tmp, out);
}

/* The paper's iteration, in its order:
 *   x_{-1} = x_0,  v = M M^T A^T b,
 *   for t = 1, 2, ...:  g_t = v - M M^T A^T A x_{t-1},
 *                       x_t = x_{t-1} + alpha g_t + beta (x_{t-1} - x_{t-2}),
 *                       stopping test.
 * M = R^-1 by triangular solves.  The paper leaves the test open; reading (the
 * counterpart of the LSQR test, with ||AM|| ~ 1): with r_t = b - A x_t and
 * s_t = M^T A^T r_t, stop after update t when ||r_t|| = 0,
 * ||s_t|| <= tol ||r_t|| or ||r_t|| <= tol ||b||.  At most maxiter updates;
 * maxiter <= 0 returns x0.  info: iters = updates made, resid_est = ||r_t||,
 * normar_est = ||s_t|| of the returned x.  history (nullable, maxiter + 1 rows
 * of n) receives x_0, x_1, .... */
static void orc_hbm_op(int64_t m, int32_t n, const orc_op *op, const double *b, const double *R, int64_t ldr,
                       const double *x0, double alpha, double beta, double tol, int32_t maxiter, double *x,
                       double *history, orc_lsqr_info *info)
{
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    double *g = (double *)malloc(sizeof(double) * (size_t)n);
    double *xprev = (double *)malloc(sizeof(double) * (size_t)n);
    double *t1 = (double *)malloc(sizeof(double) * (size_t)n);
    double *t2 = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)m);

    memcpy(x, x0, sizeof(double) * (size_t)n);
    memcpy(xprev, x0, sizeof(double) * (size_t)n);
    if (history)
        memcpy(history, x0, sizeof(double) * (size_t)n);
    info->iters = 0;
    info->converged = 0;
    info->resid_est = 0.0;
    info->normar_est = 0.0;
    double normb = orc_nrm2(m, b);
    /* v = M M^T A^T b */
    op->atv(op->ctx, b, t1);
    orc_mmt(R, ldr, n, t1, t2, v);
    for (int32_t t = 1; t <= maxiter; ++t) {
        /* g_t = v - M M^T A^T A x_{t-1} */
        op->av(op->ctx, x, y);
        op->atv(op->ctx, y, t1);
        orc_mmt(R, ldr, n, t1, t2, g);
        for (int32_t c = 0; c < n; ++c)
            g[c] = v[c] - g[c];
        /* x_t = x_{t-1} + alpha g_t + beta (x_{t-1} - x_{t-2}) */
        for (int32_t c = 0; c < n; ++c) {
            double xn = x[c] + alpha * g[c] + beta * (x[c] - xprev[c]);
            xprev[c] = x[c];
            x[c] = xn;
        }
        info->iters = t;
        if (history)
            memcpy(history + (int64_t)t * n, x, sizeof(double) * (size_t)n);
        /* stopping test on r_t and s_t = M^T A^T r_t */
        op->av(op->ctx, x, y);
        for (int64_t i = 0; i < m; ++i)
            y[i] = b[i] - y[i];
        double rn = orc_nrm2(m, y);
        op->atv(op->ctx, y, t1);
        orc_forwardsub_t(R, ldr, n, t1, t2);
        double sn = orc_nrm2(n, t2);
        info->resid_est = rn;
        info->normar_est = sn;
        if (rn == 0.0 || sn <= tol * rn || rn <= tol * normb) {
            info->converged = 1;
            break;
        }
    }
    free(v); free(g); free(xprev); free(t1); free(t2); free(y);
}

void orc_hbm(int64_t m, int32_t n, const double *A, int64_t lda, const double *b, const double *R, int64_t ldr,
             const double *x0, double alpha, double beta, double tol, int32_t maxiter, double *x, double *history,
             orc_lsqr_info *info)
{
    orc_dense D = {m, n, A, lda};
    orc_op op = {orc_dense_av, orc_dense_atv, &D};
    orc_hbm_op(m, n, &op, b, R, ldr, x0, alpha, beta, tol, maxiter, x, history, info);
}

/* ------------------------------------------------------------------------ */
/* s-step form (App. D.4.2).                                                  */
/* ------------------------------------------------------------------------ */
/* Z u = M^T A^T A M u with M = R^-1 (triangular solves); tn (n) and tm (m)
 * are scratch. */
static void orc_z_apply(int64_t m, int32_t n, const orc_op *op, const double *R, int64_t ldr, const double *u,
                        double *tn, double *tm, double *out)
{
    orc_backsub(R, ldr, n, u, tn);      /* M u */
    op->av(op->ctx, tn, tm);            /* A M u */
    op->atv(op->ctx, tm, out);          /* A^T A M u */
    orc_forwardsub_t(R, ldr, n, out, tn);
    memcpy(out, tn, sizeof(double) * (size_t)n);  /* M^T A^T A M u */
    (void)m;
}

/* Chebyshev basis of the Krylov space K_s(Z, r0), Z = (A M)^T (A M), on the
 * interval [lo, hi] that the sketch's distortion puts around Z's spectrum
 * (centre c = (hi + lo)/2, half-width h = (hi - lo)/2):
 *   u_0 = r0,  u_1 = (Z u_0 - c u_0) / h,
 *   u_{k+1} = 2 (Z u_k - c u_k) / h - u_{k-1},
 * that is u_k = T_k((Z - c I)/h) r0; no inner products are taken.
 * U (n x s, column-major, ld n) receives u_0 .. u_{s-1}; W (n x s) receives
 * Z u_0 .. Z u_{s-1}.  Needs hi > lo. */
static void orc_cheb_basis_op(int64_t m, int32_t n, const orc_op *op, const double *R, int64_t ldr,
                              const double *r0, int32_t s, double lo, double hi, double *U, double *W)
{
    double *tn = (double *)malloc(sizeof(double) * (size_t)n);
    double *tm = (double *)malloc(sizeof(double) * (size_t)m);
    const double c = 0.5 * (hi + lo), h = 0.5 * (hi - lo);
    memcpy(U, r0, sizeof(double) * (size_t)n);
    for (int32_t k = 0; k < s; ++k) {
        const double *uk = U + (int64_t)k * n;
        double *wk = W + (int64_t)k * n;
        orc_z_apply(m, n, op, R, ldr, uk, tn, tm, wk);
        if (k + 1 < s) {
            double *un = U + (int64_t)(k + 1) * n;
            for (int32_t i = 0; i < n; ++i) {
                const double y = (wk[i] - c * uk[i]) / h;
                un[i] = (k == 0) ? y : 2.0 * y - U[(int64_t)(k - 1) * n + i];
            }
        }
    }
    free(tn); free(tm);
}

void orc_cheb_basis(int64_t m, int32_t n, const double *A, int64_t lda, const double *R, int64_t ldr,
                    const double *r0, int32_t s, double lo, double hi, double *U, double *W)
{
    orc_dense D = {m, n, A, lda};
    orc_op op = {orc_dense_av, orc_dense_atv, &D};
    orc_cheb_basis_op(m, n, &op, R, ldr, r0, s, lo, hi, U, W);
}

/* Solve G c = g (s x s symmetric, column-major) by Cholesky.  A pivot at or
 * below 1e-12 times its diagonal entry (the basis has become numerically
 * dependent: the Krylov space is exhausted or the basis ill-conditioned)
 * stops the factorisation; the system is then solved on the leading k steps
 * and c_k .. c_{s-1} = 0.  Returns k. */
static int32_t orc_gram_solve(int32_t s, const double *G, const double *g, double *c)
{
    double *L = (double *)calloc((size_t)s * (size_t)s, sizeof(double));
    double *y = (double *)malloc(sizeof(double) * (size_t)s);
    int32_t k = 0;
    for (int32_t j = 0; j < s; ++j) {
        double dj = G[j + (int64_t)j * s];
        for (int32_t i = 0; i < j; ++i)
            dj -= L[j + (int64_t)i * s] * L[j + (int64_t)i * s];
        if (!(dj > 1e-12 * G[j + (int64_t)j * s]))
            break;
        const double ljj = sqrt(dj);
        L[j + (int64_t)j * s] = ljj;
        for (int32_t r = j + 1; r < s; ++r) {
            double v = G[r + (int64_t)j * s];
            for (int32_t i = 0; i < j; ++i)
                v -= L[r + (int64_t)i * s] * L[j + (int64_t)i * s];
            L[r + (int64_t)j * s] = v / ljj;
        }
        k = j + 1;
    }
    for (int32_t j = 0; j < s; ++j)
        c[j] = 0.0;
    for (int32_t j = 0; j < k; ++j) { /* L y = g */
        double v = g[j];
        for (int32_t i = 0; i < j; ++i)
            v -= L[j + (int64_t)i * s] * y[i];
        y[j] = v / L[j + (int64_t)j * s];
    }
    for (int32_t j = k - 1; j >= 0; --j) { /* L^T c = y */
        double v = y[j];
        for (int32_t i = j + 1; i < k; ++i)
            v -= L[i + (int64_t)j * s] * c[i];
        c[j] = v / L[j + (int64_t)j * s];
    }
    free(L); free(y);
    return k;
}

/* The s-step method from x0.  Each block, from the current x:
 *   r = b - A x (the data-space residual),  r0 = M^T A^T r,
 *   stopping test (as the momentum method's, after at least one block):
 *     ||r|| = 0, ||r0|| <= tol ||r|| or ||r|| <= tol ||b||;
 *   the Chebyshev basis u_0 .. u_{s-1} of K_s(Z, r0) and W = Z U;
 *   G = U^T Z U (from U^T W, symmetrised) and g = U^T r0;
 *   G c = g;  x <- x + M U c.
 * With Q = M U this is x + Q (Q^T A^T A Q)^-1 Q^T A^T r, the closed form of
 * the CG iterate over x + M K_s(Z, r0): the minimiser of ||A (x_* - .)|| over
 * that space, i.e. s CG (LSQR) steps from x in exact arithmetic.  Blocks run
 * while fewer than maxiter steps have been made (s per block), so at most
 * ceil(maxiter / s) blocks.  info: iters = steps made, resid_est = ||r||,
 * normar_est = ||r0|| at the last test.  history (nullable, one row of n
 * per block after the first x) receives x after each block. */
static void orc_sstep_op(int64_t m, int32_t n, const orc_op *op, const double *b, const double *R, int64_t ldr,
                         const double *x0, int32_t s, double lo, double hi, double tol, int32_t maxiter, double *x,
                         double *history, orc_lsqr_info *info)
{
    double *r = (double *)malloc(sizeof(double) * (size_t)m);
    double *t1 = (double *)malloc(sizeof(double) * (size_t)n);
    double *r0 = (double *)malloc(sizeof(double) * (size_t)n);
    double *U = (double *)malloc(sizeof(double) * (size_t)n * (size_t)s);
    double *W = (double *)malloc(sizeof(double) * (size_t)n * (size_t)s);
    double *G = (double *)malloc(sizeof(double) * (size_t)s * (size_t)s);
    double *g = (double *)malloc(sizeof(double) * (size_t)s);
    double *c = (double *)malloc(sizeof(double) * (size_t)s);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);

    memcpy(x, x0, sizeof(double) * (size_t)n);
    info->iters = 0;
    info->converged = 0;
    const double normb = orc_nrm2(m, b);
    int32_t blocks = 0;
    for (;;) {
        op->av(op->ctx, x, r);
        for (int64_t i = 0; i < m; ++i)
            r[i] = b[i] - r[i];
        const double rn = orc_nrm2(m, r);
        op->atv(op->ctx, r, t1);
        orc_forwardsub_t(R, ldr, n, t1, r0);
        const double fn = orc_nrm2(n, r0);
        info->resid_est = rn;
        info->normar_est = fn;
        if (info->iters >= 1 && (rn == 0.0 || fn <= tol * rn || rn <= tol * normb)) {
            info->converged = 1;
            break;
        }
        if (info->iters >= maxiter)
            break;
        orc_cheb_basis_op(m, n, op, R, ldr, r0, s, lo, hi, U, W);
        for (int32_t j = 0; j < s; ++j) {
            for (int32_t k = 0; k <= j; ++k) {
                double a = 0.0, bb = 0.0;
                for (int32_t i = 0; i < n; ++i) {
                    a += U[i + (int64_t)j * n] * W[i + (int64_t)k * n];
                    bb += U[i + (int64_t)k * n] * W[i + (int64_t)j * n];
                }
                G[j + (int64_t)k * s] = G[k + (int64_t)j * s] = 0.5 * (a + bb);
            }
            double a = 0.0;
            for (int32_t i = 0; i < n; ++i)
                a += U[i + (int64_t)j * n] * r0[i];
            g[j] = a;
        }
        orc_gram_solve(s, G, g, c);
        for (int32_t i = 0; i < n; ++i) {
            double a = 0.0;
            for (int32_t j = 0; j < s; ++j)
                a += U[i + (int64_t)j * n] * c[j];
            y[i] = a;
        }
        orc_backsub(R, ldr, n, y, t1); /* M U c */
        for (int32_t i = 0; i < n; ++i)
            x[i] += t1[i];
        info->iters += s;
        if (history)
            memcpy(history + (int64_t)blocks * n, x, sizeof(double) * (size_t)n);
        blocks += 1;
    }
    free(r); free(t1); free(r0); free(U); free(W); free(G); free(g); free(c); free(y);
}

void orc_sstep(int64_t m, int32_t n, const double *A, int64_t lda, const double *b, const double *R, int64_t ldr,
               const double *x0, int32_t s, double lo, double hi, double tol, int32_t maxiter, double *x,
               double *history, orc_lsqr_info *info)
{
    orc_dense D = {m, n, A, lda};
    orc_op op = {orc_dense_av, orc_dense_atv, &D};
    orc_sstep_op(m, n, &op, b, R, ldr, x0, s, lo, hi, tol, maxiter, x, history, info);
}

/* The Chebyshev interval for a distortion estimate eta in (0, 1): Z's
 * eigenvalues are the squared singular values of A M, which a subspace
 * embedding of distortion eta puts in [(1 - eta)^2, (1 + eta)^2]. */
void orc_sstep_interval(double eta, double *lo, double *hi)
{
    *lo = (1.0 - eta) * (1.0 - eta);
    *hi = (1.0 + eta) * (1.0 + eta);
}

/* ------------------------------------------------------------------------ */
/* Alg. 1 end to end.                                                         */
/* ------------------------------------------------------------------------ */
typedef struct orc_solve_info {
    int32_t status;    /* 0 ok, 3 rank deficient, 4 not converged, 1 invalid */
    int32_t iters;
    double resid_est;
    double normar_est;
    double t_generate, t_apply, t_qr, t_iterate; /* seconds */
} orc_solve_info;

static double orc_now(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

/* Rank test (the paper is silent; reading): R is declared rank deficient when
 * min_k |R_kk| <= d * 2^-53 * max_k |R_kk|. */
int orc_rank_deficient(const double *R, int64_t ldr, int32_t n, int32_t d)
{
    double mx = 0.0, mn = INFINITY;
    for (int32_t k = 0; k < n; ++k) {
        double a = fabs(R[k + (int64_t)k * ldr]);
        if (a > mx) mx = a;
        if (a < mn) mn = a;
    }
    return !(mn > (double)d * ldexp(1.0, -53) * mx);
}

/* Sample S (key (seed, stream)), form Y = S[A b], QR of Y,
 * x0 = R^-1 (Q^T S b)[0:n], LSQR.
 * Y_out (nullable, d x (n+1) column-major, ld d) receives the factored Y
 * (R in the upper triangle).  x receives the solution. */
/* The steps of Alg. 1 after the sketch: QR of Y, rank test, x0, then the
 * iterative method: LSQR (method 0), heavy-ball momentum with step mp[0] and
 * momentum mp[1] (method 1), or the s-step form with s = mp[0] and the
 * Chebyshev interval [mp[1], mp[2]] (method 2).  Shared by the dense and the
 * CSR solve. */
static void orc_solve_finish(int64_t m, int32_t n, const orc_op *op, const double *b, int32_t d, double *Y,
                             double *tau, double tol, int32_t maxiter, int32_t method, const double *mp, double *x,
                             double *x0_out, orc_solve_info *info, double t2)
{
    int32_t nc = n + 1;
    double *x0 = (double *)malloc(sizeof(double) * (size_t)n);
    orc_householder_qr(Y, d, d, nc, tau);
    double t3 = orc_now();
    info->t_qr = t3 - t2;
    if (orc_rank_deficient(Y, d, n, d)) {
        info->status = 3;
    } else {
        /* x0 = R^-1 z with z = (Q^T S b)[0:n] = column n of the factored Y */
        orc_backsub(Y, d, n, Y + (int64_t)n * d, x0);
        if (x0_out)
            memcpy(x0_out, x0, sizeof(double) * (size_t)n);
        orc_lsqr_info li;
        if (method == 1) /* heavy-ball momentum (App. D.3) */
            orc_hbm_op(m, n, op, b, Y, d, x0, mp[0], mp[1], tol, maxiter, x, NULL, &li);
        else if (method == 2) /* s-step form (App. D.4.2) */
            orc_sstep_op(m, n, op, b, Y, d, x0, (int32_t)mp[0], mp[1], mp[2], tol, maxiter, x, NULL, &li);
        else
            orc_lsqr_op(m, n, op, b, Y, d, x0, tol, maxiter, x, NULL, &li);
        info->iters = li.iters;
        info->resid_est = li.resid_est;
        info->normar_est = li.normar_est;
        info->status = li.converged ? 0 : 4;
    }
    info->t_iterate = orc_now() - t3;
    free(x0);
}

/* Sample S (key (seed, stream)), form Y = S[A b], QR of Y,
 * x0 = R^-1 (Q^T S b)[0:n], LSQR.
 * Y_out (nullable, d x (n+1) column-major, ld d) receives the factored Y
 * (R in the upper triangle).  x receives the solution. */
void orc_solve(int64_t m, int32_t n, const double *A, int64_t lda, const double *b,
               int32_t d, int32_t zeta, uint64_t seed, uint64_t stream, double tol, int32_t maxiter,
               double *x, double *x0_out, double *Y_out, orc_solve_info *info)
{
    memset(info, 0, sizeof(*info));
    if (zeta < 1 || zeta > ORC_MAX_ZETA || d < zeta || d < n + 1 || m < 1 || n < 1) {
        info->status = 1;
        return;
    }
    int32_t nc = n + 1;
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)m * (size_t)zeta);
    uint64_t *sign = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)m);
    double *Y = (double *)malloc(sizeof(double) * (size_t)d * (size_t)nc);
    double *tau = (double *)malloc(sizeof(double) * (size_t)nc);

    double t0 = orc_now();
    orc_sketch(seed, stream, m, d, zeta, idx, sign, NULL);
    double t1 = orc_now();
    orc_apply_sparse(m, d, zeta, idx, sign, A, lda, b, n, 1.0 / sqrt((double)zeta), Y, d, NULL, 0);
    double t2 = orc_now();
    info->t_generate = t1 - t0;
    info->t_apply = t2 - t1;
    orc_dense D = {m, n, A, lda};
    orc_op op = {orc_dense_av, orc_dense_atv, &D};
    orc_solve_finish(m, n, &op, b, d, Y, tau, tol, maxiter, 0, NULL, x, x0_out, info, t2);
    if (Y_out)
        memcpy(Y_out, Y, sizeof(double) * (size_t)d * (size_t)nc);
    free(idx); free(sign); free(Y); free(tau);
}

/* Alg. 1 with heavy-ball momentum (App. D.3) in place of LSQR: the same
 * sketch, QR and x0, then orc_hbm_op with step alpha and momentum beta. */
void orc_solve_hbm(int64_t m, int32_t n, const double *A, int64_t lda, const double *b,
                   int32_t d, int32_t zeta, uint64_t seed, uint64_t stream, double tol, int32_t maxiter,
                   double alpha, double beta, double *x, double *x0_out, orc_solve_info *info)
{
    memset(info, 0, sizeof(*info));
    if (zeta < 1 || zeta > ORC_MAX_ZETA || d < zeta || d < n + 1 || m < 1 || n < 1) {
        info->status = 1;
        return;
    }
    int32_t nc = n + 1;
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)m * (size_t)zeta);
    uint64_t *sign = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)m);
    double *Y = (double *)malloc(sizeof(double) * (size_t)d * (size_t)nc);
    double *tau = (double *)malloc(sizeof(double) * (size_t)nc);
    double hb[2] = {alpha, beta};

    double t0 = orc_now();
    orc_sketch(seed, stream, m, d, zeta, idx, sign, NULL);
    double t1 = orc_now();
    orc_apply_sparse(m, d, zeta, idx, sign, A, lda, b, n, 1.0 / sqrt((double)zeta), Y, d, NULL, 0);
    double t2 = orc_now();
    info->t_generate = t1 - t0;
    info->t_apply = t2 - t1;
    orc_dense D = {m, n, A, lda};
    orc_op op = {orc_dense_av, orc_dense_atv, &D};
    orc_solve_finish(m, n, &op, b, d, Y, tau, tol, maxiter, 1, hb, x, x0_out, info, t2);
    free(idx); free(sign); free(Y); free(tau);
}

/* Alg. 1 with the s-step form (App. D.4.2) in place of LSQR: the same
 * sketch, QR and x0, then orc_sstep_op with s steps a block and the
 * Chebyshev interval [lo, hi]. */
void orc_solve_sstep(int64_t m, int32_t n, const double *A, int64_t lda, const double *b,
                     int32_t d, int32_t zeta, uint64_t seed, uint64_t stream, double tol, int32_t maxiter,
                     int32_t s, double lo, double hi, double *x, double *x0_out, orc_solve_info *info)
{
    memset(info, 0, sizeof(*info));
    if (zeta < 1 || zeta > ORC_MAX_ZETA || d < zeta || d < n + 1 || m < 1 || n < 1 || s < 1 || !(hi > lo)) {
        info->status = 1;
        return;
    }
    int32_t nc = n + 1;
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)m * (size_t)zeta);
    uint64_t *sign = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)m);
    double *Y = (double *)malloc(sizeof(double) * (size_t)d * (size_t)nc);
    double *tau = (double *)malloc(sizeof(double) * (size_t)nc);
    double mp[3] = {(double)s, lo, hi};

    double t0 = orc_now();
    orc_sketch(seed, stream, m, d, zeta, idx, sign, NULL);
    double t1 = orc_now();
    orc_apply_sparse(m, d, zeta, idx, sign, A, lda, b, n, 1.0 / sqrt((double)zeta), Y, d, NULL, 0);
    double t2 = orc_now();
    info->t_generate = t1 - t0;
    info->t_apply = t2 - t1;
    orc_dense D = {m, n, A, lda};
    orc_op op = {orc_dense_av, orc_dense_atv, &D};
    orc_solve_finish(m, n, &op, b, d, Y, tau, tol, maxiter, 2, mp, x, x0_out, info, t2);
    free(idx); free(sign); free(Y); free(tau);
}

/* Alg. 1 with A in CSR form: the same steps, the sketch applied to the
 * stored entries (orc_apply_csr) and the LSQR products on the CSR matrix. */
void orc_solve_csr(int64_t m, int32_t n, const int64_t *indptr, const int32_t *indices, const double *values,
                   const double *b, int32_t d, int32_t zeta, uint64_t seed, uint64_t stream, double tol,
                   int32_t maxiter, double *x, double *x0_out, double *Y_out, orc_solve_info *info)
{
    memset(info, 0, sizeof(*info));
    if (zeta < 1 || zeta > ORC_MAX_ZETA || d < zeta || d < n + 1 || m < 1 || n < 1) {
        info->status = 1;
        return;
    }
    int32_t nc = n + 1;
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)m * (size_t)zeta);
    uint64_t *sign = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)m);
    double *Y = (double *)malloc(sizeof(double) * (size_t)d * (size_t)nc);
    double *tau = (double *)malloc(sizeof(double) * (size_t)nc);

    double t0 = orc_now();
    orc_sketch(seed, stream, m, d, zeta, idx, sign, NULL);
    double t1 = orc_now();
    orc_apply_csr(m, d, zeta, idx, sign, indptr, indices, values, b, n, 1.0 / sqrt((double)zeta), Y, d);
    double t2 = orc_now();
    info->t_generate = t1 - t0;
    info->t_apply = t2 - t1;
    orc_csr C = {m, n, indptr, indices, values};
    orc_op op = {orc_csr_av, orc_csr_atv, &C};
    orc_solve_finish(m, n, &op, b, d, Y, tau, tol, maxiter, 0, NULL, x, x0_out, info, t2);
    if (Y_out)
        memcpy(Y_out, Y, sizeof(double) * (size_t)d * (size_t)nc);
    free(idx); free(sign); free(Y); free(tau);
}

/* Direct solve of min ||b - A x|| by Householder QR of [A b] (m x (n+1)),
 * then back substitution: the textbook method of the paper's introduction,
 * used as a reference on tiny inputs.  A is row-major; it is copied. */
void orc_direct_solve(int64_t m, int32_t n, const double *A, int64_t lda, const double *b, double *x)
{
    int32_t nc = n + 1;
    double *W = (double *)malloc(sizeof(double) * (size_t)m * (size_t)nc);
    double *tau = (double *)malloc(sizeof(double) * (size_t)nc);
    for (int64_t i = 0; i < m; ++i) {
        for (int32_t c = 0; c < n; ++c)
            W[i + (int64_t)c * m] = A[i * lda + c];
        W[i + (int64_t)n * m] = b[i];
    }
    orc_householder_qr(W, m, (int32_t)m, nc, tau);
    orc_backsub(W, m, n, W + (int64_t)n * m, x);
    free(W);
    free(tau);
}

/* ------------------------------------------------------------------------
 * Embedding dimension (Sec. 4.3).
 *
 * orc_lambert_w0: the principal branch W(z) for z >= 0, the w >= 0 with
 * w e^w = z, found by bisection (w e^w is increasing for w >= 0; the bracket
 * [0, max(1, ln(1 + z))] holds the root because w e^w >= z at w = ln(1 + z)
 * when z >= e, and at w = 1 when z < e).  Slow and plain on purpose.
 */
double orc_lambert_w0(double z)
{
    if (!(z >= 0.0)) return NAN;
    double lo = 0.0, hi = log1p(z);
    if (hi < 1.0) hi = 1.0;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid * exp(mid) < z) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* Eq. (4.2): d = n exp(W(-m log(eps) / n^2)), the d at which the iteration
 * cost (log eps / log(n/d)) m n equals the QR cost d n^2.  cost_ratio scales
 * the iteration side (time per unit of m n over time per unit of d n^2); the
 * paper's form is cost_ratio = 1.  Returns the real d, before any rounding. */
double orc_embedding_dim(int64_t m, int32_t n, double eps, double cost_ratio)
{
    double z = cost_ratio * (-(double)m * log(eps)) / ((double)n * (double)n);
    return (double)n * exp(orc_lambert_w0(z));
}

/* Eq. (4.1): after t iterations the error is about (n/d)^(t/2); the t at
 * which that reaches eps, as a real number. */
double orc_iteration_estimate(int32_t n, int32_t d, double eps)
{
    return 2.0 * log(eps) / log((double)n / (double)d);
}
