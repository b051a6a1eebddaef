/*
 * uvadmm_oracle.c -- plain FP64 CPU oracle of the UV-decomposition ADMM
 * (Adil, Madani, Tavakkol, Davoudi, "A First-Order Numerical Algorithm without
 * Matrix Operations", Section IV and Algorithm 1).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it, to check the HIP solver against an independent,
 * obviously-correct implementation.  It shares no code, header, table or
 * helper with the HIP library.
 *
 * What it computes.  Problem (Section II, eq. prob_primal):
 *     minimize c'x  subject to  A x = b,  x in K = K_{n1} x ... x K_{nk}
 * with K a product of Lorentz cones; a cone of size 1 is the half line R_+,
 * so the nonnegative orthant is (K_1)^n.  The oracle keeps the paper's own
 * variables of the reformulated problem (eq. prob_reform): x, z, delta in R^n,
 * y, gamma in R^o (o = number of stored nonzeros) and lambda in R^m, and
 * applies U, U', V, V' as explicit sums over the nonzero index k, exactly as
 * the UV decomposition (eqs. UU, VV) defines them:
 *     U = sum_k a_k e_{i_k} edot_k',      V = sum_k eddot_{j_k} edot_k'
 * (the printed eq. VV has its two factors in the wrong order for an n x o
 * matrix; Example 1 of Section IV fixes the n x o reading used here).
 * The nonzeros are numbered in CSR (row-major) order; Section IV allows any
 * order.
 *
 * One iteration is Algorithm 1's repeat block, in the paper's order:
 *   x      <- F_V ( V(y + gamma/mu) + z + delta/mu - c/mu )          (Block 1, eq. vvt)
 *   y      <- (I - U' F_U U) ( U'(b - lambda/mu) + V'x - gamma/mu )   (Block 2, y-step with
 *                                                                     the matrix inversion lemma)
 *   z      <- proj_K( x - delta/mu )                                  (Block 2, z-step, eq. proj)
 *   lambda <- lambda + mu (U y - b)                                   (dual update)
 *   gamma  <- gamma + mu (y - V'x)                                    (dual update)
 *   delta  <- delta + mu (z - x)                                      (dual update)
 * with F_U = (I + U U')^{-1}, F_V = (I + V V')^{-1}, both diagonal (the set-up of
 * Algorithm 1, eqs. UU and VV).
 *
 * Residuals (stopping test of Section V-B, SCS form) are evaluated at z and
 * lambda with fresh sparse products; two readings of the printed test are
 * taken (see the function residuals()): the dual residual subtracts delta
 * (x is cone-constrained, not free) and the gap takes an absolute value.
 *
 * Parallelism: OpenMP over rows, columns, nonzeros or cones.  Every reduction
 * is a serial loop over a per-element array, so results do not depend on the
 * thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Loops over fewer than this many rows, columns or nonzeros run on one
 * thread (a parallel region costs more than the loop itself below it). */
#define ORC_PAR_MIN 50000

typedef struct {
    int32_t m, n;
    int64_t o;            /* number of stored nonzeros */
    /* nonzero k: row rk[k], column ck[k], value ak[k]; numbered in CSR order */
    int32_t *rk, *ck;
    double *ak;
    int64_t *row_ptr;     /* row i owns k in [row_ptr[i], row_ptr[i+1]) */
    int64_t *col_ptr;     /* column j owns kcol[col_ptr[j] .. col_ptr[j+1]) */
    int64_t *kcol;
    double *b, *c;
    int32_t n_orth, n_soc;
    int32_t *soc_size;
    int64_t *soc_off;     /* first index of each second-order cone */
    double mu;
    double *FU, *FV;      /* diagonals of (I+UU')^{-1} and (I+VV')^{-1} */
    /* Algorithm 1 state */
    double *x, *z, *delta, *lambda;
    double *y, *gamma;
    /* work */
    double *t, *s, *wrk_n, *wrk_m;
    int64_t iter;
} orc_t;

static void *xcalloc(size_t cnt, size_t sz)
{
    if (cnt == 0) cnt = 1;
    return calloc(cnt, sz);
}

void orc_destroy(orc_t *h)
{
    if (!h) return;
    free(h->rk); free(h->ck); free(h->ak); free(h->row_ptr); free(h->col_ptr);
    free(h->kcol); free(h->b); free(h->c); free(h->soc_size); free(h->soc_off);
    free(h->FU); free(h->FV); free(h->x); free(h->z); free(h->delta);
    free(h->lambda); free(h->y); free(h->gamma); free(h->t); free(h->s);
    free(h->wrk_n); free(h->wrk_m);
    free(h);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Returns NULL on any malformed input (the oracle is a checker, not a
 * validator: callers pass well-formed CSR). */
orc_t *orc_create(int32_t m, int32_t n, int64_t nnz, const int64_t *row_ptr,
                  const int32_t *col_idx, const double *val, const double *b,
                  const double *c, int32_t n_orth, int32_t n_soc,
                  const int32_t *soc_sizes, double mu)
{
    if (m < 0 || n < 0 || nnz < 0 || !(mu > 0.0)) return NULL;
    if (row_ptr[0] != 0 || row_ptr[m] != nnz) return NULL;
    int64_t ncone_cols = n_orth;
    for (int32_t q = 0; q < n_soc; ++q) {
        if (soc_sizes[q] < 1) return NULL;
        ncone_cols += soc_sizes[q];
    }
    if (ncone_cols != n) return NULL;

    orc_t *h = (orc_t *)calloc(1, sizeof(orc_t));
    if (!h) return NULL;
    h->m = m; h->n = n; h->o = nnz; h->mu = mu;
    h->n_orth = n_orth; h->n_soc = n_soc;
    h->rk = (int32_t *)xcalloc((size_t)nnz, sizeof(int32_t));
    h->ck = (int32_t *)xcalloc((size_t)nnz, sizeof(int32_t));
    h->ak = (double *)xcalloc((size_t)nnz, sizeof(double));
    h->row_ptr = (int64_t *)xcalloc((size_t)m + 1, sizeof(int64_t));
    h->col_ptr = (int64_t *)xcalloc((size_t)n + 1, sizeof(int64_t));
    h->kcol = (int64_t *)xcalloc((size_t)nnz, sizeof(int64_t));
    h->b = (double *)xcalloc((size_t)m, sizeof(double));
    h->c = (double *)xcalloc((size_t)n, sizeof(double));
    h->soc_size = (int32_t *)xcalloc((size_t)n_soc, sizeof(int32_t));
    h->soc_off = (int64_t *)xcalloc((size_t)n_soc, sizeof(int64_t));
    h->FU = (double *)xcalloc((size_t)m, sizeof(double));
    h->FV = (double *)xcalloc((size_t)n, sizeof(double));
    h->x = (double *)xcalloc((size_t)n, sizeof(double));
    h->z = (double *)xcalloc((size_t)n, sizeof(double));
    h->delta = (double *)xcalloc((size_t)n, sizeof(double));
    h->lambda = (double *)xcalloc((size_t)m, sizeof(double));
    h->y = (double *)xcalloc((size_t)nnz, sizeof(double));
    h->gamma = (double *)xcalloc((size_t)nnz, sizeof(double));
    h->t = (double *)xcalloc((size_t)nnz, sizeof(double));
    h->s = (double *)xcalloc((size_t)m, sizeof(double));
    h->wrk_n = (double *)xcalloc((size_t)n, sizeof(double));
    h->wrk_m = (double *)xcalloc((size_t)m, sizeof(double));
    if (!h->rk || !h->ck || !h->ak || !h->row_ptr || !h->col_ptr || !h->kcol ||
        !h->b || !h->c || !h->soc_size || !h->soc_off || !h->FU || !h->FV ||
        !h->x || !h->z || !h->delta || !h->lambda || !h->y || !h->gamma ||
        !h->t || !h->s || !h->wrk_n || !h->wrk_m) {
        orc_destroy(h);
        return NULL;
    }

    /* Nonzeros in CSR order: k runs over rows, then over the row's entries. */
    for (int32_t i = 0; i <= m; ++i) h->row_ptr[i] = row_ptr[i];
    for (int32_t i = 0; i < m; ++i) {
        if (row_ptr[i + 1] < row_ptr[i]) { orc_destroy(h); return NULL; }
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            if (col_idx[k] < 0 || col_idx[k] >= n) { orc_destroy(h); return NULL; }
            h->rk[k] = i;
            h->ck[k] = col_idx[k];
            h->ak[k] = val[k];
        }
    }
    memcpy(h->b, b, sizeof(double) * (size_t)m);
    memcpy(h->c, c, sizeof(double) * (size_t)n);

    /* The nonzero indices of each column (a counting sort by column, stable
     * in k), so that products with V run as sums over a column's entries. */
    for (int64_t k = 0; k < nnz; ++k) h->col_ptr[h->ck[k] + 1]++;
    for (int32_t j = 0; j < n; ++j) h->col_ptr[j + 1] += h->col_ptr[j];
    {
        int64_t *fill = (int64_t *)xcalloc((size_t)n, sizeof(int64_t));
        if (!fill) { orc_destroy(h); return NULL; }
        for (int32_t j = 0; j < n; ++j) fill[j] = h->col_ptr[j];
        for (int64_t k = 0; k < nnz; ++k) h->kcol[fill[h->ck[k]]++] = k;
        free(fill);
    }

    int64_t off = n_orth;
    for (int32_t q = 0; q < n_soc; ++q) {
        h->soc_size[q] = soc_sizes[q];
        h->soc_off[q] = off;
        off += soc_sizes[q];
    }

    /* The set-up of Algorithm 1 (eqs. UU, VV).  U U' is diagonal with entry i equal to the sum
     * of squares of row i's nonzeros (each column of U has a single nonzero
     * a_k in row i_k); V V' is diagonal with entry j equal to the number of
     * nonzeros in column j (each column of V is a single 1 in row j_k). */
    #pragma omp parallel for schedule(static) if (m >= ORC_PAR_MIN)
    for (int32_t i = 0; i < m; ++i) {
        double d = 0.0;
        for (int64_t k = h->row_ptr[i]; k < h->row_ptr[i + 1]; ++k) d += h->ak[k] * h->ak[k];
        h->FU[i] = 1.0 / (1.0 + d);
    }
    #pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
    for (int32_t j = 0; j < n; ++j) {
        double d = 0.0;
        for (int64_t p = h->col_ptr[j]; p < h->col_ptr[j + 1]; ++p) d += 1.0;
        h->FV[j] = 1.0 / (1.0 + d);
    }
    h->iter = 0;
    return h;
}

void orc_diagonals(const orc_t *h, double *FU, double *FV)
{
    if (FU) memcpy(FU, h->FU, sizeof(double) * (size_t)h->m);
    if (FV) memcpy(FV, h->FV, sizeof(double) * (size_t)h->n);
}

/* ---- projection onto K (Section IV, Block 2, eq. proj) ------------------ */

/* Projection of w (length nq) onto the Lorentz cone {w_1 >= ||w_{2:}||_2},
 * taking the three cases in the order printed with eq. proj. */
static void proj_lorentz(const double *w, double *out, int32_t nq)
{
    double a2 = 0.0;
    for (int32_t r = 1; r < nq; ++r) a2 += w[r] * w[r];
    double alpha = sqrt(a2);
    double w1 = w[0];
    if (alpha <= -w1) {
        for (int32_t r = 0; r < nq; ++r) out[r] = 0.0;
    } else if (alpha <= w1) {
        for (int32_t r = 0; r < nq; ++r) out[r] = w[r];
    } else {
        out[0] = w1 / 2.0 + alpha / 2.0;
        for (int32_t r = 1; r < nq; ++r) out[r] = w[r] / 2.0 + w1 * w[r] / (2.0 * alpha);
    }
}

/* The orthant coordinates are cones of size 1: there the case test reduces
 * to the sign of w_1 and the projection to max(w_1, 0). */
static void proj_K(int32_t n_orth, int32_t n_soc, const int32_t *soc_size,
                   const int64_t *soc_off, const double *w, double *out)
{
    #pragma omp parallel for schedule(static) if (n_orth >= ORC_PAR_MIN)
    for (int32_t j = 0; j < n_orth; ++j) proj_lorentz(w + j, out + j, 1);
    #pragma omp parallel for schedule(dynamic, 64) if (n_soc >= ORC_PAR_MIN / 16)
    for (int32_t q = 0; q < n_soc; ++q)
        proj_lorentz(w + soc_off[q], out + soc_off[q], soc_size[q]);
}

/* Stand-alone projection (w and out of length n_orth + sum(soc_sizes)). */
void orc_project(int32_t n_orth, int32_t n_soc, const int32_t *soc_sizes,
                 const double *w, double *out)
{
    int64_t *off = (int64_t *)xcalloc((size_t)n_soc, sizeof(int64_t));
    int64_t o = n_orth;
    for (int32_t q = 0; q < n_soc; ++q) { off[q] = o; o += soc_sizes[q]; }
    proj_K(n_orth, n_soc, soc_sizes, off, w, out);
    free(off);
}

/* ---- Algorithm 1 state ------------------------------------------------- */

/* Sets the six vectors Algorithm 1 requires; NULL means zero. */
void orc_set_state(orc_t *h, const double *x, const double *z, const double *delta,
                   const double *y, const double *gamma, const double *lambda)
{
    size_t n = (size_t)h->n, m = (size_t)h->m, o = (size_t)h->o;
    if (x) memcpy(h->x, x, n * 8); else memset(h->x, 0, n * 8);
    if (z) memcpy(h->z, z, n * 8); else memset(h->z, 0, n * 8);
    if (delta) memcpy(h->delta, delta, n * 8); else memset(h->delta, 0, n * 8);
    if (y) memcpy(h->y, y, o * 8); else memset(h->y, 0, o * 8);
    if (gamma) memcpy(h->gamma, gamma, o * 8); else memset(h->gamma, 0, o * 8);
    if (lambda) memcpy(h->lambda, lambda, m * 8); else memset(h->lambda, 0, m * 8);
    h->iter = 0;
}

/* Start from problem-space vectors: y = V'x and gamma = -U'lambda, the values
 * those constraints and the y-step optimality condition take at any point of
 * the reformulation that corresponds to (x, lambda).  NULL means zero. */
void orc_set_start(orc_t *h, const double *x, const double *z, const double *delta,
                   const double *lambda)
{
    orc_set_state(h, x, z, delta, NULL, NULL, lambda);
    #pragma omp parallel for schedule(static) if (h->o >= ORC_PAR_MIN)
    for (int64_t k = 0; k < h->o; ++k) {
        h->y[k] = h->x[h->ck[k]];                    /* (V'x)_k = x_{j_k} */
        h->gamma[k] = -h->ak[k] * h->lambda[h->rk[k]]; /* (U'lambda)_k = a_k lambda_{i_k} */
    }
}

void orc_get_state(const orc_t *h, double *x, double *z, double *delta,
                   double *y, double *gamma, double *lambda)
{
    size_t n = (size_t)h->n, m = (size_t)h->m, o = (size_t)h->o;
    if (x) memcpy(x, h->x, n * 8);
    if (z) memcpy(z, h->z, n * 8);
    if (delta) memcpy(delta, h->delta, n * 8);
    if (y) memcpy(y, h->y, o * 8);
    if (gamma) memcpy(gamma, h->gamma, o * 8);
    if (lambda) memcpy(lambda, h->lambda, m * 8);
}

int64_t orc_iteration(const orc_t *h) { return h->iter; }

static void y_step(orc_t *h);

/* The full state at the end of an iteration from its problem-space part
 * (x, z, delta, lambda): every iteration leaves gamma = -U'lambda (the
 * y-step's optimality condition combined with the lambda and gamma
 * updates), and y is the y-step's output at this x with that gamma. */
void orc_resume(orc_t *h, const double *x, const double *z, const double *delta,
                const double *lambda)
{
    orc_set_state(h, x, z, delta, NULL, NULL, lambda);
    #pragma omp parallel for schedule(static) if (h->o >= ORC_PAR_MIN)
    for (int64_t k = 0; k < h->o; ++k) h->gamma[k] = -h->ak[k] * h->lambda[h->rk[k]];
    y_step(h);
}

/* Block 2, y-step (matrix inversion lemma) at the current x, lambda, gamma:
 *   t = U'(b - lambda/mu) + V'x - gamma/mu,   t_k = a_k (b - lambda/mu)_{i_k} + x_{j_k} - gamma_k/mu
 *   y = (I - U' F_U U) t = t - U'(F_U (U t)). */
static void y_step(orc_t *h)
{
    const int32_t m = h->m;
    const int64_t o = h->o;
    const double mu = h->mu;
    #pragma omp parallel for schedule(static) if (o >= ORC_PAR_MIN)
    for (int64_t k = 0; k < o; ++k) {
        int32_t i = h->rk[k];
        h->t[k] = h->ak[k] * (h->b[i] - h->lambda[i] / mu) + h->x[h->ck[k]] - h->gamma[k] / mu;
    }
    #pragma omp parallel for schedule(static) if (m >= ORC_PAR_MIN)
    for (int32_t i = 0; i < m; ++i) {
        double ut = 0.0;
        for (int64_t k = h->row_ptr[i]; k < h->row_ptr[i + 1]; ++k) ut += h->ak[k] * h->t[k];
        h->s[i] = h->FU[i] * ut;
    }
    #pragma omp parallel for schedule(static) if (o >= ORC_PAR_MIN)
    for (int64_t k = 0; k < o; ++k) h->y[k] = h->t[k] - h->ak[k] * h->s[h->rk[k]];
}

/* One pass of Algorithm 1's repeat block. */
static void iterate_once(orc_t *h)
{
    const int32_t m = h->m, n = h->n;
    const int64_t o = h->o;
    const double mu = h->mu;

    /* Block 1 (eq. vvt): x = F_V (V(y + gamma/mu) + z + delta/mu - c/mu),
     * (V w)_j = sum over the nonzeros k of column j of w_k. */
    #pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
    for (int32_t j = 0; j < n; ++j) {
        double vy = 0.0;
        for (int64_t p = h->col_ptr[j]; p < h->col_ptr[j + 1]; ++p) {
            int64_t k = h->kcol[p];
            vy += h->y[k] + h->gamma[k] / mu;
        }
        h->x[j] = h->FV[j] * (vy + h->z[j] + h->delta[j] / mu - h->c[j] / mu);
    }

    y_step(h);

    /* Block 2, z-step (eq. proj): z = proj_K(x - delta/mu). */
    #pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
    for (int32_t j = 0; j < n; ++j) h->wrk_n[j] = h->x[j] - h->delta[j] / mu;
    proj_K(h->n_orth, h->n_soc, h->soc_size, h->soc_off, h->wrk_n, h->z);

    /* Multiplier update of the U-constraint: lambda = lambda + mu (U y - b). */
    #pragma omp parallel for schedule(static) if (m >= ORC_PAR_MIN)
    for (int32_t i = 0; i < m; ++i) {
        double uy = 0.0;
        for (int64_t k = h->row_ptr[i]; k < h->row_ptr[i + 1]; ++k) uy += h->ak[k] * h->y[k];
        h->lambda[i] += mu * (uy - h->b[i]);
    }
    /* Multiplier update of the V-constraint: gamma = gamma + mu (y - V'x). */
    #pragma omp parallel for schedule(static) if (o >= ORC_PAR_MIN)
    for (int64_t k = 0; k < o; ++k) h->gamma[k] += mu * (h->y[k] - h->x[h->ck[k]]);
    /* Multiplier update of z = x: delta = delta + mu (z - x). */
    #pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
    for (int32_t j = 0; j < n; ++j) h->delta[j] += mu * (h->z[j] - h->x[j]);

    h->iter++;
}

void orc_iterate(orc_t *h, int64_t k)
{
    for (int64_t it = 0; it < k; ++it) iterate_once(h);
}

static double serial_sum(const double *v, int64_t len)
{
    double s = 0.0;
    for (int64_t i = 0; i < len; ++i) s += v[i];
    return s;
}

/* Residuals of the current state, all FP64 (stopping test of Section V-B,
 * the SCS form, normalised by 1 + ||b||, 1 + ||c|| and the objective sizes):
 *   out[0] r_prim = ||A z - b||_2 / (1 + ||b||_2)
 *   out[1] r_dual = ||A'lambda + c - delta||_2 / (1 + ||c||_2)
 *   out[2] r_gap  = |c'z + b'lambda| / (1 + |c'z| + |b'lambda|)
 *   out[3] kkt    = max(out[0], out[1], out[2])
 *   out[4] primal objective c'z
 *   out[5] dual objective  -b'lambda   (lambda is the multiplier of U y = b,
 *                                       so it enters with the opposite sign)
 *   out[6] ||A x - b||_2   (the printed primal residual, at x)
 *   out[7] ||x - z||_2
 *   out[8] ||A z - b||_inf,  out[9] ||A'lambda + c - delta||_inf,
 *   out[10] max(||A z||_inf, ||b||_inf), out[11] max(||A'lambda||_inf, ||c||_inf)
 *   out[12] c'x   (the objective at x, which the stopping test of the POGS
 *                  comparison, Section V-A2, eq. stopcri, takes in its gap
 *                  |c'x + b'lambda| beside ||A x - b||_2)
 *          (the infinity-norm termination test of Section V-A1, eq.
 *          stopcri_osqp, with the same readings: at z, delta subtracted)
 * Readings: the printed dual residual ||A'lambda + c|| is the one for free x;
 * with x in K the stationarity condition of the Lagrangian (eq. lll) in x is
 * c + A'lambda - delta = 0 with delta in the dual cone, so delta is
 * subtracted.  The printed gap carries no absolute value; the comparisons
 * of Sections V-A and V-A2 take one, and so does this.  The iterate in K is
 * z (x only satisfies it in the limit), hence residuals at z. */
void orc_residuals(orc_t *h, double *out)
{
    const int32_t m = h->m, n = h->n;
    double *rm = h->wrk_m, *rn = h->wrk_n;

    double *azv = (double *)xcalloc((size_t)m, sizeof(double));
    double *atlv = (double *)xcalloc((size_t)n, sizeof(double));
    #pragma omp parallel for schedule(static) if (m >= ORC_PAR_MIN)
    for (int32_t i = 0; i < m; ++i) {
        double az = 0.0;
        for (int64_t k = h->row_ptr[i]; k < h->row_ptr[i + 1]; ++k) az += h->ak[k] * h->z[h->ck[k]];
        rm[i] = (az - h->b[i]) * (az - h->b[i]);
        azv[i] = az;
    }
    double rp2 = serial_sum(rm, m);
    #pragma omp parallel for schedule(static) if (n >= ORC_PAR_MIN)
    for (int32_t j = 0; j < n; ++j) {
        double atl = 0.0;
        for (int64_t p = h->col_ptr[j]; p < h->col_ptr[j + 1]; ++p) {
            int64_t k = h->kcol[p];
            atl += h->ak[k] * h->lambda[h->rk[k]];
        }
        double r = atl + h->c[j] - h->delta[j];
        rn[j] = r * r;
        atlv[j] = atl;
    }
    double rd2 = serial_sum(rn, n);
    double pinf = 0.0, dinf = 0.0, azinf = 0.0, atlinf = 0.0, binf = 0.0, cinf = 0.0;
    for (int32_t i = 0; i < m; ++i) {
        pinf = fmax(pinf, fabs(azv[i] - h->b[i]));
        azinf = fmax(azinf, fabs(azv[i]));
        binf = fmax(binf, fabs(h->b[i]));
    }
    for (int32_t j = 0; j < n; ++j) {
        dinf = fmax(dinf, fabs(atlv[j] + h->c[j] - h->delta[j]));
        atlinf = fmax(atlinf, fabs(atlv[j]));
        cinf = fmax(cinf, fabs(h->c[j]));
    }
    free(azv);
    free(atlv);
    double bb = 0.0, cc = 0.0, cz = 0.0, bl = 0.0, cx = 0.0;
    for (int32_t i = 0; i < m; ++i) { bb += h->b[i] * h->b[i]; bl += h->b[i] * h->lambda[i]; }
    for (int32_t j = 0; j < n; ++j) { cc += h->c[j] * h->c[j]; cz += h->c[j] * h->z[j]; cx += h->c[j] * h->x[j]; }

    #pragma omp parallel for schedule(static) if (m >= ORC_PAR_MIN)
    for (int32_t i = 0; i < m; ++i) {
        double ax = 0.0;
        for (int64_t k = h->row_ptr[i]; k < h->row_ptr[i + 1]; ++k) ax += h->ak[k] * h->x[h->ck[k]];
        rm[i] = (ax - h->b[i]) * (ax - h->b[i]);
    }
    double rpx2 = serial_sum(rm, m);
    double xz2 = 0.0;
    for (int32_t j = 0; j < n; ++j) xz2 += (h->x[j] - h->z[j]) * (h->x[j] - h->z[j]);

    out[0] = sqrt(rp2) / (1.0 + sqrt(bb));
    out[1] = sqrt(rd2) / (1.0 + sqrt(cc));
    out[2] = fabs(cz + bl) / (1.0 + fabs(cz) + fabs(bl));
    out[3] = fmax(out[0], fmax(out[1], out[2]));
    out[4] = cz;
    out[5] = -bl;
    out[6] = sqrt(rpx2);
    out[7] = sqrt(xz2);
    out[8] = pinf;
    out[9] = dinf;
    out[10] = fmax(azinf, binf);
    out[11] = fmax(atlinf, cinf);
    out[12] = cx;
}

/* Runs until kkt <= eps at a check (every check_every iterations) or until
 * max_iter iterations; returns the iteration count at the stop. */
int64_t orc_solve(orc_t *h, double eps, int64_t check_every, int64_t max_iter, double *res_out)
{
    double r[13];
    if (check_every < 1) check_every = 1;
    while (h->iter < max_iter) {
        int64_t k = check_every;
        if (h->iter + k > max_iter) k = max_iter - h->iter;
        orc_iterate(h, k);
        orc_residuals(h, r);
        if (r[3] <= eps) break;
    }
    orc_residuals(h, r);
    if (res_out) memcpy(res_out, r, sizeof(r));
    return h->iter;
}

/* Dense U (m x o) and V (n x o), row-major, for nonzeros given in any order
 * (eqs. UU, VV): U[i_k, k] = a_k and V[j_k, k] = 1.  For small matrices only;
 * used to check the construction against Example 1 of Section IV. */
void orc_uv_dense(int32_t m, int32_t n, int64_t o, const int32_t *rows,
                  const int32_t *cols, const double *vals, double *U, double *V)
{
    memset(U, 0, sizeof(double) * (size_t)m * (size_t)o);
    memset(V, 0, sizeof(double) * (size_t)n * (size_t)o);
    for (int64_t k = 0; k < o; ++k) {
        U[(size_t)rows[k] * (size_t)o + (size_t)k] = vals[k];
        V[(size_t)cols[k] * (size_t)o + (size_t)k] = 1.0;
    }
}
