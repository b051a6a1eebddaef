/*
 * standard_oracle.c -- plain FP64 CPU oracle of the standard two-block ADMM
 * for the conic problem, with the linear system of every iteration solved
 * indirectly by conjugate gradients (the alternative the paper's method is
 * set against: Section II-B, ADMM on the splitting x1 = x2, and Section
 * III-B, indirect methods with a warm-started CG).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the tests and the benchmark's CPU leg use it.  It
 * shares no code, header or helper with the HIP library (nor with the UV
 * oracle next to it).
 *
 * Problem (Section II, eq. prob_primal):
 *     minimize c'x  subject to  A x = b,  x in K,
 * K = R_+^{n_orth} x K_{s_1} x ... (orthant coordinates first, then Lorentz
 * cones, each with its t coordinate first).
 * Splitting (Section II-A): f = indicator of the cone, g = c'x on the affine
 * set {A x = b}; ADMM on x1 = x2 (Section II-B) with the paper's order:
 *   x1     <- prox_f(x2 - lam/mu)        = proj_K(x2 - lam/mu)  (eq. proj per cone)
 *   x2     <- prox_{g/mu}(x1 + lam/mu)   : with w0 = x1 + lam/mu, the block
 *             system eq. lin
 *                 [ I  A' ] [ w  ]   [ w0 - c/mu ]
 *                 [ A  0  ] [ nu ] = [ b         ]
 *             and x2 = w.  Eliminating w = w0 - c/mu - A'nu leaves
 *             (A A') nu = A (w0 - c/mu) - b, solved by textbook conjugate
 *             gradients (Hestenes-Stiefel) started from the previous nu
 *             (the warm start of Section III-B), at most cg_iters steps,
 *             stopping early once ||residual||_2 <= cg_tol (1 + ||b||_2),
 *             or at a breakdown (p'(A A')p not positive, which rounding can
 *             cause once the residual is at the level of rounding).
 *   lam    <- lam + mu (x1 - x2)
 * The paper's printed x1 step uses lam_1 where the update defines lam_12;
 * both are the one multiplier of x1 = x2 (reading).
 *
 * Multipliers of the original problem at the iterate (for the residuals):
 * the x2 problem is min c'w + mu/2 ||w - w0||^2 s.t. A w = b, whose
 * multiplier of A w = b is mu nu: lambda_A = mu nu, in the paper's sign
 * convention (stationarity c + A'lambda_A - delta = 0).  The cone multiplier
 * is delta = lam + mu (x1 - x2) taken at the x1 step with the x2 it used:
 * delta = mu (proj_K(v) - v) with v = x2 - lam/mu, which lies in the dual
 * cone (Moreau).  At a fixed point x1 = x2 and delta = lam.
 *
 * Residuals: the same SCS form as the UV oracle, at z = x1 (in K).
 * Reductions are serial loops, so results do not depend on thread counts.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t m, n;
    int64_t nnz;
    int32_t n_orth, n_soc;
    int32_t *soc_size;
    int64_t *soc_off;     /* first coordinate of each Lorentz cone */
    int64_t *rp;          /* CSR: row i owns [rp[i], rp[i+1]) */
    int32_t *ci;
    double *va;
    double *b, *c;
    double mu, cg_tol, bnorm;
    int32_t cg_iters;
    /* state */
    double *x1, *x2, *lam, *nu, *delta;
    /* work */
    double *v, *g, *r, *p, *q, *tn, *a;
    int64_t iter, cg_steps;
} ors_t;

static void *zalloc(size_t cnt, size_t sz)
{
    return calloc(cnt ? cnt : 1, sz);
}

void ors_destroy(ors_t *h)
{
    if (!h) return;
    free(h->rp); free(h->ci); free(h->va); free(h->b); free(h->c);
    free(h->x1); free(h->x2); free(h->lam); free(h->nu); free(h->delta);
    free(h->v); free(h->g); free(h->r); free(h->p); free(h->q); free(h->tn);
    free(h->soc_size); free(h->soc_off); free(h->a);
    free(h);
}

ors_t *ors_create(int32_t m, int32_t n, int64_t nnz, const int64_t *row_ptr,
                  const int32_t *col_idx, const double *val, const double *b,
                  const double *c, int32_t n_orth, int32_t n_soc, const int32_t *soc_sizes,
                  double mu, int32_t cg_iters, double cg_tol)
{
    if (m < 1 || n < 1 || nnz < 0 || !(mu > 0.0) || cg_iters < 0 || cg_tol < 0.0) return NULL;
    if (row_ptr[0] != 0 || row_ptr[m] != nnz || n_orth < 0 || n_soc < 0) return NULL;
    int64_t tot = n_orth;
    for (int32_t q = 0; q < n_soc; ++q) {
        if (soc_sizes[q] < 1) return NULL;
        tot += soc_sizes[q];
    }
    if (tot != n) return NULL;
    ors_t *h = (ors_t *)calloc(1, sizeof(ors_t));
    if (!h) return NULL;
    h->m = m; h->n = n; h->nnz = nnz; h->mu = mu;
    h->n_orth = n_orth; h->n_soc = n_soc;
    h->soc_size = (int32_t *)zalloc((size_t)n_soc, sizeof(int32_t));
    h->soc_off = (int64_t *)zalloc((size_t)n_soc, sizeof(int64_t));
    h->a = (double *)zalloc((size_t)n, sizeof(double));
    if (!h->soc_size || !h->soc_off || !h->a) {
        ors_destroy(h);
        return NULL;
    }
    for (int32_t q = 0, o = n_orth; q < n_soc; o += soc_sizes[q], ++q) {
        h->soc_size[q] = soc_sizes[q];
        h->soc_off[q] = o;
    }
    h->cg_iters = cg_iters; h->cg_tol = cg_tol;
    h->rp = (int64_t *)zalloc((size_t)m + 1, sizeof(int64_t));
    h->ci = (int32_t *)zalloc((size_t)nnz, sizeof(int32_t));
    h->va = (double *)zalloc((size_t)nnz, sizeof(double));
    h->b = (double *)zalloc((size_t)m, sizeof(double));
    h->c = (double *)zalloc((size_t)n, sizeof(double));
    h->x1 = (double *)zalloc((size_t)n, sizeof(double));
    h->x2 = (double *)zalloc((size_t)n, sizeof(double));
    h->lam = (double *)zalloc((size_t)n, sizeof(double));
    h->delta = (double *)zalloc((size_t)n, sizeof(double));
    h->nu = (double *)zalloc((size_t)m, sizeof(double));
    h->v = (double *)zalloc((size_t)n, sizeof(double));
    h->tn = (double *)zalloc((size_t)n, sizeof(double));
    h->g = (double *)zalloc((size_t)m, sizeof(double));
    h->r = (double *)zalloc((size_t)m, sizeof(double));
    h->p = (double *)zalloc((size_t)m, sizeof(double));
    h->q = (double *)zalloc((size_t)m, sizeof(double));
    if (!h->rp || !h->ci || !h->va || !h->b || !h->c || !h->x1 || !h->x2 || !h->lam ||
        !h->delta || !h->nu || !h->v || !h->tn || !h->g || !h->r || !h->p || !h->q) {
        ors_destroy(h);
        return NULL;
    }
    memcpy(h->rp, row_ptr, sizeof(int64_t) * ((size_t)m + 1));
    memcpy(h->ci, col_idx, sizeof(int32_t) * (size_t)nnz);
    memcpy(h->va, val, sizeof(double) * (size_t)nnz);
    memcpy(h->b, b, sizeof(double) * (size_t)m);
    memcpy(h->c, c, sizeof(double) * (size_t)n);
    double bb = 0.0;
    for (int32_t i = 0; i < m; ++i) bb += b[i] * b[i];
    h->bnorm = sqrt(bb);
    return h;
}

/* out = A w (m-vector) */
static void mul_A(const ors_t *h, const double *w, double *out)
{
    for (int32_t i = 0; i < h->m; ++i) {
        double s = 0.0;
        for (int64_t k = h->rp[i]; k < h->rp[i + 1]; ++k) s += h->va[k] * w[h->ci[k]];
        out[i] = s;
    }
}

/* out = A' y (n-vector), scattered row by row */
static void mul_At(const ors_t *h, const double *y, double *out)
{
    for (int32_t j = 0; j < h->n; ++j) out[j] = 0.0;
    for (int32_t i = 0; i < h->m; ++i)
        for (int64_t k = h->rp[i]; k < h->rp[i + 1]; ++k) out[h->ci[k]] += h->va[k] * y[i];
}

static double dot(const double *a, const double *b, int64_t len)
{
    double s = 0.0;
    for (int64_t i = 0; i < len; ++i) s += a[i] * b[i];
    return s;
}

/* Projection of w (length k) onto the Lorentz cone {w_1 >= ||w_{2..k}||_2}:
 * zero when the tail norm is at most -w_1, w itself when it is at most w_1,
 * else the point ((w_1 + a)/2, (1 + w_1/a)/2 * w_{2..k}) with a the tail
 * norm (eq. proj).  A cone of size 1 is the half line: max(w_1, 0). */
static void lorentz(const double *w, double *out, int32_t k)
{
    double t2 = 0.0;
    for (int32_t i = 1; i < k; ++i) t2 += w[i] * w[i];
    const double a = sqrt(t2), w1 = w[0];
    if (a <= -w1) {
        for (int32_t i = 0; i < k; ++i) out[i] = 0.0;
    } else if (a <= w1) {
        for (int32_t i = 0; i < k; ++i) out[i] = w[i];
    } else {
        const double s = 0.5 * (1.0 + w1 / a);
        out[0] = 0.5 * (w1 + a);
        for (int32_t i = 1; i < k; ++i) out[i] = s * w[i];
    }
}

/* Stand-alone projection onto K = R_+^{n_orth} x K_{sizes[0]} x ... */
void ors_project(int32_t n_orth, int32_t n_soc, const int32_t *sizes, const double *w, double *out)
{
    for (int32_t j = 0; j < n_orth; ++j) lorentz(w + j, out + j, 1);
    int64_t o = n_orth;
    for (int32_t q = 0; q < n_soc; ++q) {
        lorentz(w + o, out + o, sizes[q]);
        o += sizes[q];
    }
}

/* Any pointer may be NULL (zero).  Sets x2, lam and the CG start nu. */
void ors_set_state(ors_t *h, const double *x2, const double *lam, const double *nu)
{
    for (int32_t j = 0; j < h->n; ++j) {
        h->x2[j] = x2 ? x2[j] : 0.0;
        h->lam[j] = lam ? lam[j] : 0.0;
        h->x1[j] = 0.0;
        h->delta[j] = 0.0;
    }
    for (int32_t i = 0; i < h->m; ++i) h->nu[i] = nu ? nu[i] : 0.0;
    h->iter = 0;
    h->cg_steps = 0;
}

void ors_get_state(const ors_t *h, double *x1, double *x2, double *lam, double *nu, double *delta)
{
    const size_t n8 = sizeof(double) * (size_t)h->n, m8 = sizeof(double) * (size_t)h->m;
    if (x1) memcpy(x1, h->x1, n8);
    if (x2) memcpy(x2, h->x2, n8);
    if (lam) memcpy(lam, h->lam, n8);
    if (nu) memcpy(nu, h->nu, m8);
    if (delta) memcpy(delta, h->delta, n8);
}

int64_t ors_iteration(const ors_t *h) { return h->iter; }
int64_t ors_cg_steps(const ors_t *h) { return h->cg_steps; }

static void iterate_once(ors_t *h)
{
    const int32_t m = h->m, n = h->n;
    const double mu = h->mu;
    /* x1 <- proj_K(x2 - lam/mu); the cone multiplier delta; v = w0 - c/mu */
    for (int32_t j = 0; j < n; ++j) h->a[j] = h->x2[j] - h->lam[j] / mu;
    for (int32_t j = 0; j < h->n_orth; ++j) lorentz(h->a + j, h->x1 + j, 1);
    for (int32_t q = 0; q < h->n_soc; ++q) lorentz(h->a + h->soc_off[q], h->x1 + h->soc_off[q], h->soc_size[q]);
    for (int32_t j = 0; j < n; ++j) {
        h->delta[j] = h->lam[j] + mu * (h->x1[j] - h->x2[j]);
        h->v[j] = h->x1[j] + h->lam[j] / mu - h->c[j] / mu;
    }
    /* (A A') nu = A v - b by CG from the previous nu */
    mul_A(h, h->v, h->g);
    for (int32_t i = 0; i < m; ++i) h->g[i] -= h->b[i];
    mul_At(h, h->nu, h->tn);
    mul_A(h, h->tn, h->q);
    for (int32_t i = 0; i < m; ++i) {
        h->r[i] = h->g[i] - h->q[i];
        h->p[i] = h->r[i];
    }
    double rr = dot(h->r, h->r, m);
    const double thr = h->cg_tol * (1.0 + h->bnorm);
    for (int32_t s = 0; s < h->cg_iters && rr > thr * thr; ++s) {
        mul_At(h, h->p, h->tn);
        mul_A(h, h->tn, h->q);
        const double pq = dot(h->p, h->q, m);
        if (!(pq > 0.0)) break;   /* breakdown: p'(A A')p is not positive (p in the null space) */
        const double alpha = rr / pq;
        for (int32_t i = 0; i < m; ++i) {
            h->nu[i] += alpha * h->p[i];
            h->r[i] -= alpha * h->q[i];
        }
        const double rr_new = dot(h->r, h->r, m);
        const double beta = rr_new / rr;
        for (int32_t i = 0; i < m; ++i) h->p[i] = h->r[i] + beta * h->p[i];
        rr = rr_new;
        h->cg_steps++;
    }
    /* x2 = w = v - A'nu;  lam <- lam + mu (x1 - x2) */
    mul_At(h, h->nu, h->tn);
    for (int32_t j = 0; j < n; ++j) {
        h->x2[j] = h->v[j] - h->tn[j];
        h->lam[j] += mu * (h->x1[j] - h->x2[j]);
    }
    h->iter++;
}

void ors_iterate(ors_t *h, int64_t k)
{
    for (int64_t it = 0; it < k; ++it) iterate_once(h);
}

/* Residuals at z = x1, lambda_A = mu nu, delta (SCS form):
 *   out[0] ||A z - b|| / (1 + ||b||),  out[1] ||A'lambda_A + c - delta|| / (1 + ||c||),
 *   out[2] |c'z + b'lambda_A| / (1 + |c'z| + |b'lambda_A|),  out[3] max of the three,
 *   out[4] c'z,  out[5] -b'lambda_A,  out[6] ||x1 - x2||_2,  out[7] CG steps so far */
void ors_residuals(ors_t *h, double *out)
{
    const int32_t m = h->m, n = h->n;
    double *az = (double *)zalloc((size_t)m, sizeof(double));
    double *la = (double *)zalloc((size_t)m, sizeof(double));
    double *atl = (double *)zalloc((size_t)n, sizeof(double));
    mul_A(h, h->x1, az);
    for (int32_t i = 0; i < m; ++i) la[i] = h->mu * h->nu[i];
    mul_At(h, la, atl);
    double rp = 0.0, rd = 0.0, cc = 0.0, cz = 0.0, bl = 0.0, d12 = 0.0;
    for (int32_t i = 0; i < m; ++i) {
        rp += (az[i] - h->b[i]) * (az[i] - h->b[i]);
        bl += h->b[i] * la[i];
    }
    for (int32_t j = 0; j < n; ++j) {
        const double t = atl[j] + h->c[j] - h->delta[j];
        rd += t * t;
        cc += h->c[j] * h->c[j];
        cz += h->c[j] * h->x1[j];
        d12 += (h->x1[j] - h->x2[j]) * (h->x1[j] - h->x2[j]);
    }
    free(az); free(la); free(atl);
    out[0] = sqrt(rp) / (1.0 + h->bnorm);
    out[1] = sqrt(rd) / (1.0 + sqrt(cc));
    out[2] = fabs(cz + bl) / (1.0 + fabs(cz) + fabs(bl));
    out[3] = fmax(out[0], fmax(out[1], out[2]));
    out[4] = cz;
    out[5] = -bl;
    out[6] = sqrt(d12);
    out[7] = (double)h->cg_steps;
}
