/* A plain C client of the solver's C ABI: builds a small standard-form LP
 * with a known optimum, solves it to a 1e-4 KKT residual and prints the
 * residuals; reads the residual history of the run; then gives the same
 * handle the right-hand side 2b (optimum 2 x0, the same duals, so p* doubles)
 * and solves again from the zero start.  Exit status 0 when both solves
 * converged to their known optima and the history ends at the stopping
 * check.
 *
 * LP: A (m x n, k entries per column at rows (j + r * step) mod m), b = A x0
 * with x0 = (1, 0, 1, 0, ...), c = A'y0 + s0 with y0 = 1 and s0 = 1 where
 * x0 = 0, so (x0, -y0, s0) is a primal-dual optimum: p* = c'x0. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "uvadmm.h"

int main(void)
{
    const int32_t m = 300, n = 800, k = 4, step = 37;
    /* columns first, then converted to CSR */
    int64_t *row_ptr = calloc((size_t)m + 1, sizeof(int64_t));
    int32_t *col_idx = malloc(sizeof(int32_t) * (size_t)n * k);
    double *val = malloc(sizeof(double) * (size_t)n * k);
    double *b = calloc((size_t)m, sizeof(double)), *c = calloc((size_t)n, sizeof(double));
    double *x0 = calloc((size_t)n, sizeof(double));
    int32_t *fill = calloc((size_t)m, sizeof(int32_t));
    if (!row_ptr || !col_idx || !val || !b || !c || !x0 || !fill) return 2;
    for (int32_t j = 0; j < n; ++j)
        for (int32_t r = 0; r < k; ++r) row_ptr[(j + r * step) % m + 1]++;
    for (int32_t i = 0; i < m; ++i) row_ptr[i + 1] += row_ptr[i];
    for (int32_t j = 0; j < n; ++j) {           /* columns in increasing order keep rows sorted */
        for (int32_t r = 0; r < k; ++r) {
            const int32_t i = (j + r * step) % m;
            const int64_t p = row_ptr[i] + fill[i]++;
            col_idx[p] = j;
            val[p] = 1.0 + 0.25 * ((j * 7 + r * 3) % 5);
        }
    }
    for (int32_t j = 0; j < n; ++j) x0[j] = (j % 2 == 0) ? 1.0 : 0.0;
    double p_star = 0.0;
    for (int32_t i = 0; i < m; ++i)
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            b[i] += val[p] * x0[col_idx[p]];
            c[col_idx[p]] += val[p];               /* A'y0 with y0 = 1 */
        }
    for (int32_t j = 0; j < n; ++j) {
        if (x0[j] == 0.0) c[j] += 1.0;           /* s0 */
        p_star += c[j] * x0[j];
    }
    uv_csr A = {m, n, row_ptr[m], row_ptr, col_idx, val};
    uv_cones K = {n, 0, NULL};
    uv_opts o;
    uv_default_opts(&o);
    o.eps_kkt = 1e-4;
    o.history = 100000;
    uv_solver *s = NULL;
    int rc = solver_create(&A, b, c, &K, &o, &s);
    if (rc != UV_OK) {
        fprintf(stderr, "solver_create: %s\n", solver_strerror(rc));
        return 1;
    }
    int32_t done = 0;
    for (int round = 0; round < 100 && !done; ++round) {
        rc = solver_iterate(s, 2000, &done);
        if (rc != UV_OK) {
            fprintf(stderr, "solver_iterate: %s\n", solver_strerror(rc));
            return 1;
        }
    }
    uv_residuals r;
    rc = solver_residuals(s, &r);
    double *z = malloc(sizeof(double) * (size_t)n);
    if (rc == UV_OK && z) rc = solver_solution(s, NULL, z, NULL, NULL);
    if (rc != UV_OK || !z) return 1;
    printf("status %d iterations %lld kkt %.3e pobj %.9f p* %.9f\n", r.status, (long long)r.iter, r.kkt, r.pobj,
           p_star);
    int ok = r.status == UV_STATUS_CONVERGED && fabs(r.pobj - p_star) <= 1e-3 * (1.0 + fabs(p_star));

    /* the residual history: one record per check, the last one the stopping check */
    const int32_t cap = 100000;
    uv_history *h = malloc(sizeof(uv_history) * (size_t)cap);
    int32_t cnt = 0;
    if (!h || solver_history(s, cap, h, &cnt) != UV_OK) return 1;
    int hist_ok = cnt == (int32_t)(r.iter / o.check_every) && cnt > 0 && h[cnt - 1].iter == r.iter &&
                  h[cnt - 1].kkt == r.kkt && h[0].iter == o.check_every;
    for (int32_t q = 1; q < cnt; ++q)
        hist_ok = hist_ok && h[q].iter == h[q - 1].iter + o.check_every && h[q].seconds >= h[q - 1].seconds;
    printf("history %d records, first at %lld, last kkt %.3e\n", cnt, cnt ? (long long)h[0].iter : -1LL,
           cnt ? h[cnt - 1].kkt : 0.0);
    ok = ok && hist_ok;

    /* a new right-hand side on the same handle: no iteration before a new start */
    for (int32_t i = 0; i < m; ++i) b[i] *= 2.0;
    int32_t d2 = 0;
    rc = solver_set_rhs(s, b);
    const int refused = solver_iterate(s, 10, &d2) == UV_EINVAL;
    if (rc == UV_OK) rc = solver_set_start(s, NULL, NULL, NULL, NULL);
    for (int round = 0; rc == UV_OK && round < 100 && !d2; ++round) rc = solver_iterate(s, 2000, &d2);
    uv_residuals r2;
    if (rc == UV_OK) rc = solver_residuals(s, &r2);
    solver_destroy(s);
    if (rc != UV_OK) return 1;
    printf("rhs 2b: status %d iterations %lld pobj %.9f 2p* %.9f\n", r2.status, (long long)r2.iter, r2.pobj,
           2.0 * p_star);
    ok = ok && refused && r2.status == UV_STATUS_CONVERGED &&
         fabs(r2.pobj - 2.0 * p_star) <= 1e-3 * (1.0 + fabs(2.0 * p_star));
    free(row_ptr); free(col_idx); free(val); free(b); free(c); free(x0); free(fill); free(z); free(h);
    return ok ? 0 : 1;
}
