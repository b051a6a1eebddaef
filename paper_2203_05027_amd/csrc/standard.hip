// standard.hip -- standard two-block ADMM with an indirect solve of the
// block system eq. lin every iteration: the method the UV decomposition is
// set against (Section II-B, ADMM on the splitting x1 = x2 with f the cone
// indicator and g the objective on {A x = b}; Section III-B, indirect
// methods: conjugate gradients warm-started from the previous iteration).
// FP64; K = orthant coordinates, then Lorentz cones.  Every sparse product runs through the slab
// kernel of the UV solver (spmv.hpp) with the same slab choice, so a
// comparison of the two measures the methods, not two SpMV codes.
//
// One iteration, in the paper's order:
//   x1 = proj_K(x2 - lam/mu);  delta = lam + mu (x1 - x2);  v = x1 + lam/mu - c/mu
//   eq. lin with w0 = x1 + lam/mu: eliminating w = v - A'nu leaves
//   (A A') nu = A v - b, solved by conjugate gradients from the previous nu:
//   at most cg_iters steps, stopping once ||r||_2 <= cg_tol (1 + ||b||_2) or
//   at a breakdown (p'A A'p not positive).  w = A'nu is carried along the
//   CG updates (w += alpha A'p), so the starting residual
//   r = A (v - w) - b takes one product and x2 needs none;
//   x2 = v - w;  lam += mu (x1 - x2).
// Multipliers of the original problem: lambda_A = mu nu for A x = b (the
// paper's sign, c + A'lambda_A - delta = 0 at a solution) and delta for the
// cone; residuals (SCS form) at z = x1.
//
// CG scalars live in device memory (one workgroup reduces the per-workgroup
// partials in a fixed order), so an iteration is a fixed sequence of
// launches with no host round trip; a device flag turns the remaining CG
// launches of an iteration into no-ops once CG has stopped.  Deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/uvadmm.h"
#include "common.hpp"
#include "setup.hpp"
#include "spmv.hpp"

namespace {

struct StdStatus {
    double rr, alpha, beta, thr;  // CG: r'r, step, direction update, stop threshold on ||r||
    double r_prim, r_dual, r_gap, kkt, pobj, dobj;
    double bnorm2, cnorm2;
    long long iter, check_iter, cg_steps;
    int done;    // 1 = stop: every kernel of an iteration returns at once
    int idle;    // 1 = CG of this iteration has stopped (or done)
    int status;  // UV_STATUS_*
    int skip_col;  // 1: the check's primal half failed, its column half is skipped
};

// Sum of nb per-workgroup partials in a fixed order (one workgroup).
__device__ __forceinline__ double reduce_partials(const double *__restrict__ part, int nb)
{
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < nb; i += kWG) v[0] += part[i];
    __shared__ double out;
    uv::block_sum<1>(v, &out, 1);
    __syncthreads();
    return out;
}

__global__ void __launch_bounds__(kWG)
k_std_norms(int m, const double *__restrict__ b, int n, const double *__restrict__ c, StdStatus *st)
{
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < m; i += kWG) v[0] += b[i] * b[i];
    for (int j = threadIdx.x; j < n; j += kWG) v[1] += c[j] * c[j];
    __shared__ double out[2];
    uv::block_sum<2>(v, out, 1);
    if (threadIdx.x == 0) {
        st->bnorm2 = out[0];
        st->cnorm2 = out[1];
    }
}

// x1 step on the orthant coordinates [0, n_orth), the cone multiplier, v and
// d = v - w (w = A'nu).
__global__ void __launch_bounds__(kWG)
k_std_x1(int n_orth, const double *__restrict__ x2, const double *__restrict__ lam, const double *__restrict__ c,
         const double *__restrict__ w, double *__restrict__ x1, double *__restrict__ delta, double *__restrict__ v,
         double *__restrict__ d, double mu, double inv_mu, const StdStatus *st)
{
    if (st->done) return;
    const int j = blockIdx.x * kWG + threadIdx.x;
    if (j >= n_orth) return;
    const double l = lam[j], x2j = x2[j];
    const double a = x2j - l * inv_mu;
    const double x1j = a > 0.0 ? a : 0.0;
    x1[j] = x1j;
    delta[j] = l + mu * (x1j - x2j);
    const double vj = x1j + l * inv_mu - c[j] * inv_mu;
    v[j] = vj;
    d[j] = vj - w[j];
}

// The same on the Lorentz cones, a wavefront per cone [off[q], off[q+1]):
// the lanes take the cone's coordinates 64 apart (coalesced), a fixed
// butterfly adds the tail's squares, then eq. proj on a = x2 - lam/mu (zero,
// identity, or the boundary point).
__global__ void __launch_bounds__(kWG)
k_std_x1_soc(int n_soc, const int *__restrict__ off, const double *__restrict__ x2,
             const double *__restrict__ lam, const double *__restrict__ c, const double *__restrict__ w,
             double *__restrict__ x1, double *__restrict__ delta, double *__restrict__ v, double *__restrict__ d,
             double mu, double inv_mu, const StdStatus *st)
{
    if (st->done) return;
    const int q = blockIdx.x * (kWG / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (q >= n_soc) return;  // the whole wavefront leaves
    const int j0 = off[q], j1 = off[q + 1];
    double t2 = 0.0;
    for (int j = j0 + 1 + lane; j < j1; j += 64) {
        const double a = x2[j] - lam[j] * inv_mu;
        t2 += a * a;
    }
    const double na = sqrt(uv::group_sum<64>(t2));
    const double w1 = x2[j0] - lam[j0] * inv_mu;
    // x1_j = head for j0, scale * a_j for the tail
    double head, scale;
    if (na <= -w1) { head = 0.0; scale = 0.0; }
    else if (na <= w1) { head = w1; scale = 1.0; }
    else { head = 0.5 * (w1 + na); scale = 0.5 * (1.0 + w1 / na); }
    for (int j = j0 + lane; j < j1; j += 64) {
        const double l = lam[j], x2j = x2[j];
        const double x1j = j == j0 ? head : scale * (x2j - l * inv_mu);
        x1[j] = x1j;
        delta[j] = l + mu * (x1j - x2j);
        const double vj = x1j + l * inv_mu - c[j] * inv_mu;
        v[j] = vj;
        d[j] = vj - w[j];
    }
}

// r = p = sum_s P[s] - b and the partial sums of r'r.
template <int S>
__global__ void __launch_bounds__(kWG)
k_std_r0(int m, const double *__restrict__ P, const double *__restrict__ b, double *__restrict__ r,
         double *__restrict__ p, double *__restrict__ part, const StdStatus *st)
{
    if (st->done) return;
    const int i = blockIdx.x * kWG + threadIdx.x;
    double v[1] = {0.0};
    if (i < m) {
        double q = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s) q += P[(size_t)s * m + i];
        const double ri = q - b[i];
        r[i] = ri;
        p[i] = ri;
        v[0] = ri * ri;
    }
    uv::block_sum<1>(v, part + blockIdx.x, 1);
}

__global__ void __launch_bounds__(kWG)
k_std_cg_start(int nb, const double *__restrict__ part, StdStatus *st)
{
    if (st->done) {
        if (threadIdx.x == 0) st->idle = 1;
        return;
    }
    const double rr = reduce_partials(part, nb);
    if (threadIdx.x == 0) {
        st->rr = rr;
        st->idle = rr > st->thr * st->thr ? 0 : 1;
    }
}

// t = sum_s P[s]  (A'p from the column slabs)
template <int S>
__global__ void __launch_bounds__(kWG)
k_std_sum(int n, const double *__restrict__ P, double *__restrict__ t, const StdStatus *st)
{
    if (st->idle) return;
    const int j = blockIdx.x * kWG + threadIdx.x;
    if (j >= n) return;
    double a = 0.0;
#pragma unroll
    for (int s = 0; s < S; ++s) a += P[(size_t)s * n + j];
    t[j] = a;
}

// q = sum_s P[s]  (A A'p) and the partial sums of p'q.
template <int S>
__global__ void __launch_bounds__(kWG)
k_std_q(int m, const double *__restrict__ P, const double *__restrict__ p, double *__restrict__ q,
        double *__restrict__ part, const StdStatus *st)
{
    if (st->idle) return;
    const int i = blockIdx.x * kWG + threadIdx.x;
    double v[1] = {0.0};
    if (i < m) {
        double a = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s) a += P[(size_t)s * m + i];
        q[i] = a;
        v[0] = p[i] * a;
    }
    uv::block_sum<1>(v, part + blockIdx.x, 1);
}

__global__ void __launch_bounds__(kWG)
k_std_alpha(int nb, const double *__restrict__ part, StdStatus *st)
{
    if (st->idle) return;
    const double pq = reduce_partials(part, nb);
    if (threadIdx.x == 0) {
        if (pq > 0.0) st->alpha = st->rr / pq;
        else st->idle = 1;  // breakdown
    }
}

// nu += alpha p, r -= alpha q (partial sums of r'r); w += alpha t.
__global__ void __launch_bounds__(kWG)
k_std_step(int m, int n, const double *__restrict__ p, const double *__restrict__ q, const double *__restrict__ t,
           double *__restrict__ nu, double *__restrict__ r, double *__restrict__ w, double *__restrict__ part,
           const StdStatus *st)
{
    if (st->idle) return;
    const int i = blockIdx.x * kWG + threadIdx.x;
    const double alpha = st->alpha;
    double v[1] = {0.0};
    if (i < m) {
        nu[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        v[0] = ri * ri;
    }
    if (i < n) w[i] += alpha * t[i];
    uv::block_sum<1>(v, part + blockIdx.x, 1);
}

__global__ void __launch_bounds__(kWG)
k_std_beta(int nb, const double *__restrict__ part, StdStatus *st)
{
    if (st->idle) return;
    const double rr = reduce_partials(part, nb);
    if (threadIdx.x == 0) {
        st->beta = rr / st->rr;
        st->rr = rr;
        st->cg_steps += 1;
        if (!(rr > st->thr * st->thr)) st->idle = 1;
    }
}

__global__ void __launch_bounds__(kWG)
k_std_p(int m, const double *__restrict__ r, double *__restrict__ p, const StdStatus *st)
{
    if (st->idle) return;
    const int i = blockIdx.x * kWG + threadIdx.x;
    if (i < m) p[i] = r[i] + st->beta * p[i];
}

// x2 = v - w;  lam += mu (x1 - x2)
__global__ void __launch_bounds__(kWG)
k_std_x2(int n, const double *__restrict__ v, const double *__restrict__ w, const double *__restrict__ x1,
         double *__restrict__ x2, double *__restrict__ lam, double mu, StdStatus *st)
{
    if (st->done) return;
    const int j = blockIdx.x * kWG + threadIdx.x;
    if (j < n) {
        const double x2j = v[j] - w[j];
        x2[j] = x2j;
        lam[j] += mu * (x1[j] - x2j);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) st->iter += 1;
}

// Residual partials: rows (A z - b)^2, b'lambda_A; columns
// (A'lambda_A + c - delta)^2, c'z, with lambda_A = mu nu, z = x1.
template <int S>
__global__ void __launch_bounds__(kWG)
k_std_res_row(int m, const double *__restrict__ P, const double *__restrict__ b, const double *__restrict__ nu,
              double mu, double *__restrict__ part, int pstride)
{
    const int i = blockIdx.x * kWG + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (i < m) {
        double az = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s) az += P[(size_t)s * m + i];
        const double e = az - b[i];
        v[0] = e * e;
        v[1] = b[i] * (mu * nu[i]);
    }
    uv::block_sum<2>(v, part + blockIdx.x, pstride);
}

template <int S>
__global__ void __launch_bounds__(kWG)
k_std_res_col(int n, const double *__restrict__ P, const double *__restrict__ c, const double *__restrict__ delta,
              const double *__restrict__ z, double mu, double *__restrict__ part, int pstride, const int *skip)
{
    if (skip && *skip) return;  // the check's column half is ruled out (uniform)
    const int j = blockIdx.x * kWG + threadIdx.x;
    double v[2] = {0.0, 0.0};
    if (j < n) {
        double a = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s) a += P[(size_t)s * n + j];
        const double e = mu * a + c[j] - delta[j];
        v[0] = e * e;
        v[1] = c[j] * z[j];
    }
    uv::block_sum<2>(v, part + blockIdx.x, pstride);
}

// The primal half of a check first, as in the UV solver: the row partials
// summed as k_std_finalize sums them (bit for bit the same values); when
// r_prim > eps with finite sums the check cannot stop the run and its column
// half (the A' nu product, its partials and the finalize) is skipped.
__global__ void __launch_bounds__(kWG)
k_std_gate(int nr, const double *__restrict__ prow, double eps, StdStatus *st)
{
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < nr; i += kWG) {
        v[0] += prow[i];
        v[1] += prow[nr + i];
    }
    __shared__ double s[2];
    uv::block_sum<2>(v, s, 1);
    if (threadIdx.x != 0) return;
    if (st->done) {
        st->skip_col = 1;
        return;
    }
    const bool fails = !(sqrt(s[0]) / (1.0 + sqrt(st->bnorm2)) <= eps);
    st->skip_col = fails && isfinite(s[0]) && isfinite(s[1]) ? 1 : 0;
}

__global__ void __launch_bounds__(kWG)
k_std_finalize(int nr, const double *__restrict__ prow, int nc, const double *__restrict__ pcol, double eps,
               StdStatus *st, int gated)
{
    if (gated && st->skip_col) return;  // ruled out by k_std_gate (uniform)
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nr; i += kWG) {
        v[0] += prow[i];
        v[1] += prow[nr + i];
    }
    for (int j = threadIdx.x; j < nc; j += kWG) {
        v[2] += pcol[j];
        v[3] += pcol[nc + j];
    }
    __shared__ double s[4];
    uv::block_sum<4>(v, s, 1);
    if (threadIdx.x != 0) return;
    const double bl = s[1], cz = s[3];
    st->r_prim = sqrt(s[0]) / (1.0 + sqrt(st->bnorm2));
    st->r_dual = sqrt(s[2]) / (1.0 + sqrt(st->cnorm2));
    st->r_gap = fabs(cz + bl) / (1.0 + fabs(cz) + fabs(bl));
    st->kkt = uv::kkt_of(st->r_prim, st->r_dual, st->r_gap);
    st->pobj = cz;
    st->dobj = -bl;
    st->check_iter = st->iter;
    if (st->done) return;
    if (!isfinite(st->kkt)) {
        st->status = UV_STATUS_NUMERIC;
        st->done = 1;
    } else if (st->kkt <= eps) {
        st->status = UV_STATUS_CONVERGED;
        st->done = 1;
    }
}

}  // namespace

struct uv_standard {
    int m = 0, n = 0, nnz = 0, S_row = 1, S_col = 1, cg_iters = 10;
    int n_orth = 0, n_soc = 0;
    int *soc_off = nullptr;  // n_soc + 1 cone boundaries
    double mu = 1.0, eps = 0.0;
    int check_every = 10;
    bool gated = true;  // checks of the iteration evaluate their primal half first (opts.full_checks = 0)
    int64_t max_iter = 0, host_iter = 0;
    hipStream_t stream = nullptr, cap = nullptr;
    bool own_stream = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void *> allocs;
    int *rp = nullptr, *ci = nullptr, *cp = nullptr, *ri = nullptr;
    double *va = nullptr, *vc = nullptr;
    int *srp = nullptr, *sci = nullptr, *scp = nullptr, *sri = nullptr;  // slab copies (or the plain ones)
    double *sva = nullptr, *svc = nullptr;
    double *b = nullptr, *c = nullptr;
    double *x1 = nullptr, *x2 = nullptr, *lam = nullptr, *delta = nullptr, *v = nullptr, *d = nullptr, *w = nullptr,
           *t = nullptr;
    double *nu = nullptr, *r = nullptr, *p = nullptr, *q = nullptr;
    double *P_row = nullptr, *P_col = nullptr, *part = nullptr, *part_row = nullptr, *part_col = nullptr;
    StdStatus *st = nullptr, *st_host = nullptr;
};

namespace {

#define UV_TRY(expr)                               \
    do {                                           \
        if ((expr) != hipSuccess) return UV_EHIP;  \
    } while (0)

template <typename T>
T *salloc(uv_standard *h, size_t count)
{
    void *p = nullptr;
    if (uv::dev_malloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return nullptr;
    h->allocs.push_back(p);
    return (T *)p;
}

// A'vec into P_col (S_col partials) and A vec into P_row (S_row partials).
template <int S>
void prod_col(uv_standard *h, hipStream_t st, const double *vec, const int *skip)
{
    k_seg_chunk<double, double, S, 8><<<S * blocks_for(h->n, kWG), kWG, 0, st>>>(h->n, h->scp, h->sri, h->svc, vec,
                                                                            h->P_col, skip);
}

template <int S>
void prod_row(uv_standard *h, hipStream_t st, const double *vec, const int *skip)
{
    k_seg_chunk<double, double, S, 8><<<S * blocks_for(h->m, kWG), kWG, 0, st>>>(h->m, h->srp, h->sci, h->sva, vec,
                                                                            h->P_row, skip);
}

template <int SR, int SC>
void iteration(uv_standard *h, hipStream_t st, bool check)
{
    const int m = h->m, n = h->n;
    const unsigned gm = blocks_for(m, kWG), gn = blocks_for(n, kWG), gmn = blocks_for(std::max(m, n), kWG);
    const double mu = h->mu, im = 1.0 / h->mu;
    const int *done = &h->st->done, *idle = &h->st->idle;
    if (h->n_orth > 0)
        k_std_x1<<<blocks_for(h->n_orth, kWG), kWG, 0, st>>>(h->n_orth, h->x2, h->lam, h->c, h->w, h->x1, h->delta,
                                                              h->v, h->d, mu, im, h->st);
    if (h->n_soc > 0)
        k_std_x1_soc<<<blocks_for(h->n_soc, kWG / 64), kWG, 0, st>>>(h->n_soc, h->soc_off, h->x2, h->lam, h->c, h->w,
                                                                h->x1, h->delta, h->v, h->d, mu, im, h->st);
    prod_row<SR>(h, st, h->d, done);
    k_std_r0<SR><<<gm, kWG, 0, st>>>(m, h->P_row, h->b, h->r, h->p, h->part, h->st);
    k_std_cg_start<<<1, kWG, 0, st>>>((int)gm, h->part, h->st);
    for (int k = 0; k < h->cg_iters; ++k) {
        prod_col<SC>(h, st, h->p, idle);
        k_std_sum<SC><<<gn, kWG, 0, st>>>(n, h->P_col, h->t, h->st);
        prod_row<SR>(h, st, h->t, idle);
        k_std_q<SR><<<gm, kWG, 0, st>>>(m, h->P_row, h->p, h->q, h->part, h->st);
        k_std_alpha<<<1, kWG, 0, st>>>((int)gm, h->part, h->st);
        k_std_step<<<gmn, kWG, 0, st>>>(m, n, h->p, h->q, h->t, h->nu, h->r, h->w, h->part, h->st);
        k_std_beta<<<1, kWG, 0, st>>>((int)gmn, h->part, h->st);
        k_std_p<<<gm, kWG, 0, st>>>(m, h->r, h->p, h->st);
    }
    k_std_x2<<<gn, kWG, 0, st>>>(n, h->v, h->w, h->x1, h->x2, h->lam, mu, h->st);
    if (!check) return;
    prod_row<SR>(h, st, h->x1, nullptr);
    k_std_res_row<SR><<<gm, kWG, 0, st>>>(m, h->P_row, h->b, h->nu, mu, h->part_row, (int)gm);
    const int *skip = h->gated ? &h->st->skip_col : nullptr;
    if (h->gated) k_std_gate<<<1, kWG, 0, st>>>((int)gm, h->part_row, h->eps, h->st);
    prod_col<SC>(h, st, h->nu, skip);
    k_std_res_col<SC><<<gn, kWG, 0, st>>>(n, h->P_col, h->c, h->delta, h->x1, mu, h->part_col, (int)gn, skip);
    k_std_finalize<<<1, kWG, 0, st>>>((int)gm, h->part_row, (int)gn, h->part_col, h->eps, h->st, h->gated ? 1 : 0);
}

template <int SR>
void iteration_sc(uv_standard *h, hipStream_t st, bool check)
{
    if (h->S_col == 2) iteration<SR, 2>(h, st, check);
    else if (h->S_col == 4) iteration<SR, 4>(h, st, check);
    else iteration<SR, 1>(h, st, check);
}

void launch_iteration(uv_standard *h, hipStream_t st, bool check)
{
    if (h->S_row == 2) iteration_sc<2>(h, st, check);
    else if (h->S_row == 4) iteration_sc<4>(h, st, check);
    else iteration_sc<1>(h, st, check);
}

// Residual check of the current state only (no iteration).
template <int SR, int SC>
void check_only(uv_standard *h, hipStream_t st)
{
    const unsigned gm = blocks_for(h->m, kWG), gn = blocks_for(h->n, kWG);
    prod_row<SR>(h, st, h->x1, nullptr);
    k_std_res_row<SR><<<gm, kWG, 0, st>>>(h->m, h->P_row, h->b, h->nu, h->mu, h->part_row, (int)gm);
    prod_col<SC>(h, st, h->nu, nullptr);
    k_std_res_col<SC><<<gn, kWG, 0, st>>>(h->n, h->P_col, h->c, h->delta, h->x1, h->mu, h->part_col, (int)gn,
                                          nullptr);
    k_std_finalize<<<1, kWG, 0, st>>>((int)gm, h->part_row, (int)gn, h->part_col, h->eps, h->st, 0);
}

void launch_check(uv_standard *h, hipStream_t st)
{
    auto sc = [&](auto sr) {
        constexpr int SR = decltype(sr)::value;
        if (h->S_col == 2) check_only<SR, 2>(h, st);
        else if (h->S_col == 4) check_only<SR, 4>(h, st);
        else check_only<SR, 1>(h, st);
    };
    if (h->S_row == 2) sc(std::integral_constant<int, 2>());
    else if (h->S_row == 4) sc(std::integral_constant<int, 4>());
    else sc(std::integral_constant<int, 1>());
}

int sync_status(uv_standard *h)
{
    UV_TRY(hipMemcpyAsync(h->st_host, h->st, sizeof(StdStatus), hipMemcpyDeviceToHost, h->stream));
    UV_TRY(hipStreamSynchronize(h->stream));
    h->host_iter = h->st_host->iter;
    return UV_OK;
}

}  // namespace

extern "C" {

void standard_destroy(uv_standard *h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    for (void *p : h->allocs) (void)hipFree(p);
    if (h->st_host) (void)hipHostFree(h->st_host);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

int standard_create(const uv_csr *A, const double *b, const double *c, const uv_cones *K, const uv_opts *opts,
                    int32_t cg_iters, double cg_tol, uv_standard **out)
{
    if (!out) return UV_EINVAL;
    *out = nullptr;
    uv_opts o;
    uv_default_opts(&o);
    if (opts) o = *opts;
    if (!A || !b || !c || !A->row_ptr || A->m < 1 || A->n < 1 || A->nnz < 0) return UV_EINVAL;
    if (!(o.mu > 0.0) || !std::isfinite(o.mu) || o.precision != UV_FP64) return UV_EINVAL;
    if (o.check_every < 1 || !(o.eps_kkt >= 0.0) || o.max_iter < 0) return UV_EINVAL;
    if (o.full_checks < 0 || o.full_checks > 1) return UV_EINVAL;
    if (cg_iters < 0 || !(cg_tol >= 0.0) || !std::isfinite(cg_tol)) return UV_EINVAL;
    if (o.slabs_row != 0 && o.slabs_row != 1 && o.slabs_row != 2 && o.slabs_row != 4) return UV_EINVAL;
    if (o.slabs_col != 0 && o.slabs_col != 1 && o.slabs_col != 2 && o.slabs_col != 4) return UV_EINVAL;
    if (A->nnz > 0 && (!A->col_idx || !A->val)) return UV_EINVAL;
    if (A->nnz >= ((int64_t)1 << 31)) return UV_ETOOBIG;
    if (A->row_ptr[0] != 0 || A->row_ptr[A->m] != A->nnz) return UV_EBADCSR;
    for (int32_t i = 0; i < A->m; ++i) {
        const int64_t b0 = A->row_ptr[i], b1 = A->row_ptr[i + 1];
        if (b1 < b0 || b1 > A->nnz) return UV_EBADCSR;
        for (int64_t k = b0; k < b1; ++k) {
            if (A->col_idx[k] < 0 || A->col_idx[k] >= A->n) return UV_EBADCSR;
            if (k > b0 && A->col_idx[k] <= A->col_idx[k - 1]) return UV_EBADCSR;
        }
    }
    int32_t n_orth = A->n, n_soc = 0;
    if (K) {
        if (K->n_orthant < 0 || K->n_soc < 0 || (K->n_soc > 0 && !K->soc_sizes)) return UV_ECONE;
        int64_t tot = K->n_orthant;
        for (int32_t q = 0; q < K->n_soc; ++q) {
            if (K->soc_sizes[q] < 1) return UV_ECONE;
            tot += K->soc_sizes[q];
        }
        if (tot != A->n) return UV_ECONE;
        n_orth = K->n_orthant;
        n_soc = K->n_soc;
    }
    uv_standard *h = new (std::nothrow) uv_standard();
    if (!h) return UV_ENOMEM;
    auto fail = [&](int code) {
        standard_destroy(h);
        return code;
    };
    const int m = A->m, n = A->n, nnz = (int)A->nnz;
    h->n_orth = n_orth;
    h->n_soc = n_soc;
    h->m = m;
    h->n = n;
    h->nnz = nnz;
    h->mu = o.mu;
    h->eps = o.eps_kkt;
    h->check_every = o.check_every;
    h->gated = o.full_checks == 0;
    h->max_iter = o.max_iter;
    h->cg_iters = cg_iters;
    h->S_row = o.slabs_row ? o.slabs_row : pick_slabs_row(8 * (size_t)n);
    h->S_col = o.slabs_col ? o.slabs_col : pick_slabs_col(8 * (size_t)m);
    while (h->S_row > 1 && (h->S_row > n || (int64_t)h->S_row * m >= INT32_MAX)) h->S_row >>= 1;
    while (h->S_col > 1 && (h->S_col > m || (int64_t)h->S_col * n >= INT32_MAX)) h->S_col >>= 1;
    if (o.hip_stream) h->stream = (hipStream_t)o.hip_stream;
    else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) return fail(UV_EHIP);
        h->own_stream = true;
    }
    hipStream_t st = h->stream;
    const int nbig = std::max(m, n);
    h->rp = salloc<int>(h, m + 1);
    h->ci = salloc<int>(h, nnz);
    h->va = salloc<double>(h, nnz);
    h->cp = salloc<int>(h, n + 1);
    h->ri = salloc<int>(h, nnz);
    h->vc = salloc<double>(h, nnz);
    h->b = salloc<double>(h, m);
    h->c = salloc<double>(h, n);
    for (double **pp : {&h->x1, &h->x2, &h->lam, &h->delta, &h->v, &h->d, &h->w, &h->t}) *pp = salloc<double>(h, n);
    for (double **pp : {&h->nu, &h->r, &h->p, &h->q}) *pp = salloc<double>(h, m);
    h->P_row = salloc<double>(h, (size_t)h->S_row * m);
    h->P_col = salloc<double>(h, (size_t)h->S_col * n);
    h->part = salloc<double>(h, blocks_for(nbig, kWG));
    h->part_row = salloc<double>(h, 2 * (size_t)blocks_for(m, kWG));
    h->part_col = salloc<double>(h, 2 * (size_t)blocks_for(n, kWG));
    h->st = salloc<StdStatus>(h, 1);
    const size_t ncnt = std::max<size_t>({(size_t)n, (size_t)h->S_row * m, (size_t)h->S_col * n});
    int *cnt = salloc<int>(h, ncnt);
    int *bsum = salloc<int>(h, blocks_for((int64_t)ncnt, 4 * kWG));
    for (void *p : {(void *)h->rp, (void *)h->ci, (void *)h->va, (void *)h->cp, (void *)h->ri, (void *)h->vc,
                    (void *)h->b, (void *)h->c, (void *)h->x1, (void *)h->x2, (void *)h->lam, (void *)h->delta,
                    (void *)h->v, (void *)h->d, (void *)h->w, (void *)h->t, (void *)h->nu, (void *)h->r,
                    (void *)h->p, (void *)h->q, (void *)h->P_row, (void *)h->P_col, (void *)h->part,
                    (void *)h->part_row, (void *)h->part_col, (void *)h->st, (void *)cnt, (void *)bsum})
        if (!p) return fail(UV_ENOMEM);
    if (uv::host_malloc(&h->st_host, sizeof(StdStatus), hipHostMallocDefault) != hipSuccess)
        return fail(UV_ENOMEM);
    std::vector<int> rp32(m + 1);
    for (int i = 0; i <= m; ++i) rp32[i] = (int)A->row_ptr[i];
    if (hipMemcpy(h->rp, rp32.data(), 4 * (size_t)(m + 1), hipMemcpyHostToDevice) != hipSuccess) return fail(UV_EHIP);
    if (nnz > 0 && (hipMemcpy(h->ci, A->col_idx, 4 * (size_t)nnz, hipMemcpyHostToDevice) != hipSuccess ||
                    hipMemcpy(h->va, A->val, 8 * (size_t)nnz, hipMemcpyHostToDevice) != hipSuccess))
        return fail(UV_EHIP);
    if (hipMemcpy(h->b, b, 8 * (size_t)m, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->c, c, 8 * (size_t)n, hipMemcpyHostToDevice) != hipSuccess)
        return fail(UV_EHIP);
    if (n_soc > 0) {
        std::vector<int> offs(n_soc + 1);
        offs[0] = n_orth;
        for (int q = 0; q < n_soc; ++q) offs[q + 1] = offs[q] + K->soc_sizes[q];
        h->soc_off = salloc<int>(h, n_soc + 1);
        if (!h->soc_off) return fail(UV_ENOMEM);
        if (hipMemcpy(h->soc_off, offs.data(), 4 * (size_t)(n_soc + 1), hipMemcpyHostToDevice) != hipSuccess)
            return fail(UV_EHIP);
    }
    if (!build_csc(m, n, nnz, h->rp, h->ci, h->va, h->cp, h->ri, h->vc, cnt, bsum, st)) return fail(UV_EHIP);
    h->srp = h->rp; h->sci = h->ci; h->sva = h->va;
    h->scp = h->cp; h->sri = h->ri; h->svc = h->vc;
    for (int pass = 0; pass < 2; ++pass) {
        const int S = pass == 0 ? h->S_row : h->S_col;
        if (S == 1) continue;
        const int nr = pass == 0 ? m : n, width = pass == 0 ? n : m;
        int *off = salloc<int>(h, (size_t)S * nr + 1);
        int *sidx = salloc<int>(h, nnz);
        double *sval = salloc<double>(h, nnz);
        if (!off || !sidx || !sval) return fail(UV_ENOMEM);
        const int wd = (width + S - 1) / S;
        const bool ok = pass == 0 ? build_slabs(m, nnz, h->rp, h->ci, h->va, S, wd, off, sidx, sval, cnt, bsum, st)
                                  : build_slabs(n, nnz, h->cp, h->ri, h->vc, S, wd, off, sidx, sval, cnt, bsum, st);
        if (!ok) return fail(UV_EHIP);
        if (pass == 0) { h->srp = off; h->sci = sidx; h->sva = sval; }
        else { h->scp = off; h->sri = sidx; h->svc = sval; }
    }
    // CG stop threshold from ||b|| summed on the host in index order.
    double bb = 0.0;
    for (int i = 0; i < m; ++i) bb += b[i] * b[i];
    std::memset(h->st_host, 0, sizeof(StdStatus));
    h->st_host->thr = cg_tol * (1.0 + std::sqrt(bb));
    h->st_host->status = UV_STATUS_RUNNING;
    if (hipMemcpyAsync(h->st, h->st_host, sizeof(StdStatus), hipMemcpyHostToDevice, st) != hipSuccess)
        return fail(UV_EHIP);
    k_std_norms<<<1, kWG, 0, st>>>(m, h->b, n, h->c, h->st);
    for (double *pv : {h->x1, h->x2, h->lam, h->delta, h->w})
        if (hipMemsetAsync(pv, 0, 8 * (size_t)n, st) != hipSuccess) return fail(UV_EHIP);
    if (hipMemsetAsync(h->nu, 0, 8 * (size_t)m, st) != hipSuccess) return fail(UV_EHIP);
    if (hipGetLastError() != hipSuccess) return fail(UV_EHIP);
    if (sync_status(h) != UV_OK) return fail(UV_EHIP);
    if (o.use_graph) {
        if (hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess) return fail(UV_EHIP);
        if (hipStreamBeginCapture(h->cap, hipStreamCaptureModeRelaxed) != hipSuccess) return fail(UV_EHIP);
        for (int i = 0; i < h->check_every; ++i) launch_iteration(h, h->cap, i == h->check_every - 1);
        if (hipStreamEndCapture(h->cap, &h->graph) != hipSuccess) return fail(UV_EHIP);
        if (hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0) != hipSuccess) return fail(UV_EHIP);
    }
    *out = h;
    return UV_OK;
}

int standard_set_state(uv_standard *h, const double *x2, const double *lam, const double *nu)
{
    if (!h) return UV_EINVAL;
    hipStream_t st = h->stream;
    const size_t n8 = 8 * (size_t)h->n, m8 = 8 * (size_t)h->m;
    auto put = [&](double *dst, const double *src, size_t bytes) -> int {
        if (src) UV_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
        else UV_TRY(hipMemsetAsync(dst, 0, bytes, st));
        return UV_OK;
    };
    int rc;
    if ((rc = put(h->x2, x2, n8)) != UV_OK || (rc = put(h->lam, lam, n8)) != UV_OK ||
        (rc = put(h->nu, nu, m8)) != UV_OK)
        return rc;
    UV_TRY(hipMemsetAsync(h->x1, 0, n8, st));
    UV_TRY(hipMemsetAsync(h->delta, 0, n8, st));
    // fresh status (running, CG not idle), then w = A'nu for the carried product
    StdStatus *s = h->st_host;
    const double thr = s->thr, bn = s->bnorm2, cn = s->cnorm2;
    std::memset(s, 0, sizeof(StdStatus));
    s->thr = thr;
    s->bnorm2 = bn;
    s->cnorm2 = cn;
    s->status = UV_STATUS_RUNNING;
    s->check_iter = -1;
    UV_TRY(hipMemcpyAsync(h->st, s, sizeof(StdStatus), hipMemcpyHostToDevice, st));
    const unsigned gn = blocks_for(h->n, kWG);
    if (h->S_col == 2) {
        prod_col<2>(h, st, h->nu, nullptr);
        k_std_sum<2><<<gn, kWG, 0, st>>>(h->n, h->P_col, h->w, h->st);
    } else if (h->S_col == 4) {
        prod_col<4>(h, st, h->nu, nullptr);
        k_std_sum<4><<<gn, kWG, 0, st>>>(h->n, h->P_col, h->w, h->st);
    } else {
        prod_col<1>(h, st, h->nu, nullptr);
        k_std_sum<1><<<gn, kWG, 0, st>>>(h->n, h->P_col, h->w, h->st);
    }
    UV_TRY(hipGetLastError());
    return sync_status(h);
}

int standard_iterate(uv_standard *h, int64_t k, int32_t *done)
{
    if (!h || k < 0) return UV_EINVAL;
    if (done) *done = 0;
    if (!h->st_host->done) {
        int64_t left = k;
        if (h->max_iter > 0) left = std::min<int64_t>(left, h->max_iter - h->host_iter);
        int64_t it = h->host_iter, since = 0;
        const int ce = h->check_every;
        const int64_t look = 50 * (int64_t)ce;  // read the stop flag every 50 checks
        while (left > 0) {
            if (h->exec && it % ce == 0 && left >= ce) {
                UV_TRY(hipGraphLaunch(h->exec, h->stream));
                it += ce;
                left -= ce;
                since += ce;
            } else {
                launch_iteration(h, h->stream, (it + 1) % ce == 0);
                it += 1;
                left -= 1;
                since += 1;
            }
            if (left > 0 && since >= look) {  // stop launching once a check has stopped the run
                UV_TRY(hipGetLastError());
                int rc = sync_status(h);
                if (rc != UV_OK) return rc;
                if (h->st_host->done) break;
                since = 0;
            }
        }
        UV_TRY(hipGetLastError());
        int rc = sync_status(h);
        if (rc != UV_OK) return rc;
    }
    StdStatus *s = h->st_host;
    if (!s->done && h->max_iter > 0 && h->host_iter >= h->max_iter) {
        s->status = UV_STATUS_MAX_ITER;
        s->done = 1;
        UV_TRY(hipMemcpyAsync(h->st, s, sizeof(StdStatus), hipMemcpyHostToDevice, h->stream));
        UV_TRY(hipStreamSynchronize(h->stream));
    }
    if (done) *done = s->done;
    return s->status == UV_STATUS_NUMERIC ? UV_ENUMERIC : UV_OK;
}

int standard_residuals(uv_standard *h, uv_residuals *r, int64_t *cg_steps)
{
    if (!h || !r) return UV_EINVAL;
    if (h->st_host->check_iter != h->st_host->iter) {
        launch_check(h, h->stream);
        UV_TRY(hipGetLastError());
        int rc = sync_status(h);
        if (rc != UV_OK) return rc;
    }
    const StdStatus *s = h->st_host;
    std::memset(r, 0, sizeof(*r));
    r->r_prim = s->r_prim;
    r->r_dual = s->r_dual;
    r->r_gap = s->r_gap;
    r->kkt = s->kkt;
    r->pobj = s->pobj;
    r->dobj = s->dobj;
    r->iter = s->iter;
    r->status = s->status;
    if (cg_steps) *cg_steps = s->cg_steps;
    return UV_OK;
}

int standard_solution(uv_standard *h, double *x1, double *x2, double *lam, double *nu, double *delta)
{
    if (!h) return UV_EINVAL;
    struct { double *dst; const double *src; size_t len; } cp[] = {
        {x1, h->x1, (size_t)h->n}, {x2, h->x2, (size_t)h->n}, {lam, h->lam, (size_t)h->n},
        {nu, h->nu, (size_t)h->m}, {delta, h->delta, (size_t)h->n}};
    for (auto &e : cp)
        if (e.dst && hipMemcpy(e.dst, e.src, 8 * e.len, hipMemcpyDeviceToHost) != hipSuccess) return UV_EHIP;
    return UV_OK;
}

int standard_launch_shape(uv_standard *h, int32_t *slabs_row, int32_t *slabs_col)
{
    if (!h) return UV_EINVAL;
    if (slabs_row) *slabs_row = h->S_row;
    if (slabs_col) *slabs_col = h->S_col;
    return UV_OK;
}

}  // extern "C"
