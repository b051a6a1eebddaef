// literal.hip -- Algorithm 1 as printed, on the GPU: the per-nonzero
// variables y and gamma of the reformulation (eq. prob_reform) are stored and
// updated, U, U', V, V' are applied as sums over the nonzero index (eqs. UU,
// VV).  FP64, orthant cone.  It is the ablation of the reduced form (which
// keeps neither y nor gamma) and a second, independent GPU implementation of
// the iteration.
//
// Nonzero k is numbered in CSR order (row-major).  Per iteration:
//   column pass (column j, its nonzeros through the CSC permutation kcol):
//     x_j = F_V (sum_k (y_k + gamma_k/mu) + z_j + delta_j/mu - c_j/mu)      (Block 1)
//     z_j = max(x_j - delta_j/mu, 0),  delta_j += mu (z_j - x_j)             (z-step, delta)
//   row pass (row i, its nonzeros k in CSR order):
//     t_k = a_k (b_i - lambda_i/mu) + x_{j_k} - gamma_k/mu                   (U'(b - lambda/mu) + V'x - gamma/mu)
//     s_i = F_U sum_k a_k t_k,  y_k = t_k - a_k s_i                          (y-step, inversion lemma)
//     lambda_i += mu (sum_k a_k y_k - b_i),  gamma_k += mu (y_k - x_{j_k})   (dual updates)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/uvadmm.h"
#include "common.hpp"
#include "setup.hpp"

namespace {

template <int L>
__global__ void __launch_bounds__(kWG)
k_lit_col(int n, const int *__restrict__ cp, const int *__restrict__ kcol, const double *__restrict__ y,
          const double *__restrict__ gam, double *__restrict__ x, double *__restrict__ z,
          double *__restrict__ delta, const double *__restrict__ c, double mu, double inv_mu)
{
    const int lane = threadIdx.x & (L - 1);
    const int col = blockIdx.x * (kWG / L) + threadIdx.x / L;
    if (col >= n) return;
    const int beg = cp[col], end = cp[col + 1];
    double acc = 0.0;
    for (int p = beg + lane; p < end; p += L) {
        const int k = kcol[p];
        acc += y[k] + gam[k] * inv_mu;
    }
    acc = uv::group_sum<L>(acc);
    if (lane == 0) {
        const double d = delta[col];
        const double xn = (acc + z[col] + d * inv_mu - c[col] * inv_mu) / (double)(1 + end - beg);
        const double v = xn - d * inv_mu;
        const double zn = v > 0.0 ? v : 0.0;
        x[col] = xn;
        z[col] = zn;
        delta[col] = d + mu * (zn - xn);
    }
}

template <int L>
__global__ void __launch_bounds__(kWG)
k_lit_row(int m, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ va,
          const double *__restrict__ x, const double *__restrict__ b, const double *__restrict__ fu,
          double *__restrict__ lam, double *__restrict__ y, double *__restrict__ gam, double mu, double inv_mu)
{
    const int lane = threadIdx.x & (L - 1);
    const int row = blockIdx.x * (kWG / L) + threadIdx.x / L;
    if (row >= m) return;
    const int beg = rp[row], end = rp[row + 1];
    const double bl = b[row] - lam[row] * inv_mu;
    // U t for this row
    double ut = 0.0;
    for (int k = beg + lane; k < end; k += L) {
        const double t = va[k] * bl + x[ci[k]] - gam[k] * inv_mu;
        ut += va[k] * t;
    }
    ut = uv::group_sum<L>(ut);
    const double s = fu[row] * ut;
    // y, U y, gamma
    double uy = 0.0;
    for (int k = beg + lane; k < end; k += L) {
        const double xj = x[ci[k]];
        const double t = va[k] * bl + xj - gam[k] * inv_mu;
        const double yk = t - va[k] * s;
        y[k] = yk;
        uy += va[k] * yk;
        gam[k] += mu * (yk - xj);
    }
    uy = uv::group_sum<L>(uy);
    if (lane == 0) lam[row] += mu * (uy - b[row]);
}

// kcol: the nonzero index k (CSR position) of each CSC position: entry p of
// column j sits in row ri[p]; its k is found by binary search for j among
// that row's sorted column indices.  No atomics, no sort: deterministic.
__global__ void __launch_bounds__(kWG)
k_lit_kcol(int n, const int *__restrict__ cp, const int *__restrict__ ri, const int *__restrict__ rp,
           const int *__restrict__ ci, int *__restrict__ kcol)
{
    const int j = blockIdx.x * kWG + threadIdx.x;
    if (j >= n) return;
    for (int p = cp[j]; p < cp[j + 1]; ++p) {
        int lo = rp[ri[p]], hi = rp[ri[p] + 1];
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (ci[mid] < j) lo = mid + 1;
            else hi = mid;
        }
        kcol[p] = lo;
    }
}

}  // namespace

struct uv_literal {
    int m = 0, n = 0, nnz = 0, L_row = 4, L_col = 4;
    double mu = 1.0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::vector<void *> allocs;
    int *rp = nullptr, *ci = nullptr, *cp = nullptr, *ri = nullptr, *kcol = nullptr;
    double *va = nullptr, *vc = nullptr, *b = nullptr, *c = nullptr, *fu = nullptr;
    double *x = nullptr, *z = nullptr, *delta = nullptr, *lam = nullptr, *y = nullptr, *gam = nullptr;
};

namespace {

template <typename T>
T *lalloc(uv_literal *h, size_t count)
{
    void *p = nullptr;
    if (uv::dev_malloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return nullptr;
    h->allocs.push_back(p);
    return (T *)p;
}

void lit_iteration(uv_literal *h, hipStream_t st, hipEvent_t mid = nullptr)
{
    const double mu = h->mu, im = 1.0 / h->mu;
#define UV_LIT_COL(LL)                                                                                      \
    k_lit_col<LL><<<blocks_for(h->n, kWG / LL), kWG, 0, st>>>(h->n, h->cp, h->kcol, h->y, h->gam, h->x, h->z, \
                                                              h->delta, h->c, mu, im)
#define UV_LIT_ROW(LL)                                                                                      \
    k_lit_row<LL><<<blocks_for(h->m, kWG / LL), kWG, 0, st>>>(h->m, h->rp, h->ci, h->va, h->x, h->b, h->fu, \
                                                              h->lam, h->y, h->gam, mu, im)
    switch (h->L_col) {
    case 1: UV_LIT_COL(1); break;
    case 2: UV_LIT_COL(2); break;
    case 4: UV_LIT_COL(4); break;
    case 8: UV_LIT_COL(8); break;
    default: UV_LIT_COL(16); break;
    }
    if (mid) (void)hipEventRecord(mid, st);
    switch (h->L_row) {
    case 1: UV_LIT_ROW(1); break;
    case 2: UV_LIT_ROW(2); break;
    case 4: UV_LIT_ROW(4); break;
    case 8: UV_LIT_ROW(8); break;
    default: UV_LIT_ROW(16); break;
    }
#undef UV_LIT_COL
#undef UV_LIT_ROW
}

int pick_l(double avg)
{
    int L = 1;
    while (L < 16 && L * 4 < avg) L <<= 1;
    return L;
}

}  // namespace

extern "C" {

void literal_destroy(uv_literal *h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (void *p : h->allocs) (void)hipFree(p);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

int literal_create(const uv_csr *A, const double *b, const double *c, const uv_opts *opts, uv_literal **out)
{
    if (!out) return UV_EINVAL;
    *out = nullptr;
    uv_opts o;
    uv_default_opts(&o);
    if (opts) o = *opts;
    if (!A || !b || !c || !A->row_ptr || A->m < 1 || A->n < 1 || A->nnz < 0) return UV_EINVAL;
    if (!(o.mu > 0.0) || !std::isfinite(o.mu)) return UV_EINVAL;
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
    uv_literal *h = new (std::nothrow) uv_literal();
    if (!h) return UV_ENOMEM;
    auto fail = [&](int code) {
        literal_destroy(h);
        return code;
    };
    h->m = A->m;
    h->n = A->n;
    h->nnz = (int)A->nnz;
    h->mu = o.mu;
    h->L_row = pick_l((double)A->nnz / A->m);
    h->L_col = pick_l((double)A->nnz / A->n);
    if (o.hip_stream) h->stream = (hipStream_t)o.hip_stream;
    else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) return fail(UV_EHIP);
        h->own_stream = true;
    }
    const int m = h->m, n = h->n, nnz = h->nnz;
    hipStream_t st = h->stream;
    h->rp = lalloc<int>(h, m + 1);
    h->ci = lalloc<int>(h, nnz);
    h->va = lalloc<double>(h, nnz);
    h->cp = lalloc<int>(h, n + 1);
    h->ri = lalloc<int>(h, nnz);
    h->vc = lalloc<double>(h, nnz);
    h->kcol = lalloc<int>(h, nnz);
    h->b = lalloc<double>(h, m);
    h->c = lalloc<double>(h, n);
    h->fu = lalloc<double>(h, m);
    h->x = lalloc<double>(h, n);
    h->z = lalloc<double>(h, n);
    h->delta = lalloc<double>(h, n);
    h->lam = lalloc<double>(h, m);
    h->y = lalloc<double>(h, nnz);
    h->gam = lalloc<double>(h, nnz);
    int *cnt = lalloc<int>(h, n);
    int *bsum = lalloc<int>(h, blocks_for(n, 4 * kWG));
    for (void *p : {(void *)h->rp, (void *)h->ci, (void *)h->va, (void *)h->cp, (void *)h->ri, (void *)h->vc,
                    (void *)h->kcol, (void *)h->b, (void *)h->c, (void *)h->fu, (void *)h->x, (void *)h->z,
                    (void *)h->delta, (void *)h->lam, (void *)h->y, (void *)h->gam, (void *)cnt, (void *)bsum})
        if (!p) return fail(UV_ENOMEM);
    std::vector<int> rp32(m + 1);
    for (int i = 0; i <= m; ++i) rp32[i] = (int)A->row_ptr[i];
    if (hipMemcpy(h->rp, rp32.data(), 4 * (size_t)(m + 1), hipMemcpyHostToDevice) != hipSuccess) return fail(UV_EHIP);
    if (nnz > 0 && (hipMemcpy(h->ci, A->col_idx, 4 * (size_t)nnz, hipMemcpyHostToDevice) != hipSuccess ||
                    hipMemcpy(h->va, A->val, 8 * (size_t)nnz, hipMemcpyHostToDevice) != hipSuccess))
        return fail(UV_EHIP);
    if (hipMemcpy(h->b, b, 8 * (size_t)m, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->c, c, 8 * (size_t)n, hipMemcpyHostToDevice) != hipSuccess)
        return fail(UV_EHIP);
    if (!build_csc(m, n, nnz, h->rp, h->ci, h->va, h->cp, h->ri, h->vc, cnt, bsum, st)) return fail(UV_EHIP);
    k_lit_kcol<<<blocks_for(n, kWG), kWG, 0, st>>>(n, h->cp, h->ri, h->rp, h->ci, h->kcol);
    k_row_factor<double><<<blocks_for(m, kWG), kWG, 0, st>>>(m, h->rp, h->va, h->fu);
    for (void *p : {(void *)h->x, (void *)h->z, (void *)h->delta})
        if (hipMemsetAsync(p, 0, 8 * (size_t)n, st) != hipSuccess) return fail(UV_EHIP);
    if (hipMemsetAsync(h->lam, 0, 8 * (size_t)m, st) != hipSuccess ||
        hipMemsetAsync(h->y, 0, 8 * (size_t)std::max(nnz, 1), st) != hipSuccess ||
        hipMemsetAsync(h->gam, 0, 8 * (size_t)std::max(nnz, 1), st) != hipSuccess)
        return fail(UV_EHIP);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) return fail(UV_EHIP);
    *out = h;
    return UV_OK;
}

int literal_iterate(uv_literal *h, int64_t k)
{
    if (!h || k < 0) return UV_EINVAL;
    for (int64_t i = 0; i < k; ++i) lit_iteration(h, h->stream);
    if (hipGetLastError() != hipSuccess) return UV_EHIP;
    return hipStreamSynchronize(h->stream) == hipSuccess ? UV_OK : UV_EHIP;
}

int literal_solution(uv_literal *h, double *x, double *z, double *lambda, double *delta, double *y, double *gamma)
{
    if (!h) return UV_EINVAL;
    struct { double *dst; const double *src; size_t len; } cp[] = {
        {x, h->x, (size_t)h->n}, {z, h->z, (size_t)h->n}, {lambda, h->lam, (size_t)h->m},
        {delta, h->delta, (size_t)h->n}, {y, h->y, (size_t)h->nnz}, {gamma, h->gam, (size_t)h->nnz}};
    for (auto &e : cp)
        if (e.dst && e.len && hipMemcpy(e.dst, e.src, 8 * e.len, hipMemcpyDeviceToHost) != hipSuccess) return UV_EHIP;
    return UV_OK;
}

int literal_time(uv_literal *h, int32_t iters, double *ms_col, double *ms_row)
{
    if (!h || iters < 1 || !ms_col || !ms_row) return UV_EINVAL;
    std::vector<hipEvent_t> ev(3 * (size_t)iters, nullptr);
    int rc = UV_OK;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) { rc = UV_EHIP; break; }
    double tc = 0.0, tr = 0.0;
    if (rc == UV_OK) {
        for (int i = 0; i < iters; ++i) {
            (void)hipEventRecord(ev[3 * i], h->stream);
            lit_iteration(h, h->stream, ev[3 * i + 1]);
            (void)hipEventRecord(ev[3 * i + 2], h->stream);
        }
        if (hipStreamSynchronize(h->stream) != hipSuccess) rc = UV_EHIP;
    }
    if (rc == UV_OK) {
        for (int i = 0; i < iters; ++i) {
            float a = 0.f, b = 0.f;
            (void)hipEventElapsedTime(&a, ev[3 * i], ev[3 * i + 1]);
            (void)hipEventElapsedTime(&b, ev[3 * i + 1], ev[3 * i + 2]);
            tc += a;
            tr += b;
        }
        *ms_col = tc / iters;
        *ms_row = tr / iters;
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

}  // extern "C"
