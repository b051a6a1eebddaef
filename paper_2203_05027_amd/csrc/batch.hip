// batch.hip -- many independent problems (orthant cone) solved together by
// one persistent launch.
//
// The instances are packed as one block-diagonal matrix with global row and
// column numbers, so the setup (CSC copy, F_U) is the single-problem setup
// run once.  A workgroup takes the next instance from a queue (instances
// ordered by decreasing nonzero count, so the long ones start first), stages
// its x and u in LDS (the two gathered vectors of the sweep), and runs the
// reduced-form iteration of Algorithm 1 on it -- column pass (A'u, x-step,
// projection, delta update), barrier, row pass (A x, lambda update),
// barrier -- for up to `budget` iterations, checking the FP64 residuals every
// check_every iterations.  A finished instance (converged, max_iter or
// numeric failure) is masked out of later launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/uvadmm.h"
#include "common.hpp"
#include "setup.hpp"

namespace {

constexpr int kMaxThreads = 1024;
constexpr int kLdsMax = 160 * 1024 - 1024;  // LDS of one gfx950 CU less the kernel's static LDS

struct BInst {
    int m, n;
    int row_off, col_off;  // first global row / column of the instance
    int Lr, Lc;            // lanes per row / per column
    int status;
    int ch_off;            // first 64-column slice of the instance (sliced column copy)
    long long iter, check_iter;
    double r_prim, r_dual, r_gap, kkt, pobj, dobj, res_ax_b;
    double bnorm2, cnorm2;
};

template <typename T>
__device__ __forceinline__ T group_sum_rt(T v, int L)
{
    return uv::lane_sum<T>(v, L);
}

// Sum over the workgroup (blockDim.x a multiple of 64), deterministic;
// result in thread 0.
template <int K>
__device__ __forceinline__ void block_sum_rt(double (&v)[K])
{
    __shared__ double s[K][kMaxThreads / 64];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = uv::group_sum<64>(v[k]);
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64, nw = blockDim.x / 64;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) s[k][w] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double t = 0.0;
            for (int i = 0; i < nw; ++i) t += s[k][i];
            v[k] = t;
        }
    }
}

// Instance-local row and column numbers fit 16 bits: x and u of an
// instance must fit in LDS, so m + n < 40,704 in either precision.
typedef unsigned short lidx_t;

// sum over the entries k = beg + lane, beg + lane + L, ... < end of
// val[k] * vs[idx[k]] (idx instance-local): U entries per lane have their
// index and value loads in flight together (the entries are added in the
// same order as one at a time, so the result does not depend on U).
template <int U, typename T, typename TV, typename TS>
__device__ __forceinline__ T seg_sum(int beg, int end, int lane, int L, const lidx_t *__restrict__ idx,
                                     const TV *__restrict__ val, const TS *vs)
{
    T acc = 0;
    for (int k0 = beg + lane; k0 < end; k0 += L * U) {
        int j[U];
        TV v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * L;
            j[u] = 0;
            v[u] = (TV)0;
            if (k < end) {
                j[u] = idx[k];
                v[u] = val[k];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * L < end) acc += (T)v[u] * (T)vs[j[u]];
    }
    return acc;
}

// The same over two vectors at once (the residual check's A z and A x): one
// stream of the entries for both sums.
template <int U, typename TS1, typename TS2>
__device__ __forceinline__ void seg_sum2(int beg, int end, int lane, int L, const lidx_t *__restrict__ idx,
                                         const double *__restrict__ val, const TS1 *vs1, const TS2 *vs2,
                                         double &s1, double &s2)
{
    double a1 = 0.0, a2 = 0.0;
    for (int k0 = beg + lane; k0 < end; k0 += L * U) {
        int j[U];
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u * L;
            j[u] = 0;
            v[u] = 0.0;
            if (k < end) {
                j[u] = idx[k];
                v[u] = val[k];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (k0 + u * L < end) {
                a1 += v[u] * (double)vs1[j[u]];
                a2 += v[u] * (double)vs2[j[u]];
            }
    }
    s1 = a1;
    s2 = a2;
}

// Sliced column copy (lanes per column 0): the columns of an instance are
// cut into slices of 64; slice h stores entry t of its column l at
// s0 + 64 t + l, so lane l's t-th load is one coalesced 64-wide access.  The
// slice is as wide as its longest column; lane l reads only its cnt
// entries, in column order, so the sum is that of one lane per column.
template <int U, typename T, typename TV, typename TS>
__device__ __forceinline__ T sell_sum(int s0, int w, int cnt, int lane, const lidx_t *__restrict__ idx,
                                      const TV *__restrict__ val, const TS *vs)
{
    T acc = 0;
    for (int t0 = 0; t0 < w; t0 += U) {
        int j[U];
        TV v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = s0 + (t0 + u) * 64 + lane;
            j[u] = 0;
            v[u] = (TV)0;
            if (t0 + u < cnt) {
                j[u] = idx[k];
                v[u] = val[k];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (t0 + u < cnt) acc += (T)v[u] * (T)vs[j[u]];
    }
    return acc;
}

// Fills the sliced column copy from the compressed columns, one workgroup
// per instance (slots past a column's end hold zeros).
__global__ void __launch_bounds__(256)
k_sell_fill(const BInst *__restrict__ inst, const int *__restrict__ cp, const int *__restrict__ ri,
            const double *__restrict__ vc, const int *__restrict__ sptr, lidx_t *__restrict__ sidx,
            double *__restrict__ sval)
{
    const BInst &I = inst[blockIdx.x];
    const int nch = (I.n + 63) >> 6;
    for (int p = threadIdx.x; p < nch * 64; p += 256) {
        const int h = p >> 6, l = p & 63, j = p;  // local column j = 64 h + l
        const int s0 = sptr[I.ch_off + h], w = (sptr[I.ch_off + h + 1] - s0) >> 6;
        const int beg = j < I.n ? cp[I.col_off + j] : 0;
        const int len = j < I.n ? cp[I.col_off + j + 1] - beg : 0;
        for (int t = 0; t < w; ++t) {
            const int k = s0 + t * 64 + l;
            sidx[k] = t < len ? (lidx_t)(ri[beg + t] - I.row_off) : (lidx_t)0;
            sval[k] = t < len ? vc[beg + t] : 0.0;
        }
    }
}

// Instance-local copies of the global row (CSC) and column (CSR) numbers,
// one workgroup per instance: its entries are contiguous in both forms.
__global__ void __launch_bounds__(256)
k_local_idx(const BInst *__restrict__ inst, const int *__restrict__ rp, const int *__restrict__ ci,
            const int *__restrict__ cp, const int *__restrict__ ri, lidx_t *__restrict__ cl, lidx_t *__restrict__ rl)
{
    const BInst &I = inst[blockIdx.x];
    for (int k = rp[I.row_off] + threadIdx.x; k < rp[I.row_off + I.m]; k += 256) cl[k] = (lidx_t)(ci[k] - I.col_off);
    for (int k = cp[I.col_off] + threadIdx.x; k < cp[I.col_off + I.n]; k += 256) rl[k] = (lidx_t)(ri[k] - I.row_off);
}

// ||b_i||^2, ||c_i||^2 per instance (one workgroup each).
__global__ void __launch_bounds__(256)
k_batch_norms(BInst *inst, const double *__restrict__ b64, const double *__restrict__ c64)
{
    BInst *I = inst + blockIdx.x;
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < I->m; i += 256) v[0] += b64[I->row_off + i] * b64[I->row_off + i];
    for (int j = threadIdx.x; j < I->n; j += 256) v[1] += c64[I->col_off + j] * c64[I->col_off + j];
    block_sum_rt<2>(v);
    if (threadIdx.x == 0) {
        I->bnorm2 = v[0];
        I->cnorm2 = v[1];
    }
}

__global__ void k_batch_reset(int *queue) { *queue = 0; }

// u = -lambda/mu on one instance's rows (the start mapping).
template <typename T>
__global__ void __launch_bounds__(256)
k_batch_start_u(int r0, int m, const double *__restrict__ lam, T *__restrict__ u, double inv_mu)
{
    int i = blockIdx.x * 256 + threadIdx.x;
    if (i < m) u[r0 + i] = (T)(-lam[r0 + i] * inv_mu);
}

template <typename T, bool ZC>
__global__ void __launch_bounds__(kMaxThreads)
k_batch(BInst *__restrict__ inst, const int *__restrict__ order, int nq, int *__restrict__ queue,
        const int *__restrict__ budget_p, const int *__restrict__ rp, const lidx_t *__restrict__ cl,
        const T *__restrict__ va, const double *__restrict__ va64, const int *__restrict__ cp,
        const lidx_t *__restrict__ rl, const T *__restrict__ vc, const double *__restrict__ vc64,
        const T *__restrict__ b, const double *__restrict__ b64, const T *__restrict__ fu,
        const T *__restrict__ c, const double *__restrict__ c64, T *__restrict__ x, T *__restrict__ z,
        T *__restrict__ u, double *__restrict__ lam, double *__restrict__ delta, double mu, double inv_mu,
        double eps, int check_every, long long max_iter, const int *__restrict__ sptr,
        const lidx_t *__restrict__ sidx, const T *__restrict__ sval, const double *__restrict__ sval64, int gated)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    T *xs = reinterpret_cast<T *>(lds_raw);
    __shared__ int s_q, s_stop, s_skip;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int budget = *budget_p;
    for (;;) {
        if (tid == 0) s_q = atomicAdd(queue, 1);
        __syncthreads();
        const int q = s_q;
        __syncthreads();  // every thread has read s_q before it is reused
        if (q >= nq) return;
        BInst *I = inst + order[q];
        if (I->status != UV_STATUS_RUNNING) continue;
        const int m = I->m, n = I->n, r0 = I->row_off, c0 = I->col_off;
        const int Lr = I->Lr, Lc = I->Lc;
        long long it = I->iter;
        T *us = xs + n;
        // ZC: z and c of the instance in LDS as well (after u), so the column
        // pass streams only delta and the entries
        T *zi = ZC ? us + m : z + c0;
        const T *ci_ = ZC ? us + m + n : c + c0;
        for (int j = tid; j < n; j += nthr) xs[j] = x[c0 + j];
        for (int i = tid; i < m; i += nthr) us[i] = u[r0 + i];
        if (ZC)
            for (int j = tid; j < n; j += nthr) {
                zi[j] = z[c0 + j];
                us[m + n + j] = c[c0 + j];
            }
        __syncthreads();
        // lane groups per column (Lc > 0) or the sliced copy (Lc == 0: a wavefront per 64 columns)
        const int Lc1 = Lc > 0 ? Lc : 1;
        const int gc = tid / Lc1, lc = tid % Lc1, Gc = nthr / Lc1;
        const int wv = tid >> 6, lane64 = tid & 63, nwv = nthr >> 6, nch = (n + 63) >> 6, ch0 = I->ch_off;
        const int gr = tid / Lr, lr = tid % Lr, Gr = nthr / Lr;
        int stop = 0;
        for (int k = 0; k < budget && !stop; ++k) {
            // column pass: p = N x + A'u, x-step, projection onto R_+, delta
            auto col_update = [&](int j, int cnt, T atu, double d, T zj, T cj) {
                const T dm = (T)(d * inv_mu);
                const T p = (T)cnt * xs[j] + atu;
                const T xn = (p + zj + dm - cj * (T)inv_mu) / (T)(1 + cnt);
                const T v = xn - dm;
                const T zn = v > (T)0 ? v : (T)0;
                xs[j] = xn;
                zi[j] = zn;
                delta[c0 + j] = d + mu * ((double)zn - (double)xn);
            };
            if (Lc == 0) {
                for (int h = wv; h < nch; h += nwv) {
                    const int j = (h << 6) + lane64;
                    T zj = 0, cj = 0;
                    double d = 0.0;
                    int cnt = 0;
                    if (j < n) {  // the update's own loads, in flight with the sum's
                        d = delta[c0 + j];
                        zj = zi[j];
                        cj = ci_[j];
                        cnt = cp[c0 + j + 1] - cp[c0 + j];
                    }
                    const int s0 = sptr[ch0 + h], w = (sptr[ch0 + h + 1] - s0) >> 6;
                    const T atu = sell_sum<4, T>(s0, w, cnt, lane64, sidx, sval, us);
                    if (j < n) col_update(j, cnt, atu, d, zj, cj);
                }
            } else
            for (int jb = 0; jb < n; jb += Gc) {
                const int j = jb + gc;
                T atu = 0, zj = 0, cj = 0;
                double d = 0.0;
                int beg = 0, end = 0;
                if (j < n) {
                    beg = cp[c0 + j];
                    end = cp[c0 + j + 1];
                    if (lc == 0) {  // the update's own loads, in flight with the sum's
                        d = delta[c0 + j];
                        zj = zi[j];
                        cj = ci_[j];
                    }
                    atu = seg_sum<4, T>(beg, end, lc, Lc, rl, vc, us);
                }
                atu = group_sum_rt(atu, Lc);
                if (j < n && lc == 0) col_update(j, end - beg, atu, d, zj, cj);
            }
            __syncthreads();
            // row pass: q = A x, lambda update, u.  At a check iteration the
            // row pass forms A x and A z in FP64 with the FP64 values of A
            // (the check's row sums) and the iteration takes its q from that
            // A x, so the check adds no second row product.
            const bool chk = (it + 1) % check_every == 0 || (max_iter > 0 && it + 1 >= max_iter);
            double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            for (int ib = 0; ib < m; ib += Gr) {
                const int i = ib + gr;
                T q = 0, fi = 0, bi = 0;
                double l0 = 0.0, qz = 0.0, qx = 0.0;
                if (i < m) {
                    const int beg = rp[r0 + i], end = rp[r0 + i + 1];
                    if (lr == 0) {
                        fi = fu[r0 + i];
                        bi = b[r0 + i];
                        l0 = lam[r0 + i];
                    }
                    if (chk) seg_sum2<4>(beg, end, lr, Lr, cl, va64, zi, xs, qz, qx);
                    else q = seg_sum<4, T>(beg, end, lr, Lr, cl, va, xs);
                }
                if (chk) {
                    qz = group_sum_rt(qz, Lr);
                    qx = group_sum_rt(qx, Lr);
                    q = (T)qx;
                } else {
                    q = group_sum_rt(q, Lr);
                }
                if (i < m && lr == 0) {
                    const T e = fi * (bi - q);
                    const double li = l0 - mu * (double)e;
                    lam[r0 + i] = li;
                    us[i] = (T)((double)e - li * inv_mu);
                    if (chk) {
                        const double bd = b64[r0 + i];
                        a[0] += (qz - bd) * (qz - bd);
                        a[1] += bd * li;
                        a[2] += (qx - bd) * (qx - bd);
                    }
                }
            }
            __syncthreads();
            ++it;
            if (chk && gated && !(max_iter > 0 && it >= max_iter)) {
                // primal half first: when r_prim > eps (with finite row sums)
                // this check cannot stop the instance, and its column half is
                // skipped (the row sums are reduced as below, bit for bit)
                double g[3] = {a[0], a[1], a[2]};
                block_sum_rt<3>(g);
                if (tid == 0)
                    s_skip = !(sqrt(g[0]) / (1.0 + sqrt(I->bnorm2)) <= eps) && isfinite(g[0]) && isfinite(g[1]) &&
                             isfinite(g[2]);
                __syncthreads();
                if (s_skip) continue;
            }
            if (chk) {
                // FP64 residuals at (z, lambda, delta) with the FP64 values of A:
                // the row sums came with the row pass, the column sums here
                auto col_res = [&](int j, double atl) {
                    const double r = atl + c64[c0 + j] - delta[c0 + j];
                    a[3] += r * r;
                    a[4] += c64[c0 + j] * (double)zi[j];
                };
                if (Lc == 0) {
                    for (int h = wv; h < nch; h += nwv) {
                        const int j = (h << 6) + lane64;
                        const int cnt = j < n ? cp[c0 + j + 1] - cp[c0 + j] : 0;
                        const int s0 = sptr[ch0 + h], w = (sptr[ch0 + h + 1] - s0) >> 6;
                        const double atl = sell_sum<4, double>(s0, w, cnt, lane64, sidx, sval64, lam + r0);
                        if (j < n) col_res(j, atl);
                    }
                } else
                for (int jb = 0; jb < n; jb += Gc) {
                    const int j = jb + gc;
                    double atl = 0.0;
                    if (j < n) atl = seg_sum<4, double>(cp[c0 + j], cp[c0 + j + 1], lc, Lc, rl, vc64, lam + r0);
                    atl = group_sum_rt(atl, Lc);
                    if (j < n && lc == 0) col_res(j, atl);
                }
                block_sum_rt<5>(a);
                if (tid == 0) {
                    const double rpr = sqrt(a[0]) / (1.0 + sqrt(I->bnorm2));
                    const double rdu = sqrt(a[3]) / (1.0 + sqrt(I->cnorm2));
                    const double cz = a[4], bl = a[1];
                    const double rg = fabs(cz + bl) / (1.0 + fabs(cz) + fabs(bl));
                    const double kkt = uv::kkt_of(rpr, rdu, rg);
                    I->r_prim = rpr;
                    I->r_dual = rdu;
                    I->r_gap = rg;
                    I->kkt = kkt;
                    I->pobj = cz;
                    I->dobj = -bl;
                    I->res_ax_b = sqrt(a[2]);
                    I->check_iter = it;
                    int st = UV_STATUS_RUNNING;
                    if (!isfinite(kkt)) st = UV_STATUS_NUMERIC;
                    else if (kkt <= eps) st = UV_STATUS_CONVERGED;
                    else if (max_iter > 0 && it >= max_iter) st = UV_STATUS_MAX_ITER;
                    I->status = st;
                    s_stop = st != UV_STATUS_RUNNING;
                }
                __syncthreads();
                stop = s_stop;
            }
        }
        for (int j = tid; j < n; j += nthr) x[c0 + j] = xs[j];
        if (ZC)
            for (int j = tid; j < n; j += nthr) z[c0 + j] = zi[j];
        for (int i = tid; i < m; i += nthr) u[r0 + i] = us[i];
        if (tid == 0) I->iter = it;
        __syncthreads();  // LDS is reused by the next instance
    }
}

inline int bucket_of(int m) { return m < 128 ? 0 : m < 512 ? 1 : m < 2048 ? 2 : 3; }

}  // namespace

struct uv_batch {
    int count = 0;
    int M = 0, N = 0;  // total rows / columns
    int nnz = 0;
    uv_opts o{};
    hipStream_t stream = nullptr, cap = nullptr;
    bool own_stream = false;
    std::vector<void *> allocs;
    int *rp = nullptr, *ci = nullptr, *cp = nullptr, *ri = nullptr;
    lidx_t *cl = nullptr, *rl = nullptr;  // instance-local column (CSR) and row (CSC) numbers
    // sliced column copy: slice offsets (64 slots per unit of width), local rows, values
    int *sptr = nullptr;
    lidx_t *sidx = nullptr;
    double *sval64 = nullptr;
    void *sval = nullptr;
    double *va64 = nullptr, *vc64 = nullptr, *b64 = nullptr, *c64 = nullptr;
    void *va = nullptr, *vc = nullptr, *b = nullptr, *c = nullptr, *fu = nullptr;
    void *x = nullptr, *z = nullptr, *u = nullptr;
    double *lam = nullptr, *delta = nullptr, *scratch = nullptr;
    BInst *inst = nullptr;
    BInst *inst_host = nullptr;  // pinned mirror
    int *order = nullptr, *queue = nullptr, *budget = nullptr;
    int *budget_host = nullptr;  // pinned
    std::vector<int> order_host;
    int threads = 256;
    int xu_bytes = 0;   // x and u of the largest instance (16-byte aligned)
    int zc_bytes = 0;   // x, u, z and c of the largest instance
    bool zc = false;    // z and c staged in LDS too
    int lds_bytes = 0;  // dynamic LDS per workgroup of the launch
    int grid = 0;
    int tiles[2 * 4] = {2, 1, 2, 1, 2, 1, 2, 1};  // (Lr, Lc) per size bucket
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

template <typename T>
T *balloc(uv_batch *h, size_t count)
{
    void *p = nullptr;
    if (uv::dev_malloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return nullptr;
    h->allocs.push_back(p);
    return (T *)p;
}

#define UV_BTRY(expr)                              \
    do {                                           \
        if ((expr) != hipSuccess) return UV_EHIP;  \
    } while (0)

int batch_launch(uv_batch *h, hipStream_t st, const int *order, int nq)
{
    k_batch_reset<<<1, 1, 0, st>>>(h->queue);
    const uv_opts &o = h->o;
    const double mu = o.mu, im = 1.0 / o.mu;
#define UV_BATCH_ARGS(T)                                                                                     \
    h->inst, order, nq, h->queue, h->budget, h->rp, h->cl, (const T *)h->va, h->va64, h->cp, h->rl,          \
        (const T *)h->vc, h->vc64, (const T *)h->b, h->b64, (const T *)h->fu, (const T *)h->c, h->c64,      \
        (T *)h->x, (T *)h->z, (T *)h->u, h->lam, h->delta, mu, im, o.eps_kkt, o.check_every, (long long)o.max_iter, \
        h->sptr, h->sidx, (const T *)h->sval, h->sval64, o.full_checks == 0 ? 1 : 0
    const int grid = std::max(1, std::min(h->grid, nq));
    if (o.precision == UV_MIXED)
        h->zc ? k_batch<float, true><<<grid, h->threads, h->lds_bytes, st>>>(UV_BATCH_ARGS(float))
              : k_batch<float, false><<<grid, h->threads, h->lds_bytes, st>>>(UV_BATCH_ARGS(float));
    else
        h->zc ? k_batch<double, true><<<grid, h->threads, h->lds_bytes, st>>>(UV_BATCH_ARGS(double))
              : k_batch<double, false><<<grid, h->threads, h->lds_bytes, st>>>(UV_BATCH_ARGS(double));
#undef UV_BATCH_ARGS
    return hipGetLastError() == hipSuccess ? UV_OK : UV_EHIP;
}

// The sliced column copy (lanes per column 0): slices of 64 columns, each as
// wide as its longest column, filled on the device from the compressed
// columns.  Needs the instances' col_off / n on the host and cp on the
// device; sets every instance's ch_off.
int build_slices(uv_batch *h)
{
    const bool mixed = h->o.precision == UV_MIXED;
    std::vector<int> cph((size_t)h->N + 1);
    UV_BTRY(hipMemcpy(cph.data(), h->cp, sizeof(int) * cph.size(), hipMemcpyDeviceToHost));
    std::vector<int> sptr(1, 0);
    int64_t slots = 0;
    for (int i = 0; i < h->count; ++i) {
        BInst &I = h->inst_host[i];
        I.ch_off = (int)sptr.size() - 1;
        for (int j0 = 0; j0 < I.n; j0 += 64) {
            int w = 0;
            for (int j = j0; j < std::min(j0 + 64, I.n); ++j)
                w = std::max(w, cph[(size_t)I.col_off + j + 1] - cph[(size_t)I.col_off + j]);
            slots += 64 * (int64_t)w;
            if (slots >= ((int64_t)1 << 31)) return UV_ETOOBIG;
            sptr.push_back((int)slots);
        }
    }
    h->sptr = balloc<int>(h, sptr.size());
    h->sidx = balloc<lidx_t>(h, slots);
    h->sval64 = balloc<double>(h, slots);
    h->sval = mixed ? (void *)balloc<float>(h, slots) : (void *)h->sval64;
    if (!h->sptr || !h->sidx || !h->sval64 || !h->sval) return UV_ENOMEM;
    UV_BTRY(hipMemcpy(h->sptr, sptr.data(), sizeof(int) * sptr.size(), hipMemcpyHostToDevice));
    UV_BTRY(hipMemcpy(h->inst, h->inst_host, sizeof(BInst) * h->count, hipMemcpyHostToDevice));
    hipStream_t st = h->stream;
    k_sell_fill<<<h->count, 256, 0, st>>>(h->inst, h->cp, h->ri, h->vc64, h->sptr, h->sidx, h->sval64);
    if (mixed && slots > 0)
        k_narrow<float><<<blocks_for(slots, kWG), kWG, 0, st>>>(slots, h->sval64, (float *)h->sval);
    UV_BTRY(hipGetLastError());
    UV_BTRY(hipStreamSynchronize(st));
    return UV_OK;
}

int apply_tiles(uv_batch *h)
{
    // lanes per row / column from the tile table, by size bucket
    for (int i = 0; i < h->count; ++i) {
        const int bk = bucket_of(h->inst_host[i].m);
        h->inst_host[i].Lr = h->tiles[2 * bk];
        h->inst_host[i].Lc = h->tiles[2 * bk + 1];
    }
    UV_BTRY(hipMemcpyAsync(h->inst, h->inst_host, sizeof(BInst) * h->count, hipMemcpyHostToDevice, h->stream));
    UV_BTRY(hipStreamSynchronize(h->stream));
    return UV_OK;
}

template <typename T, bool ZC>
int occupancy_of(uv_batch *h, int *per_cu)
{
    // LDS above the default 64 KiB per workgroup has to be asked for
    if (h->lds_bytes > 64 * 1024 &&
        hipFuncSetAttribute((const void *)k_batch<T, ZC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            h->lds_bytes) != hipSuccess)
        return UV_ETOOBIG;
    UV_BTRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, k_batch<T, ZC>, h->threads, h->lds_bytes));
    return UV_OK;
}

// LDS per workgroup (x and u of the largest instance, and z and c too when
// every instance's fit: ZC) and the persistent grid the occupancy allows.
int occupancy_grid(uv_batch *h)
{
    h->zc = h->zc_bytes <= kLdsMax;
    h->lds_bytes = h->zc ? h->zc_bytes : h->xu_bytes;
    int dev = 0, cus = 0;
    UV_BTRY(hipGetDevice(&dev));
    UV_BTRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int per_cu = 0, rc;
    if (h->o.precision == UV_MIXED)
        rc = h->zc ? occupancy_of<float, true>(h, &per_cu) : occupancy_of<float, false>(h, &per_cu);
    else
        rc = h->zc ? occupancy_of<double, true>(h, &per_cu) : occupancy_of<double, false>(h, &per_cu);
    if (rc != UV_OK) return rc;
    h->grid = std::max(1, per_cu) * cus;
    return UV_OK;
}

int rebuild_graph(uv_batch *h)
{
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->exec = nullptr;
    h->graph = nullptr;
    if (!h->o.use_graph) return UV_OK;
    if (hipStreamBeginCapture(h->cap, hipStreamCaptureModeRelaxed) != hipSuccess) return UV_EHIP;
    int rc = batch_launch(h, h->cap, h->order, h->count);
    if (hipStreamEndCapture(h->cap, &h->graph) != hipSuccess || rc != UV_OK) return UV_EHIP;
    if (hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0) != hipSuccess) return UV_EHIP;
    return UV_OK;
}

}  // namespace

extern "C" {

void batch_destroy(uv_batch *h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    for (void *p : h->allocs) (void)hipFree(p);
    if (h->inst_host) (void)hipHostFree(h->inst_host);
    if (h->budget_host) (void)hipHostFree(h->budget_host);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

int batch_create(int32_t count, const uv_csr *A, const double *const *b, const double *const *c,
                 const uv_opts *opts, uv_batch **out)
{
    if (!out) return UV_EINVAL;
    *out = nullptr;
    if (count < 1 || !A || !b || !c) return UV_EINVAL;
    uv_opts o;
    uv_default_opts(&o);
    if (opts) o = *opts;
    if (!(o.mu > 0.0) || !std::isfinite(o.mu) || o.check_every < 1 || !(o.eps_kkt >= 0.0) || o.max_iter < 0 ||
        (o.precision != UV_FP64 && o.precision != UV_MIXED) || o.full_checks < 0 || o.full_checks > 1)
        return UV_EINVAL;
    const size_t ts = o.precision == UV_MIXED ? 4 : 8;
    int64_t M = 0, N = 0, NNZ = 0;
    size_t lds = 0, lds_zc = 0;
    for (int i = 0; i < count; ++i) {
        const uv_csr &a = A[i];
        if (!b[i] || !c[i] || !a.row_ptr || a.m < 1 || a.n < 1 || a.nnz < 0) return UV_EINVAL;
        if (a.nnz > 0 && (!a.col_idx || !a.val)) return UV_EINVAL;
        if (a.row_ptr[0] != 0 || a.row_ptr[a.m] != a.nnz) return UV_EBADCSR;
        for (int32_t r = 0; r < a.m; ++r) {
            const int64_t b0 = a.row_ptr[r], b1 = a.row_ptr[r + 1];
            if (b1 < b0 || b1 > a.nnz) return UV_EBADCSR;
            for (int64_t k = b0; k < b1; ++k) {
                if (a.col_idx[k] < 0 || a.col_idx[k] >= a.n) return UV_EBADCSR;
                if (k > b0 && a.col_idx[k] <= a.col_idx[k - 1]) return UV_EBADCSR;
            }
        }
        M += a.m;
        N += a.n;
        NNZ += a.nnz;
        lds = std::max(lds, (size_t)(a.m + a.n) * ts);
        lds_zc = std::max(lds_zc, (size_t)(a.m + 3 * (size_t)a.n) * ts);
    }
    if (NNZ >= ((int64_t)1 << 31) || M >= ((int64_t)1 << 31) || N >= ((int64_t)1 << 31)) return UV_ETOOBIG;
    if (lds > (size_t)kLdsMax) return UV_ETOOBIG;  // x and u of every instance must fit in LDS

    uv_batch *h = new (std::nothrow) uv_batch();
    if (!h) return UV_ENOMEM;
    h->count = count;
    h->M = (int)M;
    h->N = (int)N;
    h->nnz = (int)NNZ;
    h->o = o;
    h->xu_bytes = (int)((lds + 15) / 16 * 16);
    h->zc_bytes = (int)std::min<size_t>((lds_zc + 15) / 16 * 16, (size_t)1 << 30);
    h->lds_bytes = h->xu_bytes;
    int rc = UV_OK;
    auto fail = [&](int code) {
        batch_destroy(h);
        return code;
    };
    if (o.hip_stream) h->stream = (hipStream_t)o.hip_stream;
    else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) return fail(UV_EHIP);
        h->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess) return fail(UV_EHIP);
    hipStream_t st = h->stream;
    const bool mixed = o.precision == UV_MIXED;

    h->rp = balloc<int>(h, M + 1);
    h->ci = balloc<int>(h, NNZ);
    h->va64 = balloc<double>(h, NNZ);
    h->cp = balloc<int>(h, N + 1);
    h->ri = balloc<int>(h, NNZ);
    h->vc64 = balloc<double>(h, NNZ);
    h->cl = balloc<lidx_t>(h, NNZ);
    h->rl = balloc<lidx_t>(h, NNZ);
    h->b64 = balloc<double>(h, M);
    h->c64 = balloc<double>(h, N);
    h->lam = balloc<double>(h, M);
    h->delta = balloc<double>(h, N);
    h->scratch = balloc<double>(h, std::max(M, N));
    h->x = balloc<char>(h, ts * N);
    h->z = balloc<char>(h, ts * N);
    h->u = balloc<char>(h, ts * M);
    h->fu = balloc<char>(h, ts * M);
    if (mixed) {
        h->va = balloc<float>(h, NNZ);
        h->vc = balloc<float>(h, NNZ);
        h->b = balloc<float>(h, M);
        h->c = balloc<float>(h, N);
    } else {
        h->va = h->va64;
        h->vc = h->vc64;
        h->b = h->b64;
        h->c = h->c64;
    }
    h->inst = balloc<BInst>(h, count);
    h->order = balloc<int>(h, count);
    h->queue = balloc<int>(h, 1);
    h->budget = balloc<int>(h, 1);
    int *cnt = balloc<int>(h, N);
    int *bsum = balloc<int>(h, blocks_for(N, 4 * kWG));
    for (void *p : {(void *)h->rp, (void *)h->ci, (void *)h->va64, (void *)h->cp, (void *)h->ri, (void *)h->vc64, (void *)h->cl, (void *)h->rl,
                    (void *)h->b64, (void *)h->c64, (void *)h->lam, (void *)h->delta, (void *)h->scratch, h->x,
                    h->z, h->u, h->fu, h->va, h->vc, h->b, h->c, (void *)h->inst, (void *)h->order,
                    (void *)h->queue, (void *)h->budget, (void *)cnt, (void *)bsum})
        if (!p) return fail(UV_ENOMEM);
    if (uv::host_malloc(&h->inst_host, sizeof(BInst) * count, hipHostMallocDefault) != hipSuccess) {
        h->inst_host = nullptr;
        return fail(UV_ENOMEM);
    }
    if (uv::host_malloc(&h->budget_host, sizeof(int), hipHostMallocDefault) != hipSuccess) {
        h->budget_host = nullptr;
        return fail(UV_ENOMEM);
    }

    // Pack the block-diagonal matrix with global indices.
    {
        std::vector<int> rp32(M + 1), ci32(NNZ);
        std::vector<double> va(NNZ), bb(M), cc(N);
        int64_t ro = 0, co = 0, ko = 0;
        for (int i = 0; i < count; ++i) {
            const uv_csr &a = A[i];
            BInst &I = h->inst_host[i];
            std::memset(&I, 0, sizeof(I));
            I.m = a.m;
            I.n = a.n;
            I.row_off = (int)ro;
            I.col_off = (int)co;
            I.status = UV_STATUS_RUNNING;
            I.check_iter = -1;
            for (int r = 0; r < a.m; ++r) rp32[ro + r] = (int)(ko + a.row_ptr[r]);
            for (int64_t k = 0; k < a.nnz; ++k) {
                ci32[ko + k] = (int)(co + a.col_idx[k]);
                va[ko + k] = a.val[k];
            }
            std::memcpy(&bb[ro], b[i], sizeof(double) * a.m);
            std::memcpy(&cc[co], c[i], sizeof(double) * a.n);
            ro += a.m;
            co += a.n;
            ko += a.nnz;
        }
        rp32[M] = (int)NNZ;
        if (hipMemcpy(h->rp, rp32.data(), sizeof(int) * (M + 1), hipMemcpyHostToDevice) != hipSuccess) return fail(UV_EHIP);
        if (NNZ > 0) {
            if (hipMemcpy(h->ci, ci32.data(), sizeof(int) * NNZ, hipMemcpyHostToDevice) != hipSuccess) return fail(UV_EHIP);
            if (hipMemcpy(h->va64, va.data(), sizeof(double) * NNZ, hipMemcpyHostToDevice) != hipSuccess) return fail(UV_EHIP);
        }
        if (hipMemcpy(h->b64, bb.data(), sizeof(double) * M, hipMemcpyHostToDevice) != hipSuccess) return fail(UV_EHIP);
        if (hipMemcpy(h->c64, cc.data(), sizeof(double) * N, hipMemcpyHostToDevice) != hipSuccess) return fail(UV_EHIP);
    }
    // Longest instances first.
    h->order_host.resize(count);
    std::iota(h->order_host.begin(), h->order_host.end(), 0);
    std::stable_sort(h->order_host.begin(), h->order_host.end(), [&](int p, int q) {
        return A[p].nnz + A[p].m + A[p].n > A[q].nnz + A[q].m + A[q].n;
    });
    if (hipMemcpy(h->order, h->order_host.data(), sizeof(int) * count, hipMemcpyHostToDevice) != hipSuccess) return fail(UV_EHIP);

    if (!build_csc((int)M, (int)N, (int)NNZ, h->rp, h->ci, h->va64, h->cp, h->ri, h->vc64, cnt, bsum, st))
        return fail(UV_EHIP);
    if (mixed) {
        k_row_factor<float><<<blocks_for(M, kWG), kWG, 0, st>>>((int)M, h->rp, h->va64, (float *)h->fu);
        if (NNZ > 0) {
            k_narrow<float><<<blocks_for(NNZ, kWG), kWG, 0, st>>>(NNZ, h->va64, (float *)h->va);
            k_narrow<float><<<blocks_for(NNZ, kWG), kWG, 0, st>>>(NNZ, h->vc64, (float *)h->vc);
        }
        k_narrow<float><<<blocks_for(M, kWG), kWG, 0, st>>>(M, h->b64, (float *)h->b);
        k_narrow<float><<<blocks_for(N, kWG), kWG, 0, st>>>(N, h->c64, (float *)h->c);
    } else {
        k_row_factor<double><<<blocks_for(M, kWG), kWG, 0, st>>>((int)M, h->rp, h->va64, (double *)h->fu);
    }
    // zero start
    if (hipMemsetAsync(h->x, 0, ts * N, st) != hipSuccess || hipMemsetAsync(h->z, 0, ts * N, st) != hipSuccess ||
        hipMemsetAsync(h->u, 0, ts * M, st) != hipSuccess || hipMemsetAsync(h->lam, 0, 8 * M, st) != hipSuccess ||
        hipMemsetAsync(h->delta, 0, 8 * N, st) != hipSuccess)
        return fail(UV_EHIP);
    if (hipMemcpyAsync(h->inst, h->inst_host, sizeof(BInst) * count, hipMemcpyHostToDevice, st) != hipSuccess)
        return fail(UV_EHIP);
    k_batch_norms<<<count, 256, 0, st>>>(h->inst, h->b64, h->c64);
    k_local_idx<<<count, 256, 0, st>>>(h->inst, h->rp, h->ci, h->cp, h->ri, h->cl, h->rl);
    if (hipGetLastError() != hipSuccess) return fail(UV_EHIP);
    if (hipMemcpyAsync(h->inst_host, h->inst, sizeof(BInst) * count, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return fail(UV_EHIP);
    if ((rc = build_slices(h)) != UV_OK) return fail(rc);
    if ((rc = apply_tiles(h)) != UV_OK) return fail(rc);
    if ((rc = occupancy_grid(h)) != UV_OK) return fail(rc);
    if ((rc = rebuild_graph(h)) != UV_OK) return fail(rc);
    *out = h;
    return UV_OK;
}

int batch_set_tiles(uv_batch *h, int32_t threads, const int32_t *lanes)
{
    if (!h || !lanes) return UV_EINVAL;
    if (threads != 64 && threads != 128 && threads != 256 && threads != 512 && threads != 1024) return UV_EINVAL;
    for (int k = 0; k < 8; ++k) {
        const int lo = k % 2 ? 0 : 1;  // lanes per row >= 1; lanes per column >= 0 (0: sliced copy)
        if (lanes[k] < lo || lanes[k] > 64 || (lanes[k] & (lanes[k] - 1)) || lanes[k] > threads) return UV_EINVAL;
    }
    UV_BTRY(hipStreamSynchronize(h->stream));
    UV_BTRY(hipMemcpy(h->inst_host, h->inst, sizeof(BInst) * h->count, hipMemcpyDeviceToHost));
    h->threads = threads;
    std::memcpy(h->tiles, lanes, sizeof(h->tiles));
    int rc;
    if ((rc = apply_tiles(h)) != UV_OK) return rc;
    if ((rc = occupancy_grid(h)) != UV_OK) return rc;
    return rebuild_graph(h);
}

int batch_get_tiles(const uv_batch *h, int32_t *threads, int32_t *lanes)
{
    if (!h) return UV_EINVAL;
    if (threads) *threads = h->threads;
    if (lanes) std::memcpy(lanes, h->tiles, sizeof(h->tiles));
    return UV_OK;
}

int batch_iterate(uv_batch *h, int64_t k, int32_t *n_active)
{
    if (!h || k < 0) return UV_EINVAL;
    int64_t left = k;
    while (left > 0) {
        const int step = (int)std::min<int64_t>(left, 1 << 30);
        *h->budget_host = step;
        UV_BTRY(hipMemcpyAsync(h->budget, h->budget_host, sizeof(int), hipMemcpyHostToDevice, h->stream));
        if (h->exec) UV_BTRY(hipGraphLaunch(h->exec, h->stream));
        else {
            int rc = batch_launch(h, h->stream, h->order, h->count);
            if (rc != UV_OK) return rc;
        }
        left -= step;
    }
    UV_BTRY(hipMemcpyAsync(h->inst_host, h->inst, sizeof(BInst) * h->count, hipMemcpyDeviceToHost, h->stream));
    UV_BTRY(hipStreamSynchronize(h->stream));
    if (n_active) {
        int a = 0;
        for (int i = 0; i < h->count; ++i) a += h->inst_host[i].status == UV_STATUS_RUNNING;
        *n_active = a;
    }
    return UV_OK;
}

int batch_residuals(uv_batch *h, int32_t i, uv_residuals *r)
{
    if (!h || !r || i < 0 || i >= h->count) return UV_EINVAL;
    const BInst &I = h->inst_host[i];
    r->r_prim = I.r_prim;
    r->r_dual = I.r_dual;
    r->r_gap = I.r_gap;
    r->kkt = I.kkt;
    r->pobj = I.pobj;
    r->dobj = I.dobj;
    r->res_ax_b = I.res_ax_b;
    r->prim_inf = r->dual_inf = r->scale_p = r->scale_d = 0.0;
    r->pobj_x = r->gap_x = 0.0;
    r->iter = I.iter;
    r->status = I.status;
    return I.status == UV_STATUS_NUMERIC ? UV_ENUMERIC : UV_OK;
}

int batch_solution(uv_batch *h, int32_t i, double *x, double *z, double *lambda, double *delta)
{
    if (!h || i < 0 || i >= h->count) return UV_EINVAL;
    const BInst &I = h->inst_host[i];
    hipStream_t st = h->stream;
    const bool mixed = h->o.precision == UV_MIXED;
    auto get_t = [&](double *dst, void *src, int off, int len) -> int {
        if (!dst) return UV_OK;
        const void *from;
        if (mixed) {
            k_widen<float><<<blocks_for(len, kWG), kWG, 0, st>>>(len, (const float *)src + off, h->scratch);
            from = h->scratch;
        } else {
            from = (const double *)src + off;
        }
        if (hipMemcpyAsync(dst, from, 8 * (size_t)len, hipMemcpyDeviceToHost, st) != hipSuccess) return UV_EHIP;
        return hipStreamSynchronize(st) == hipSuccess ? UV_OK : UV_EHIP;
    };
    int rc;
    if ((rc = get_t(x, h->x, I.col_off, I.n)) != UV_OK) return rc;
    if ((rc = get_t(z, h->z, I.col_off, I.n)) != UV_OK) return rc;
    if (lambda) UV_BTRY(hipMemcpyAsync(lambda, h->lam + I.row_off, 8 * (size_t)I.m, hipMemcpyDeviceToHost, st));
    if (delta) UV_BTRY(hipMemcpyAsync(delta, h->delta + I.col_off, 8 * (size_t)I.n, hipMemcpyDeviceToHost, st));
    UV_BTRY(hipStreamSynchronize(st));
    return UV_OK;
}

int batch_set_start(uv_batch *h, int32_t i, const double *x, const double *z, const double *delta,
                    const double *lambda)
{
    if (!h || i < 0 || i >= h->count) return UV_EINVAL;
    BInst &I = h->inst_host[i];
    hipStream_t st = h->stream;
    const bool mixed = h->o.precision == UV_MIXED;
    const size_t ts = mixed ? 4 : 8;
    auto put_t = [&](void *dst, const double *src, int off, int len) -> int {
        char *d = (char *)dst + ts * off;
        if (!src) return hipMemsetAsync(d, 0, ts * len, st) == hipSuccess ? UV_OK : UV_EHIP;
        if (!mixed) return hipMemcpyAsync(d, src, 8 * (size_t)len, hipMemcpyHostToDevice, st) == hipSuccess
                               ? UV_OK : UV_EHIP;
        if (hipMemcpyAsync(h->scratch, src, 8 * (size_t)len, hipMemcpyHostToDevice, st) != hipSuccess)
            return UV_EHIP;
        k_narrow<float><<<blocks_for(len, kWG), kWG, 0, st>>>(len, h->scratch, (float *)d);
        return hipStreamSynchronize(st) == hipSuccess ? UV_OK : UV_EHIP;
    };
    int rc;
    if ((rc = put_t(h->x, x, I.col_off, I.n)) != UV_OK) return rc;
    if ((rc = put_t(h->z, z, I.col_off, I.n)) != UV_OK) return rc;
    if (delta) UV_BTRY(hipMemcpyAsync(h->delta + I.col_off, delta, 8 * (size_t)I.n, hipMemcpyHostToDevice, st));
    else UV_BTRY(hipMemsetAsync(h->delta + I.col_off, 0, 8 * (size_t)I.n, st));
    if (lambda) UV_BTRY(hipMemcpyAsync(h->lam + I.row_off, lambda, 8 * (size_t)I.m, hipMemcpyHostToDevice, st));
    else UV_BTRY(hipMemsetAsync(h->lam + I.row_off, 0, 8 * (size_t)I.m, st));
    const double im = 1.0 / h->o.mu;
    if (mixed) k_batch_start_u<float><<<blocks_for(I.m, 256), 256, 0, st>>>(I.row_off, I.m, h->lam, (float *)h->u, im);
    else k_batch_start_u<double><<<blocks_for(I.m, 256), 256, 0, st>>>(I.row_off, I.m, h->lam, (double *)h->u, im);
    UV_BTRY(hipGetLastError());
    I.iter = 0;
    I.check_iter = -1;
    I.status = UV_STATUS_RUNNING;
    UV_BTRY(hipMemcpyAsync(h->inst + i, &I, sizeof(BInst), hipMemcpyHostToDevice, st));
    UV_BTRY(hipStreamSynchronize(st));
    return UV_OK;
}

// Times `iters` iterations of the instances in size bucket `bucket` (-1 =
// all) with the current tiles, from a copy of the current state that is put
// back afterwards.  *ms is the launch's duration.
int batch_time(uv_batch *h, int32_t bucket, int32_t iters, double *ms)
{
    if (!h || !ms || iters < 1 || bucket < -1 || bucket > 3) return UV_EINVAL;
    hipStream_t st = h->stream;
    const size_t ts = h->o.precision == UV_MIXED ? 4 : 8;
    std::vector<int> sel;
    UV_BTRY(hipStreamSynchronize(st));
    UV_BTRY(hipMemcpy(h->inst_host, h->inst, sizeof(BInst) * h->count, hipMemcpyDeviceToHost));
    for (int q = 0; q < h->count; ++q) {
        const int i = h->order_host[q];
        if (bucket < 0 || bucket_of(h->inst_host[i].m) == bucket) sel.push_back(i);
    }
    *ms = 0.0;
    if (sel.empty()) return UV_OK;
    // save state
    std::vector<BInst> inst_save(h->inst_host, h->inst_host + h->count);
    char *save = nullptr;
    const size_t bytes_xz = ts * h->N, bytes_u = ts * h->M;
    const size_t total = 2 * bytes_xz + bytes_u + 8 * (size_t)h->M + 8 * (size_t)h->N;
    if (uv::dev_malloc(&save, total) != hipSuccess) return UV_ENOMEM;
    char *p = save;
    int rc = UV_OK;
    auto cp_ = [&](void *dst, const void *src, size_t n) {
        if (rc == UV_OK && hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, st) != hipSuccess) rc = UV_EHIP;
    };
    cp_(p, h->x, bytes_xz);
    cp_(p + bytes_xz, h->z, bytes_xz);
    cp_(p + 2 * bytes_xz, h->u, bytes_u);
    cp_(p + 2 * bytes_xz + bytes_u, h->lam, 8 * (size_t)h->M);
    cp_(p + 2 * bytes_xz + bytes_u + 8 * (size_t)h->M, h->delta, 8 * (size_t)h->N);
    const bool saved = rc == UV_OK;  // restore below only from a complete copy
    int *dsel = nullptr;
    if (rc == UV_OK && uv::dev_malloc(&dsel, sizeof(int) * sel.size()) != hipSuccess) rc = UV_ENOMEM;
    if (rc == UV_OK && hipMemcpyAsync(dsel, sel.data(), sizeof(int) * sel.size(), hipMemcpyHostToDevice, st) != hipSuccess)
        rc = UV_EHIP;
    // run the timed launch with every selected instance marked running
    std::vector<BInst> tmp = inst_save;
    for (int i : sel) tmp[i].status = UV_STATUS_RUNNING;
    if (rc == UV_OK && hipMemcpyAsync(h->inst, tmp.data(), sizeof(BInst) * h->count, hipMemcpyHostToDevice, st) != hipSuccess)
        rc = UV_EHIP;
    // no early stop while timing: eps = 0 and no iteration cap
    const uv_opts keep = h->o;
    h->o.eps_kkt = 0.0;
    h->o.max_iter = 0;
    *h->budget_host = iters;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == UV_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) rc = UV_EHIP;
    if (rc == UV_OK && hipMemcpyAsync(h->budget, h->budget_host, sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess)
        rc = UV_EHIP;
    if (rc == UV_OK) {
        (void)hipEventRecord(e0, st);
        rc = batch_launch(h, st, dsel, (int)sel.size());
        (void)hipEventRecord(e1, st);
    }
    if (rc == UV_OK && hipStreamSynchronize(st) != hipSuccess) rc = UV_EHIP;
    float t = 0.f;
    if (rc == UV_OK) {
        (void)hipEventElapsedTime(&t, e0, e1);
        *ms = t;
    }
    h->o = keep;
    // restore, whatever happened in between (an error keeps its code)
    auto back = [&](void *dst, const void *src, size_t n) {
        if (hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, st) != hipSuccess) rc = UV_EHIP;
    };
    if (saved) {
        back(h->x, p, bytes_xz);
        back(h->z, p + bytes_xz, bytes_xz);
        back(h->u, p + 2 * bytes_xz, bytes_u);
        back(h->lam, p + 2 * bytes_xz + bytes_u, 8 * (size_t)h->M);
        back(h->delta, p + 2 * bytes_xz + bytes_u + 8 * (size_t)h->M, 8 * (size_t)h->N);
    }
    if (hipMemcpyAsync(h->inst, inst_save.data(), sizeof(BInst) * h->count, hipMemcpyHostToDevice, st) != hipSuccess)
        rc = UV_EHIP;
    if (hipStreamSynchronize(st) != hipSuccess) rc = UV_EHIP;
    std::memcpy(h->inst_host, inst_save.data(), sizeof(BInst) * h->count);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (dsel) (void)hipFree(dsel);
    (void)hipFree(save);
    return rc;
}

int batch_info(const uv_batch *h, int64_t *info)
{
    if (!h || !info) return UV_EINVAL;
    info[0] = h->count;
    info[1] = h->M;
    info[2] = h->N;
    info[3] = h->nnz;
    info[4] = h->grid;
    info[5] = h->lds_bytes;
    return UV_OK;
}

}  // extern "C"
