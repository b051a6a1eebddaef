// family.hip -- one matrix A and cost c, B right-hand sides b_1..b_B (a
// parametric family of LPs, orthant cone), iterated together.
//
// Every per-instance vector is stored instance-fastest: v[j * B + l] is
// entry j of instance l.  A wavefront takes one row (or column) of A and 64
// instances, so each nonzero of A is read once per 64 instances (a uniform,
// scalar load) and its gather of x or u is one contiguous 64-entry line.
// The iteration is the reduced form of Algorithm 1 used by the single
// solver; each instance is checked every check_every iterations and frozen
// (its stores are masked) once it stops.
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

constexpr int kResBlocks = 512;  // fixed grid of the residual passes

struct FInst {
    long long iter;  // the member's iterations when stopped (or at the last check)
    long long iter0; // family iteration count when the member started
    double r_prim, r_dual, r_gap, kkt, pobj, dobj, res_ax_b;
    double bnorm2;
    int status;
    int pad;
};

struct FShared {
    long long iter;  // iterations done by the family
    int active;      // instances still running
    int pad;
    double cnorm2;
};

// Work item of wave `wave` of workgroup `blk` in the sweep passes: segment
// (column or row) `seg` for the 64-instance group `grp`.  Workgroups go to
// the 8 XCDs in turn; when ng divides 8 the workgroup on XCD x always takes
// group x % ng, so an XCD's L2 holds the gathered lines of its own groups
// only (8 / ng workgroups of a round share a group, 4 segments each; 5-8 %
// faster per iteration at B = 256 on the 5e4 x 1e5 family than spreading
// every group over every XCD).  Otherwise a workgroup takes the ng groups of
// consecutive segments in turn.  Either way every (segment, group) pair is
// one wave's.
__device__ __forceinline__ void fam_item(int blk, int wave, int ng, int &seg, int &grp)
{
    if ((8 % ng) == 0) {
        const int x = blk & 7, per = 8 / ng;
        grp = x % ng;
        seg = ((blk >> 3) * per + x / ng) * 4 + wave;
    } else {
        const int gw = blk * 4 + wave;
        seg = gw / ng;
        grp = gw % ng;
    }
}

// Workgroups of a sweep pass over nseg segments (see fam_item).
inline unsigned fam_blocks(int nseg, int ng)
{
    if ((8 % ng) == 0) {
        const int per_round = 4 * (8 / ng);
        return (unsigned)(((int64_t)nseg + per_round - 1) / per_round * 8);
    }
    return (unsigned)(((int64_t)nseg * ng + 3) / 4);
}

// column pass: wave = (column j, 64 instances)
template <typename T>
__global__ void __launch_bounds__(256)
k_fam_col(int n, int B, const int *__restrict__ cp, const int *__restrict__ ri, const T *__restrict__ vc,
          const T *__restrict__ U, T *__restrict__ X, T *__restrict__ Z, double *__restrict__ D,
          const T *__restrict__ c, const FInst *__restrict__ inst, double mu, double inv_mu,
          const FShared *__restrict__ sh)
{
    if (sh->active == 0) return;
    const int lane = threadIdx.x & 63;
    int js, g;
    fam_item(blockIdx.x, threadIdx.x >> 6, B >> 6, js, g);
    const int j = __builtin_amdgcn_readfirstlane(js), l = __builtin_amdgcn_readfirstlane(g) * 64 + lane;
    if (j >= n) return;
    const int beg = cp[j], end = cp[j + 1];
    const size_t o = (size_t)j * B + l;
    const T xo = X[o], zo = Z[o], cj = c[j];
    const double d = D[o];
    T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int k = beg;
    for (; k + 3 < end; k += 4) {
        const int r0 = ri[k], r1 = ri[k + 1], r2 = ri[k + 2], r3 = ri[k + 3];
        const T v0 = vc[k], v1 = vc[k + 1], v2 = vc[k + 2], v3 = vc[k + 3];
        a0 += v0 * U[(size_t)r0 * B + l];
        a1 += v1 * U[(size_t)r1 * B + l];
        a2 += v2 * U[(size_t)r2 * B + l];
        a3 += v3 * U[(size_t)r3 * B + l];
    }
    for (; k < end; ++k) a0 += vc[k] * U[(size_t)ri[k] * B + l];
    const T atu = (a0 + a1) + (a2 + a3);
    if (inst[l].status != UV_STATUS_RUNNING) return;
    const int cnt = end - beg;
    const T dm = (T)(d * inv_mu);
    const T p = (T)cnt * xo + atu;
    const T xn = (p + zo + dm - cj * (T)inv_mu) / (T)(1 + cnt);
    const T v = xn - dm;
    const T zn = v > (T)0 ? v : (T)0;
    X[o] = xn;
    Z[o] = zn;
    D[o] = d + mu * ((double)zn - (double)xn);
}

// row pass: wave = (row i, 64 instances)
template <typename T>
__global__ void __launch_bounds__(256)
k_fam_row(int m, int B, const int *__restrict__ rp, const int *__restrict__ ci, const T *__restrict__ va,
          const T *__restrict__ X, const T *__restrict__ BV, const T *__restrict__ fu, double *__restrict__ LAM,
          T *__restrict__ U, const FInst *__restrict__ inst, double mu, double inv_mu, FShared *sh)
{
    if (sh->active == 0) return;
    const int lane = threadIdx.x & 63;
    int is, g;
    fam_item(blockIdx.x, threadIdx.x >> 6, B >> 6, is, g);
    const int i = __builtin_amdgcn_readfirstlane(is), l = __builtin_amdgcn_readfirstlane(g) * 64 + lane;
    if (blockIdx.x == 0 && threadIdx.x == 0) sh->iter += 1;
    if (i >= m) return;
    const int beg = rp[i], end = rp[i + 1];
    const size_t o = (size_t)i * B + l;
    const T bi = BV[o], fi = fu[i];
    const double l0 = LAM[o];
    T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int k = beg;
    for (; k + 3 < end; k += 4) {
        const int j0 = ci[k], j1 = ci[k + 1], j2 = ci[k + 2], j3 = ci[k + 3];
        const T v0 = va[k], v1 = va[k + 1], v2 = va[k + 2], v3 = va[k + 3];
        a0 += v0 * X[(size_t)j0 * B + l];
        a1 += v1 * X[(size_t)j1 * B + l];
        a2 += v2 * X[(size_t)j2 * B + l];
        a3 += v3 * X[(size_t)j3 * B + l];
    }
    for (; k < end; ++k) a0 += va[k] * X[(size_t)ci[k] * B + l];
    const T q = (a0 + a1) + (a2 + a3);
    if (inst[l].status != UV_STATUS_RUNNING) return;
    const T e = fi * (bi - q);
    const double li = l0 - mu * (double)e;
    LAM[o] = li;
    U[o] = (T)((double)e - li * inv_mu);
}

// Residual partials over rows: per instance ||A z - b||^2, b'lambda,
// ||A x - b||^2 (FP64 values of A).  part[(blk * 3 + k) * B + l].  The grid
// is kResBlocks * (B / 64): workgroup w takes the 64-instance group
// w / kResBlocks and the row chunk blk = w % kResBlocks (rows blk * 4 + wave,
// then every kResBlocks * 4-th); each wavefront sums a row's entries four at
// a time with their gathers in flight together.
template <typename T>
__global__ void __launch_bounds__(256)
k_fam_res_row(int m, int B, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ va,
              const T *__restrict__ X, const T *__restrict__ Z, const double *__restrict__ BV,
              const double *__restrict__ LAM, double *__restrict__ part)
{
    __shared__ double s[3][4][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int blk = blockIdx.x % kResBlocks, l = (blockIdx.x / kResBlocks) * 64 + lane;
    double a[3] = {0.0, 0.0, 0.0};
    for (int i = blk * 4 + w; i < m; i += kResBlocks * 4) {
        const int beg = rp[i], end = rp[i + 1];
        double z0 = 0.0, z1 = 0.0, z2 = 0.0, z3 = 0.0, x0 = 0.0, x1 = 0.0, x2 = 0.0, x3 = 0.0;
        int k = beg;
        for (; k + 3 < end; k += 4) {
            const size_t o0 = (size_t)ci[k] * B + l, o1 = (size_t)ci[k + 1] * B + l;
            const size_t o2 = (size_t)ci[k + 2] * B + l, o3 = (size_t)ci[k + 3] * B + l;
            const double v0 = va[k], v1 = va[k + 1], v2 = va[k + 2], v3 = va[k + 3];
            z0 += v0 * (double)Z[o0];
            z1 += v1 * (double)Z[o1];
            z2 += v2 * (double)Z[o2];
            z3 += v3 * (double)Z[o3];
            x0 += v0 * (double)X[o0];
            x1 += v1 * (double)X[o1];
            x2 += v2 * (double)X[o2];
            x3 += v3 * (double)X[o3];
        }
        for (; k < end; ++k) {
            const size_t o = (size_t)ci[k] * B + l;
            z0 += va[k] * (double)Z[o];
            x0 += va[k] * (double)X[o];
        }
        const double qz = (z0 + z1) + (z2 + z3), qx = (x0 + x1) + (x2 + x3);
        const double bi = BV[(size_t)i * B + l];
        a[0] += (qz - bi) * (qz - bi);
        a[1] += bi * LAM[(size_t)i * B + l];
        a[2] += (qx - bi) * (qx - bi);
    }
    for (int k = 0; k < 3; ++k) s[k][w][lane] = a[k];
    __syncthreads();
    if (w == 0)
        for (int k = 0; k < 3; ++k)
            part[((size_t)blk * 3 + k) * B + l] = ((s[k][0][lane] + s[k][1][lane]) + s[k][2][lane]) + s[k][3][lane];
}

// The row pass of a check iteration, on the grid of k_fam_res_row: each
// row's A z and A x in FP64 (FP64 values of A, the same sums in the same
// order as k_fam_res_row), the iteration's lambda and u updates from that
// A x (rounded to the sweep type), and the row partials of the check with
// the updated lambda -- one pass where the row pass and k_fam_res_row took
// two.
template <typename T>
__global__ void __launch_bounds__(256)
k_fam_row_check(int m, int B, const int *__restrict__ rp, const int *__restrict__ ci,
                const double *__restrict__ va, const T *__restrict__ X, const T *__restrict__ Z,
                const T *__restrict__ BV, const double *__restrict__ BV64, const T *__restrict__ fu,
                double *__restrict__ LAM, T *__restrict__ U, const FInst *__restrict__ inst, double mu,
                double inv_mu, FShared *sh, double *__restrict__ part)
{
    if (sh->active == 0) return;
    __shared__ double s[3][4][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int blk = blockIdx.x % kResBlocks, l = (blockIdx.x / kResBlocks) * 64 + lane;
    if (blockIdx.x == 0 && threadIdx.x == 0) sh->iter += 1;
    const bool run = inst[l].status == UV_STATUS_RUNNING;
    double a[3] = {0.0, 0.0, 0.0};
    for (int i = blk * 4 + w; i < m; i += kResBlocks * 4) {
        const int beg = rp[i], end = rp[i + 1];
        double z0 = 0.0, z1 = 0.0, z2 = 0.0, z3 = 0.0, x0 = 0.0, x1 = 0.0, x2 = 0.0, x3 = 0.0;
        int k = beg;
        for (; k + 3 < end; k += 4) {
            const size_t o0 = (size_t)ci[k] * B + l, o1 = (size_t)ci[k + 1] * B + l;
            const size_t o2 = (size_t)ci[k + 2] * B + l, o3 = (size_t)ci[k + 3] * B + l;
            const double v0 = va[k], v1 = va[k + 1], v2 = va[k + 2], v3 = va[k + 3];
            z0 += v0 * (double)Z[o0];
            z1 += v1 * (double)Z[o1];
            z2 += v2 * (double)Z[o2];
            z3 += v3 * (double)Z[o3];
            x0 += v0 * (double)X[o0];
            x1 += v1 * (double)X[o1];
            x2 += v2 * (double)X[o2];
            x3 += v3 * (double)X[o3];
        }
        for (; k < end; ++k) {
            const size_t o = (size_t)ci[k] * B + l;
            z0 += va[k] * (double)Z[o];
            x0 += va[k] * (double)X[o];
        }
        const double qz = (z0 + z1) + (z2 + z3), qx = (x0 + x1) + (x2 + x3);
        const size_t o = (size_t)i * B + l;
        double li = LAM[o];
        if (run) {
            const T e = fu[i] * (BV[o] - (T)qx);
            li = li - mu * (double)e;
            LAM[o] = li;
            U[o] = (T)((double)e - li * inv_mu);
        }
        const double bi = BV64[o];
        a[0] += (qz - bi) * (qz - bi);
        a[1] += bi * li;
        a[2] += (qx - bi) * (qx - bi);
    }
    for (int k = 0; k < 3; ++k) s[k][w][lane] = a[k];
    __syncthreads();
    if (w == 0)
        for (int k = 0; k < 3; ++k)
            part[((size_t)blk * 3 + k) * B + l] = ((s[k][0][lane] + s[k][1][lane]) + s[k][2][lane]) + s[k][3][lane];
}

// Residual partials over columns: ||A'lambda + c - delta||^2, c'z (same
// grid and order as the row partials).
template <typename T>
__global__ void __launch_bounds__(256)
k_fam_res_col(int n, int B, const int *__restrict__ cp, const int *__restrict__ ri, const double *__restrict__ vc,
              const double *__restrict__ LAM, const double *__restrict__ c, const double *__restrict__ D,
              const T *__restrict__ Z, double *__restrict__ part)
{
    __shared__ double s[2][4][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int blk = blockIdx.x % kResBlocks, l = (blockIdx.x / kResBlocks) * 64 + lane;
    double a[2] = {0.0, 0.0};
    for (int j = blk * 4 + w; j < n; j += kResBlocks * 4) {
        const int beg = cp[j], end = cp[j + 1];
        double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
        int k = beg;
        for (; k + 3 < end; k += 4) {
            t0 += vc[k] * LAM[(size_t)ri[k] * B + l];
            t1 += vc[k + 1] * LAM[(size_t)ri[k + 1] * B + l];
            t2 += vc[k + 2] * LAM[(size_t)ri[k + 2] * B + l];
            t3 += vc[k + 3] * LAM[(size_t)ri[k + 3] * B + l];
        }
        for (; k < end; ++k) t0 += vc[k] * LAM[(size_t)ri[k] * B + l];
        const double t = (t0 + t1) + (t2 + t3);
        const size_t o = (size_t)j * B + l;
        const double r = t + c[j] - D[o];
        a[0] += r * r;
        a[1] += c[j] * (double)Z[o];
    }
    for (int k = 0; k < 2; ++k) s[k][w][lane] = a[k];
    __syncthreads();
    if (w == 0)
        for (int k = 0; k < 2; ++k)
            part[((size_t)blk * 2 + k) * B + l] = ((s[k][0][lane] + s[k][1][lane]) + s[k][2][lane]) + s[k][3][lane];
}

constexpr int kFold = 16;  // partial blocks added per thread in the first stage of the check's sum
static_assert(kResBlocks % kFold == 0, "the partial blocks fold into whole groups");

// First stage of the check's sum: red[(g * 5 + k) * B + l] = the sum, in
// block order, of component k of instance l over the partial blocks
// g * kFold .. (g + 1) * kFold - 1 (components 0-2 from the row pass, 3-4
// from the column pass).  k_fam_finalize then adds the groups in order, so
// the result is fixed and independent of the launch.
__global__ void __launch_bounds__(256)
k_fam_fold(int B, int nblk, const double *__restrict__ prow, const double *__restrict__ pcol, double *__restrict__ red)
{
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    const int ng = nblk / kFold;
    if (t >= (size_t)ng * 5 * B) return;
    const int l = (int)(t % B), k = (int)((t / B) % 5), g = (int)(t / ((size_t)B * 5));
    double v[kFold];
#pragma unroll
    for (int r = 0; r < kFold; ++r) {
        const size_t b = (size_t)g * kFold + r;
        v[r] = k < 3 ? prow[(b * 3 + k) * B + l] : pcol[(b * 2 + (k - 3)) * B + l];
    }
    double s = 0.0;
#pragma unroll
    for (int r = 0; r < kFold; ++r) s += v[r];
    red[t] = s;
}

// One thread per instance: add the group sums of k_fam_fold in order, decide.
__global__ void __launch_bounds__(1024)
k_fam_finalize(int B, int nblk, const double *__restrict__ red, double eps, long long max_iter, FInst *inst,
               FShared *sh)
{
    __shared__ int s_active[1024];
    const int l = threadIdx.x;
    int running = 0;
    if (l < B) {
        FInst &I = inst[l];
        if (I.status == UV_STATUS_RUNNING) {
            double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            for (int b0 = 0; b0 < nblk; b0 += 8) {  // eight blocks' loads in flight, added in block order
                double t[8][5];
#pragma unroll
                for (int r = 0; r < 8; ++r) {
                    const int b = b0 + r < nblk ? b0 + r : nblk - 1;
                    for (int k = 0; k < 5; ++k) t[r][k] = red[((size_t)b * 5 + k) * B + l];
                }
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    if (b0 + r < nblk)
                        for (int k = 0; k < 5; ++k) a[k] += t[r][k];
            }
            const double rpr = sqrt(a[0]) / (1.0 + sqrt(I.bnorm2));
            const double rdu = sqrt(a[3]) / (1.0 + sqrt(sh->cnorm2));
            const double cz = a[4], bl = a[1];
            const double rg = fabs(cz + bl) / (1.0 + fabs(cz) + fabs(bl));
            const double kkt = uv::kkt_of(rpr, rdu, rg);
            I.r_prim = rpr;
            I.r_dual = rdu;
            I.r_gap = rg;
            I.kkt = kkt;
            I.pobj = cz;
            I.dobj = -bl;
            I.res_ax_b = sqrt(a[2]);
            I.iter = sh->iter - I.iter0;
            if (!isfinite(kkt)) I.status = UV_STATUS_NUMERIC;
            else if (kkt <= eps) I.status = UV_STATUS_CONVERGED;
            else if (max_iter > 0 && I.iter >= max_iter) I.status = UV_STATUS_MAX_ITER;
            running = I.status == UV_STATUS_RUNNING;
        }
    }
    s_active[l] = running;
    __syncthreads();
    if (l == 0) {
        int t = 0;
        for (int i = 0; i < (int)blockDim.x; ++i) t += s_active[i];
        sh->active = t;
    }
}

// Instance-major host layout <-> instance-fastest device layout.
template <typename S, typename T>
__global__ void __launch_bounds__(256)
k_fam_to_dev(int len, int B, int nb, const S *__restrict__ src, T *__restrict__ dst)
{
    // src[l * len + j] (l < nb) -> dst[j * B + l]; instances >= nb get 0
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (size_t)len * B) return;
    const int j = (int)(t / B), l = (int)(t % B);
    dst[t] = l < nb ? (T)src[(size_t)l * len + j] : (T)0;
}

template <typename S, typename T>
__global__ void __launch_bounds__(256)
k_fam_from_dev(int len, int B, int nb, const S *__restrict__ src, T *__restrict__ dst, size_t ld, int off)
{
    // src[j * B + l] -> dst[l * ld + off + j] for l < nb
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (size_t)len * nb) return;
    const int l = (int)(t / len), j = (int)(t % len);
    dst[(size_t)l * ld + off + j] = (T)src[(size_t)j * B + l];
}

// One instance's column: src[j * B + slot] -> dst[j] (FP64).
template <typename S>
__global__ void __launch_bounds__(256)
k_fam_slot_from_dev(int len, int B, int slot, const S *__restrict__ src, double *__restrict__ dst)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j < len) dst[j] = (double)src[(size_t)j * B + slot];
}

// u = -lambda/mu for all instances, and per-instance reset.
template <typename T>
__global__ void __launch_bounds__(256)
k_fam_start(size_t len, const double *__restrict__ LAM, T *__restrict__ U, double inv_mu)
{
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t < len) U[t] = (T)(-LAM[t] * inv_mu);
}

// Warm start from predicted (x, lambda): z = max(x, 0),
// delta = max(c + A'lambda, 0) (the dual-feasible part of the stationarity
// condition c + A'lambda - delta = 0), u = -lambda/mu.
template <typename T>
__global__ void __launch_bounds__(256)
k_fam_dual_start(int n, int B, const int *__restrict__ cp, const int *__restrict__ ri,
                 const double *__restrict__ vc, const double *__restrict__ LAM, const double *__restrict__ c,
                 const T *__restrict__ X, T *__restrict__ Z, double *__restrict__ D)
{
    const int gw = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int ng = B >> 6;
    const int j = gw / ng, l = (gw % ng) * 64 + lane;
    if (j >= n) return;
    double t = 0.0;
    for (int k = cp[j]; k < cp[j + 1]; ++k) t += vc[k] * LAM[(size_t)ri[k] * B + l];
    const size_t o = (size_t)j * B + l;
    const double s = c[j] + t;
    D[o] = s > 0.0 ? s : 0.0;
    const T xo = X[o];
    Z[o] = xo > (T)0 ? xo : (T)0;
}

__global__ void __launch_bounds__(1024)
k_fam_reset(int B, int nb, FInst *inst, FShared *sh, const double *__restrict__ BV64)
{
    (void)BV64;
    const int l = threadIdx.x;
    if (l < B) {
        inst[l].status = l < nb ? UV_STATUS_RUNNING : UV_STATUS_CONVERGED;  // padding lanes never run
        inst[l].iter = 0;
        inst[l].iter0 = 0;
    }
    if (l == 0) {
        sh->iter = 0;
        sh->active = nb;
    }
}

// ||b_l||^2 per instance in two fixed-order stages: part[c * B + l] sums
// the rows c, c + kBChunks, c + 2 kBChunks, ... (eight loads in flight),
// then one thread per instance adds the kBChunks partials in order.
constexpr int kBChunks = 256;
static_assert(kBChunks % 8 == 0 && kBChunks <= 3 * kResBlocks, "partials fit the check's row scratch");

__global__ void __launch_bounds__(256)
k_fam_bnorm_part(int m, int B, const double *__restrict__ BV64, double *__restrict__ part)
{
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (size_t)kBChunks * B) return;
    const int l = (int)(t % B), c = (int)(t / B);
    double s = 0.0;
    for (int i0 = c; i0 < m; i0 += 8 * kBChunks) {
        double v[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int i = i0 + r * kBChunks;
            v[r] = i < m ? BV64[(size_t)i * B + l] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) s += v[r] * v[r];
    }
    part[t] = s;
}

__global__ void __launch_bounds__(1024) k_fam_bnorm(int B, const double *__restrict__ part, FInst *inst)
{
    const int l = threadIdx.x;
    if (l >= B) return;
    double s = 0.0;
    for (int c0 = 0; c0 < kBChunks; c0 += 8) {
        double v[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = part[(size_t)(c0 + r) * B + l];
#pragma unroll
        for (int r = 0; r < 8; ++r) s += v[r];
    }
    inst[l].bnorm2 = s;
}

// Refill: right-hand side of the members entering slots[q] (q < count),
// from the FP64 rows b[q * m + i] staged on the device.
template <typename T>
__global__ void __launch_bounds__(256)
k_fam_slot_rhs(int m, int B, int count, const int *__restrict__ slots, const double *__restrict__ b,
               T *__restrict__ BV, double *__restrict__ BV64)
{
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (size_t)count * m) return;
    const int q = (int)(t / m), i = (int)(t % m);
    const size_t o = (size_t)i * B + slots[q];
    BV[o] = (T)b[t];
    BV64[o] = b[t];
}

// Refill: start of the entering members, x and lambda from the FP32 rows
// xl[q * ld + (0..n-1)] and xl[q * ld + n + (0..m-1)] (parts as in
// family_set_start_predicted), or zero when xl is null.
template <typename T>
__global__ void __launch_bounds__(256)
k_fam_slot_xl(int n, int m, int B, int count, const int *__restrict__ slots, const float *__restrict__ xl,
              long long ld, int parts, T *__restrict__ X, double *__restrict__ LAM)
{
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    const int len = n + m;
    if (t >= (size_t)count * len) return;
    const int q = (int)(t / len), j = (int)(t % len);
    const int sl = slots[q];
    const bool use = xl && (j < n ? (parts & 1) : (parts & 2));
    const float v = use ? xl[(size_t)q * ld + j] : 0.0f;
    if (j < n) X[(size_t)j * B + sl] = (T)v;
    else LAM[(size_t)(j - n) * B + sl] = (double)v;
}

// Refill: z = max(x, 0) and delta = max(c + A'lambda, 0) of the entering
// members (the arithmetic of k_fam_dual_start; zero for a zero start).
template <typename T>
__global__ void __launch_bounds__(256)
k_fam_slot_zd(int n, int B, int count, const int *__restrict__ slots, const int *__restrict__ cp,
              const int *__restrict__ ri, const double *__restrict__ vc, const double *__restrict__ LAM,
              const double *__restrict__ c, const T *__restrict__ X, T *__restrict__ Z, double *__restrict__ D,
              int zero)
{
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (size_t)count * n) return;
    const int q = (int)(t / n), j = (int)(t % n);
    const int sl = slots[q];
    const size_t o = (size_t)j * B + sl;
    if (zero) {
        Z[o] = (T)0;
        D[o] = 0.0;
        return;
    }
    double a = 0.0;
    for (int k = cp[j]; k < cp[j + 1]; ++k) a += vc[k] * LAM[(size_t)ri[k] * B + sl];
    const double v = c[j] + a;
    D[o] = v > 0.0 ? v : 0.0;
    const T xo = X[o];
    Z[o] = xo > (T)0 ? xo : (T)0;
}

// Refill: u = -lambda/mu of the entering members.
template <typename T>
__global__ void __launch_bounds__(256)
k_fam_slot_u(int m, int B, int count, const int *__restrict__ slots, const double *__restrict__ LAM,
             T *__restrict__ U, double inv_mu)
{
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= (size_t)count * m) return;
    const int q = (int)(t / m), i = (int)(t % m);
    const size_t o = (size_t)i * B + slots[q];
    U[o] = (T)(-LAM[o] * inv_mu);
}

// Refill: the entering members run from the family's current iteration;
// the running count is taken again.
__global__ void __launch_bounds__(1024)
k_fam_slot_reset(int B, int count, const int *__restrict__ slots, FInst *inst, FShared *sh)
{
    __shared__ int s_run[1024];
    const int l = threadIdx.x;
    if (l < count) {
        FInst &I = inst[slots[l]];
        I.status = UV_STATUS_RUNNING;
        I.iter = 0;
        I.iter0 = sh->iter;
    }
    __syncthreads();
    s_run[l] = l < B && inst[l].status == UV_STATUS_RUNNING;
    __syncthreads();
    if (l == 0) {
        int t = 0;
        for (int i = 0; i < (int)blockDim.x; ++i) t += s_run[i];
        sh->active = t;
    }
}

}  // namespace

struct uv_family {
    int m = 0, n = 0, nnz = 0, B = 0, nb = 0;
    uv_opts o{};
    hipStream_t stream = nullptr, cap = nullptr;
    bool own_stream = false;
    std::vector<void *> allocs;
    int *rp = nullptr, *ci = nullptr, *cp = nullptr, *ri = nullptr;
    double *va64 = nullptr, *vc64 = nullptr, *c64 = nullptr;
    void *va = nullptr, *vc = nullptr, *c = nullptr, *fu = nullptr;
    void *X = nullptr, *Z = nullptr, *U = nullptr, *BV = nullptr;
    double *LAM = nullptr, *D = nullptr, *BV64 = nullptr;
    double *prow = nullptr, *pcol = nullptr, *pred = nullptr;
    double *stage = nullptr;  // B * max(m, n) doubles of staging
    FInst *inst = nullptr, *inst_host = nullptr;
    FShared *sh = nullptr, *sh_host = nullptr;
    int *slots = nullptr;     // slot list of a refill (B entries)
    bool refilled = false;    // a member entered after the last set_rhs / set_start
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t host_iter = 0;
};

namespace {

template <typename T>
T *falloc(uv_family *h, size_t count)
{
    void *p = nullptr;
    if (uv::dev_malloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return nullptr;
    h->allocs.push_back(p);
    return (T *)p;
}

#define UV_FTRY(expr)                              \
    do {                                           \
        if ((expr) != hipSuccess) return UV_EHIP;  \
    } while (0)

template <typename T>
void fam_iteration_t(uv_family *h, hipStream_t st, bool check)
{
    const double mu = h->o.mu, im = 1.0 / h->o.mu;
    const int ng = h->B / 64;
    k_fam_col<T><<<fam_blocks(h->n, ng), 256, 0, st>>>(
        h->n, h->B, h->cp, h->ri, (const T *)h->vc, (const T *)h->U, (T *)h->X, (T *)h->Z, h->D, (const T *)h->c,
        h->inst, mu, im, h->sh);
    if (!check) {
        k_fam_row<T><<<fam_blocks(h->m, ng), 256, 0, st>>>(
            h->m, h->B, h->rp, h->ci, (const T *)h->va, (const T *)h->X, (const T *)h->BV, (const T *)h->fu, h->LAM,
            (T *)h->U, h->inst, mu, im, h->sh);
    } else {
        k_fam_row_check<T><<<kResBlocks * ng, 256, 0, st>>>(
            h->m, h->B, h->rp, h->ci, h->va64, (const T *)h->X, (const T *)h->Z, (const T *)h->BV, h->BV64,
            (const T *)h->fu, h->LAM, (T *)h->U, h->inst, mu, im, h->sh, h->prow);
        k_fam_res_col<T><<<kResBlocks * (h->B / 64), 256, 0, st>>>(h->n, h->B, h->cp, h->ri, h->vc64, h->LAM, h->c64, h->D,
                                                     (const T *)h->Z, h->pcol);
        const int ng = kResBlocks / kFold;
        k_fam_fold<<<blocks_for((int64_t)ng * 5 * h->B, 256), 256, 0, st>>>(h->B, kResBlocks, h->prow, h->pcol,
                                                                           h->pred);
        k_fam_finalize<<<1, 1024, 0, st>>>(h->B, ng, h->pred, h->o.eps_kkt, (long long)h->o.max_iter, h->inst,
                                           h->sh);
    }
}

void fam_iteration(uv_family *h, hipStream_t st, bool check)
{
    if (h->o.precision == UV_MIXED) fam_iteration_t<float>(h, st, check);
    else fam_iteration_t<double>(h, st, check);
}

int fam_sync(uv_family *h)
{
    UV_FTRY(hipMemcpyAsync(h->inst_host, h->inst, sizeof(FInst) * h->B, hipMemcpyDeviceToHost, h->stream));
    UV_FTRY(hipMemcpyAsync(h->sh_host, h->sh, sizeof(FShared), hipMemcpyDeviceToHost, h->stream));
    UV_FTRY(hipStreamSynchronize(h->stream));
    h->host_iter = h->sh_host->iter;
    return UV_OK;
}

template <typename S>
int upload_cols(uv_family *h, const S *src, int len, void *dst, bool to_f64)
{
    // host instance-major (nb x len) -> device instance-fastest (len x B)
    hipStream_t st = h->stream;
    const size_t bytes = sizeof(S) * (size_t)h->nb * len;
    UV_FTRY(hipMemcpyAsync(h->stage, src, bytes, hipMemcpyHostToDevice, st));
    const unsigned g = blocks_for((int64_t)len * h->B, 256);
    if (to_f64) k_fam_to_dev<S, double><<<g, 256, 0, st>>>(len, h->B, h->nb, (const S *)h->stage, (double *)dst);
    else if (h->o.precision == UV_MIXED)
        k_fam_to_dev<S, float><<<g, 256, 0, st>>>(len, h->B, h->nb, (const S *)h->stage, (float *)dst);
    else k_fam_to_dev<S, double><<<g, 256, 0, st>>>(len, h->B, h->nb, (const S *)h->stage, (double *)dst);
    UV_FTRY(hipGetLastError());
    UV_FTRY(hipStreamSynchronize(st));  // the staging buffer is reused
    return UV_OK;
}

int fam_rebuild_graph(uv_family *h)
{
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    h->exec = nullptr;
    h->graph = nullptr;
    if (!h->o.use_graph) return UV_OK;
    if (hipStreamBeginCapture(h->cap, hipStreamCaptureModeRelaxed) != hipSuccess) return UV_EHIP;
    for (int i = 0; i < h->o.check_every; ++i) fam_iteration(h, h->cap, i == h->o.check_every - 1);
    if (hipStreamEndCapture(h->cap, &h->graph) != hipSuccess) return UV_EHIP;
    if (hipGraphInstantiate(&h->exec, h->graph, nullptr, nullptr, 0) != hipSuccess) return UV_EHIP;
    return UV_OK;
}

}  // namespace

extern "C" {

void family_destroy(uv_family *h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->exec) (void)hipGraphExecDestroy(h->exec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    for (void *p : h->allocs) (void)hipFree(p);
    if (h->inst_host) (void)hipHostFree(h->inst_host);
    if (h->sh_host) (void)hipHostFree(h->sh_host);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

int family_create(const uv_csr *A, const double *c, int32_t B, const uv_opts *opts, uv_family **out)
{
    if (!out) return UV_EINVAL;
    *out = nullptr;
    if (!A || !c || B < 64 || B > 1024 || B % 64) return UV_EINVAL;
    uv_opts o;
    uv_default_opts(&o);
    if (opts) o = *opts;
    if (!(o.mu > 0.0) || !std::isfinite(o.mu) || o.check_every < 1 || !(o.eps_kkt >= 0.0) || o.max_iter < 0 ||
        (o.precision != UV_FP64 && o.precision != UV_MIXED))
        return UV_EINVAL;
    if (A->m < 1 || A->n < 1 || A->nnz < 0 || !A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val)))
        return UV_EINVAL;
    if (A->nnz >= ((int64_t)1 << 31)) return UV_ETOOBIG;
    if ((int64_t)B * std::max(A->m, A->n) >= ((int64_t)1 << 40)) return UV_ETOOBIG;
    if (A->row_ptr[0] != 0 || A->row_ptr[A->m] != A->nnz) return UV_EBADCSR;
    for (int32_t i = 0; i < A->m; ++i) {
        const int64_t b0 = A->row_ptr[i], b1 = A->row_ptr[i + 1];
        if (b1 < b0 || b1 > A->nnz) return UV_EBADCSR;
        for (int64_t k = b0; k < b1; ++k) {
            if (A->col_idx[k] < 0 || A->col_idx[k] >= A->n) return UV_EBADCSR;
            if (k > b0 && A->col_idx[k] <= A->col_idx[k - 1]) return UV_EBADCSR;
        }
    }
    uv_family *h = new (std::nothrow) uv_family();
    if (!h) return UV_ENOMEM;
    auto fail = [&](int code) {
        family_destroy(h);
        return code;
    };
    h->m = A->m;
    h->n = A->n;
    h->nnz = (int)A->nnz;
    h->B = B;
    h->nb = 0;
    h->o = o;
    const int m = h->m, n = h->n, nnz = h->nnz;
    const bool mixed = o.precision == UV_MIXED;
    const size_t ts = mixed ? 4 : 8;
    if (o.hip_stream) h->stream = (hipStream_t)o.hip_stream;
    else {
        if (hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) != hipSuccess) return fail(UV_EHIP);
        h->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess) return fail(UV_EHIP);
    hipStream_t st = h->stream;
    h->rp = falloc<int>(h, m + 1);
    h->ci = falloc<int>(h, nnz);
    h->va64 = falloc<double>(h, nnz);
    h->cp = falloc<int>(h, n + 1);
    h->ri = falloc<int>(h, nnz);
    h->vc64 = falloc<double>(h, nnz);
    h->c64 = falloc<double>(h, n);
    h->fu = falloc<char>(h, ts * m);
    if (mixed) {
        h->va = falloc<float>(h, nnz);
        h->vc = falloc<float>(h, nnz);
        h->c = falloc<float>(h, n);
    } else {
        h->va = h->va64;
        h->vc = h->vc64;
        h->c = h->c64;
    }
    const size_t Bn = (size_t)B * n, Bm = (size_t)B * m;
    h->X = falloc<char>(h, ts * Bn);
    h->Z = falloc<char>(h, ts * Bn);
    h->U = falloc<char>(h, ts * Bm);
    h->BV = falloc<char>(h, ts * Bm);
    h->LAM = falloc<double>(h, Bm);
    h->D = falloc<double>(h, Bn);
    h->BV64 = falloc<double>(h, Bm);
    h->prow = falloc<double>(h, (size_t)kResBlocks * 3 * B);
    h->pcol = falloc<double>(h, (size_t)kResBlocks * 2 * B);
    h->pred = falloc<double>(h, (size_t)(kResBlocks / kFold) * 5 * B);
    h->stage = falloc<double>(h, (size_t)B * std::max(m, n));
    h->inst = falloc<FInst>(h, B);
    h->sh = falloc<FShared>(h, 1);
    h->slots = falloc<int>(h, B);
    int *cnt = falloc<int>(h, n);
    int *bsum = falloc<int>(h, blocks_for(n, 4 * kWG));
    for (void *p : {(void *)h->rp, (void *)h->ci, (void *)h->va64, (void *)h->cp, (void *)h->ri, (void *)h->vc64,
                    (void *)h->c64, h->fu, h->va, h->vc, h->c, h->X, h->Z, h->U, h->BV, (void *)h->LAM,
                    (void *)h->D, (void *)h->BV64, (void *)h->prow, (void *)h->pcol, (void *)h->pred, (void *)h->stage,
                    (void *)h->inst, (void *)h->sh, (void *)h->slots, (void *)cnt, (void *)bsum})
        if (!p) return fail(UV_ENOMEM);
    if (uv::host_malloc(&h->inst_host, sizeof(FInst) * B, hipHostMallocDefault) != hipSuccess) {
        h->inst_host = nullptr;
        return fail(UV_ENOMEM);
    }
    if (uv::host_malloc(&h->sh_host, sizeof(FShared), hipHostMallocDefault) != hipSuccess) {
        h->sh_host = nullptr;
        return fail(UV_ENOMEM);
    }
    {
        std::vector<int> rp32(m + 1);
        for (int i = 0; i <= m; ++i) rp32[i] = (int)A->row_ptr[i];
        if (hipMemcpy(h->rp, rp32.data(), 4 * (size_t)(m + 1), hipMemcpyHostToDevice) != hipSuccess) return fail(UV_EHIP);
    }
    if (nnz > 0 && (hipMemcpy(h->ci, A->col_idx, 4 * (size_t)nnz, hipMemcpyHostToDevice) != hipSuccess ||
                    hipMemcpy(h->va64, A->val, 8 * (size_t)nnz, hipMemcpyHostToDevice) != hipSuccess))
        return fail(UV_EHIP);
    if (hipMemcpy(h->c64, c, 8 * (size_t)n, hipMemcpyHostToDevice) != hipSuccess) return fail(UV_EHIP);
    if (!build_csc(m, n, nnz, h->rp, h->ci, h->va64, h->cp, h->ri, h->vc64, cnt, bsum, st)) return fail(UV_EHIP);
    if (mixed) {
        k_row_factor<float><<<blocks_for(m, kWG), kWG, 0, st>>>(m, h->rp, h->va64, (float *)h->fu);
        if (nnz > 0) {
            k_narrow<float><<<blocks_for(nnz, kWG), kWG, 0, st>>>(nnz, h->va64, (float *)h->va);
            k_narrow<float><<<blocks_for(nnz, kWG), kWG, 0, st>>>(nnz, h->vc64, (float *)h->vc);
        }
        k_narrow<float><<<blocks_for(n, kWG), kWG, 0, st>>>(n, h->c64, (float *)h->c);
    } else {
        k_row_factor<double><<<blocks_for(m, kWG), kWG, 0, st>>>(m, h->rp, h->va64, (double *)h->fu);
    }
    if (hipGetLastError() != hipSuccess) return fail(UV_EHIP);
    {
        double cn = 0.0;
        for (int j = 0; j < n; ++j) cn += c[j] * c[j];
        FShared s0{};
        s0.cnorm2 = cn;
        if (hipMemcpy(h->sh, &s0, sizeof(s0), hipMemcpyHostToDevice) != hipSuccess) return fail(UV_EHIP);
        std::vector<FInst> i0(B);
        std::memset(i0.data(), 0, sizeof(FInst) * B);
        for (auto &x : i0) x.status = UV_STATUS_CONVERGED;  // nothing runs before a right-hand side is set
        if (hipMemcpy(h->inst, i0.data(), sizeof(FInst) * B, hipMemcpyHostToDevice) != hipSuccess) return fail(UV_EHIP);
    }
    if (hipStreamSynchronize(st) != hipSuccess) return fail(UV_EHIP);
    int rc = fam_rebuild_graph(h);
    if (rc != UV_OK) return fail(rc);
    if ((rc = fam_sync(h)) != UV_OK) return fail(rc);
    *out = h;
    return UV_OK;
}

int family_set_rhs(uv_family *h, int32_t nb, const double *b)
{
    if (!h || !b || nb < 1 || nb > h->B) return UV_EINVAL;
    h->nb = nb;
    int rc;
    if ((rc = upload_cols<double>(h, b, h->m, h->BV, false)) != UV_OK) return rc;
    if ((rc = upload_cols<double>(h, b, h->m, h->BV64, true)) != UV_OK) return rc;
    // the check's row partials serve as scratch (kResBlocks * 3 * B >= kBChunks * B doubles)
    k_fam_bnorm_part<<<blocks_for((int64_t)kBChunks * h->B, 256), 256, 0, h->stream>>>(h->m, h->B, h->BV64, h->prow);
    k_fam_bnorm<<<1, 1024, 0, h->stream>>>(h->B, h->prow, h->inst);
    UV_FTRY(hipGetLastError());
    return family_set_start(h, nullptr, nullptr, nullptr, nullptr);
}

int family_set_start(uv_family *h, const double *x, const double *z, const double *delta, const double *lambda)
{
    if (!h || h->nb < 1) return UV_EINVAL;
    hipStream_t st = h->stream;
    const size_t ts = h->o.precision == UV_MIXED ? 4 : 8;
    const size_t Bn = (size_t)h->B * h->n, Bm = (size_t)h->B * h->m;
    int rc;
    if (x) { if ((rc = upload_cols<double>(h, x, h->n, h->X, false)) != UV_OK) return rc; }
    else UV_FTRY(hipMemsetAsync(h->X, 0, ts * Bn, st));
    if (z) { if ((rc = upload_cols<double>(h, z, h->n, h->Z, false)) != UV_OK) return rc; }
    else UV_FTRY(hipMemsetAsync(h->Z, 0, ts * Bn, st));
    if (delta) { if ((rc = upload_cols<double>(h, delta, h->n, h->D, true)) != UV_OK) return rc; }
    else UV_FTRY(hipMemsetAsync(h->D, 0, 8 * Bn, st));
    if (lambda) { if ((rc = upload_cols<double>(h, lambda, h->m, h->LAM, true)) != UV_OK) return rc; }
    else UV_FTRY(hipMemsetAsync(h->LAM, 0, 8 * Bm, st));
    const double im = 1.0 / h->o.mu;
    if (h->o.precision == UV_MIXED) k_fam_start<float><<<blocks_for(Bm, 256), 256, 0, st>>>(Bm, h->LAM, (float *)h->U, im);
    else k_fam_start<double><<<blocks_for(Bm, 256), 256, 0, st>>>(Bm, h->LAM, (double *)h->U, im);
    k_fam_reset<<<1, 1024, 0, st>>>(h->B, h->nb, h->inst, h->sh, h->BV64);
    h->refilled = false;
    UV_FTRY(hipGetLastError());
    return fam_sync(h);
}

int family_set_start_predicted(uv_family *h, const float *xl_dev, int64_t ld, int32_t parts)
{
    // xl_dev: device, instance-major rows [x (n) ; lambda (m)] with row stride ld
    if (!h || !xl_dev || h->nb < 1 || ld < (int64_t)h->n + h->m || parts < 1 || parts > 3) return UV_EINVAL;
    hipStream_t st = h->stream;
    const int B = h->B, nb = h->nb;
    const size_t Bm = (size_t)B * h->m;
    // x then lambda: pack the rows into the staging buffer, then transpose
    // into the instance-fastest layout (instances >= nb get 0)
    for (int part = 0; part < 2; ++part) {
        if (!(parts & (1 << part))) {  // this half of the prediction is not used: zero
            const size_t ts = h->o.precision == UV_MIXED ? 4 : 8;
            if (part == 0) UV_FTRY(hipMemsetAsync(h->X, 0, ts * (size_t)B * h->n, st));
            else UV_FTRY(hipMemsetAsync(h->LAM, 0, 8 * (size_t)B * h->m, st));
            continue;
        }
        const int len = part == 0 ? h->n : h->m;
        const int off = part == 0 ? 0 : h->n;
        float *stg = (float *)h->stage;
        UV_FTRY(hipMemcpy2DAsync(stg, sizeof(float) * len, xl_dev + off, sizeof(float) * ld, sizeof(float) * len, nb,
                                 hipMemcpyDeviceToDevice, st));
        const unsigned g = blocks_for((int64_t)len * B, 256);
        if (part == 0) {
            if (h->o.precision == UV_MIXED) k_fam_to_dev<float, float><<<g, 256, 0, st>>>(len, B, nb, stg, (float *)h->X);
            else k_fam_to_dev<float, double><<<g, 256, 0, st>>>(len, B, nb, stg, (double *)h->X);
        } else {
            k_fam_to_dev<float, double><<<g, 256, 0, st>>>(len, B, nb, stg, h->LAM);
        }
        UV_FTRY(hipGetLastError());
        UV_FTRY(hipStreamSynchronize(st));
    }
    const int ng = B / 64;
    const double im = 1.0 / h->o.mu;
    if (h->o.precision == UV_MIXED) {
        k_fam_dual_start<float><<<blocks_for((int64_t)h->n * ng, 4), 256, 0, st>>>(
            h->n, B, h->cp, h->ri, h->vc64, h->LAM, h->c64, (const float *)h->X, (float *)h->Z, h->D);
        k_fam_start<float><<<blocks_for(Bm, 256), 256, 0, st>>>(Bm, h->LAM, (float *)h->U, im);
    } else {
        k_fam_dual_start<double><<<blocks_for((int64_t)h->n * ng, 4), 256, 0, st>>>(
            h->n, B, h->cp, h->ri, h->vc64, h->LAM, h->c64, (const double *)h->X, (double *)h->Z, h->D);
        k_fam_start<double><<<blocks_for(Bm, 256), 256, 0, st>>>(Bm, h->LAM, (double *)h->U, im);
    }
    k_fam_reset<<<1, 1024, 0, st>>>(h->B, h->nb, h->inst, h->sh, h->BV64);
    h->refilled = false;
    UV_FTRY(hipGetLastError());
    return fam_sync(h);
}

int family_refill(uv_family *h, int32_t count, const int32_t *slots, const double *b, const float *xl_dev,
                  int64_t ld, int32_t parts)
{
    if (!h || count < 0 || (count > 0 && (!slots || !b))) return UV_EINVAL;
    if (count == 0) return UV_OK;
    if (count > h->nb || (xl_dev && (ld < (int64_t)h->n + h->m || parts < 1 || parts > 3))) return UV_EINVAL;
    std::vector<char> seen(h->B, 0);
    for (int q = 0; q < count; ++q) {
        const int sl = slots[q];
        if (sl < 0 || sl >= h->nb || seen[sl] || h->inst_host[sl].status == UV_STATUS_RUNNING) return UV_EINVAL;
        seen[sl] = 1;
    }
    hipStream_t st = h->stream;
    const int B = h->B, m = h->m, n = h->n;
    const bool mixed = h->o.precision == UV_MIXED;
    const double im = 1.0 / h->o.mu;
    UV_FTRY(hipMemcpyAsync(h->slots, slots, sizeof(int) * count, hipMemcpyHostToDevice, st));
    // b rows through the staging buffer (count <= B rows of m doubles)
    UV_FTRY(hipMemcpyAsync(h->stage, b, sizeof(double) * (size_t)count * m, hipMemcpyHostToDevice, st));
    const unsigned gm = blocks_for((int64_t)count * m, 256), gn = blocks_for((int64_t)count * n, 256);
    const unsigned gx = blocks_for((int64_t)count * (n + m), 256);
    if (mixed) {
        k_fam_slot_rhs<float><<<gm, 256, 0, st>>>(m, B, count, h->slots, h->stage, (float *)h->BV, h->BV64);
        k_fam_slot_xl<float><<<gx, 256, 0, st>>>(n, m, B, count, h->slots, xl_dev, ld, parts, (float *)h->X, h->LAM);
        k_fam_slot_zd<float><<<gn, 256, 0, st>>>(n, B, count, h->slots, h->cp, h->ri, h->vc64, h->LAM, h->c64,
                                                 (const float *)h->X, (float *)h->Z, h->D, xl_dev ? 0 : 1);
        k_fam_slot_u<float><<<gm, 256, 0, st>>>(m, B, count, h->slots, h->LAM, (float *)h->U, im);
    } else {
        k_fam_slot_rhs<double><<<gm, 256, 0, st>>>(m, B, count, h->slots, h->stage, (double *)h->BV, h->BV64);
        k_fam_slot_xl<double><<<gx, 256, 0, st>>>(n, m, B, count, h->slots, xl_dev, ld, parts, (double *)h->X,
                                                  h->LAM);
        k_fam_slot_zd<double><<<gn, 256, 0, st>>>(n, B, count, h->slots, h->cp, h->ri, h->vc64, h->LAM, h->c64,
                                                  (const double *)h->X, (double *)h->Z, h->D, xl_dev ? 0 : 1);
        k_fam_slot_u<double><<<gm, 256, 0, st>>>(m, B, count, h->slots, h->LAM, (double *)h->U, im);
    }
    // ||b||^2 of every slot again (same fixed order as at set_rhs; the
    // check's row partials serve as scratch)
    k_fam_bnorm_part<<<blocks_for((int64_t)kBChunks * B, 256), 256, 0, st>>>(m, B, h->BV64, h->prow);
    k_fam_bnorm<<<1, 1024, 0, st>>>(B, h->prow, h->inst);
    k_fam_slot_reset<<<1, 1024, 0, st>>>(B, count, h->slots, h->inst, h->sh);
    UV_FTRY(hipGetLastError());
    h->refilled = true;
    return fam_sync(h);
}

int family_iterate(uv_family *h, int64_t k, int32_t *n_active)
{
    if (!h || k < 0) return UV_EINVAL;
    if (h->sh_host->active > 0) {
        // without refills every member started at family iteration 0, so
        // max_iter caps the family's count (the last check falls on it);
        // after a refill the cap is each member's, applied at the checks
        const bool cap = h->o.max_iter > 0 && !h->refilled;
        int64_t left = k;
        if (cap) left = std::min<int64_t>(left, h->o.max_iter - h->host_iter);
        int64_t it = h->host_iter, since = 0;
        const int ce = h->o.check_every;
        const int64_t look = 50 * (int64_t)ce;  // read the active count every 50 checks
        while (left > 0) {
            if (h->exec && it % ce == 0 && left >= ce) {
                UV_FTRY(hipGraphLaunch(h->exec, h->stream));
                it += ce;
                left -= ce;
                since += ce;
            } else {
                fam_iteration(h, h->stream, (it + 1) % ce == 0 || (cap && it + 1 >= h->o.max_iter));
                it += 1;
                left -= 1;
                since += 1;
            }
            if (left > 0 && since >= look) {  // stop launching once every member has stopped
                UV_FTRY(hipGetLastError());
                int rc = fam_sync(h);
                if (rc != UV_OK) return rc;
                if (h->sh_host->active == 0) break;
                since = 0;
            }
        }
        UV_FTRY(hipGetLastError());
        int rc = fam_sync(h);
        if (rc != UV_OK) return rc;
    }
    if (n_active) *n_active = h->sh_host->active;
    return UV_OK;
}

int family_residuals(uv_family *h, uv_residuals *r)
{
    if (!h || !r) return UV_EINVAL;
    int rc = UV_OK;
    for (int l = 0; l < h->nb; ++l) {
        const FInst &I = h->inst_host[l];
        r[l].r_prim = I.r_prim;
        r[l].r_dual = I.r_dual;
        r[l].r_gap = I.r_gap;
        r[l].kkt = I.kkt;
        r[l].pobj = I.pobj;
        r[l].dobj = I.dobj;
        r[l].res_ax_b = I.res_ax_b;
        r[l].prim_inf = r[l].dual_inf = r[l].scale_p = r[l].scale_d = 0.0;
        r[l].pobj_x = r[l].gap_x = 0.0;
        r[l].iter = I.status == UV_STATUS_RUNNING ? h->host_iter - I.iter0 : I.iter;
        r[l].status = I.status;
        if (I.status == UV_STATUS_NUMERIC) rc = UV_ENUMERIC;
    }
    return rc;
}

int family_solution(uv_family *h, double *x, double *z, double *lambda, double *delta)
{
    if (!h || h->nb < 1) return UV_EINVAL;
    hipStream_t st = h->stream;
    const int B = h->B, nb = h->nb;
    const bool mixed = h->o.precision == UV_MIXED;
    auto get = [&](double *dst, const void *src, int len, bool f64) -> int {
        if (!dst) return UV_OK;
        const unsigned g = blocks_for((int64_t)len * nb, 256);
        if (f64 || !mixed)
            k_fam_from_dev<double, double><<<g, 256, 0, st>>>(len, B, nb, (const double *)src, h->stage, (size_t)len, 0);
        else
            k_fam_from_dev<float, double><<<g, 256, 0, st>>>(len, B, nb, (const float *)src, h->stage, (size_t)len, 0);
        if (hipMemcpyAsync(dst, h->stage, 8 * (size_t)len * nb, hipMemcpyDeviceToHost, st) != hipSuccess) return UV_EHIP;
        return hipStreamSynchronize(st) == hipSuccess ? UV_OK : UV_EHIP;
    };
    int rc;
    if ((rc = get(x, h->X, h->n, false)) != UV_OK) return rc;
    if ((rc = get(z, h->Z, h->n, false)) != UV_OK) return rc;
    if ((rc = get(lambda, h->LAM, h->m, true)) != UV_OK) return rc;
    if ((rc = get(delta, h->D, h->n, true)) != UV_OK) return rc;
    return UV_OK;
}

int family_member_state(uv_family *h, int32_t slot, double *x, double *z, double *lambda, double *delta)
{
    if (!h || slot < 0 || slot >= h->nb) return UV_EINVAL;
    hipStream_t st = h->stream;
    const bool mixed = h->o.precision == UV_MIXED;
    auto get = [&](double *dst, const void *src, int len, bool f64) -> int {
        if (!dst) return UV_OK;
        const unsigned g = blocks_for(len, 256);
        if (f64 || !mixed)
            k_fam_slot_from_dev<double><<<g, 256, 0, st>>>(len, h->B, slot, (const double *)src, h->stage);
        else
            k_fam_slot_from_dev<float><<<g, 256, 0, st>>>(len, h->B, slot, (const float *)src, h->stage);
        if (hipMemcpyAsync(dst, h->stage, 8 * (size_t)len, hipMemcpyDeviceToHost, st) != hipSuccess) return UV_EHIP;
        return hipStreamSynchronize(st) == hipSuccess ? UV_OK : UV_EHIP;
    };
    int rc;
    if ((rc = get(x, h->X, h->n, false)) != UV_OK) return rc;
    if ((rc = get(z, h->Z, h->n, false)) != UV_OK) return rc;
    if ((rc = get(lambda, h->LAM, h->m, true)) != UV_OK) return rc;
    if ((rc = get(delta, h->D, h->n, true)) != UV_OK) return rc;
    return UV_OK;
}

int family_solution_device(uv_family *h, float *dst_dev, int64_t ld)
{
    // instance-major FP32 rows [z (n) ; lambda (m)] into a device matrix
    if (!h || !dst_dev || h->nb < 1 || ld < (int64_t)h->n + h->m) return UV_EINVAL;
    hipStream_t st = h->stream;
    const int B = h->B, nb = h->nb;
    unsigned g = blocks_for((int64_t)h->n * nb, 256);
    if (h->o.precision == UV_MIXED)
        k_fam_from_dev<float, float><<<g, 256, 0, st>>>(h->n, B, nb, (const float *)h->Z, dst_dev, (size_t)ld, 0);
    else
        k_fam_from_dev<double, float><<<g, 256, 0, st>>>(h->n, B, nb, (const double *)h->Z, dst_dev, (size_t)ld, 0);
    g = blocks_for((int64_t)h->m * nb, 256);
    k_fam_from_dev<double, float><<<g, 256, 0, st>>>(h->m, B, nb, h->LAM, dst_dev, (size_t)ld, h->n);
    UV_FTRY(hipGetLastError());
    UV_FTRY(hipStreamSynchronize(st));
    return UV_OK;
}

}  // extern "C"
