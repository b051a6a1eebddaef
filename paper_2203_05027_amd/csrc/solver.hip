// solver.hip -- single-problem UV-decomposition ADMM on gfx950.
//
// The iteration is Algorithm 1's repeat block (Section IV) in a reduced form
// that stores no per-nonzero vectors.  The y-step's optimality condition and
// the two dual updates of lambda and gamma give U'lambda + gamma = 0 after
// every iteration, so with gamma = -U'lambda:
//   * U y - b = F_U (A x - b)           -> lambda <- lambda + mu F_U (A x - b)
//   * V(y + gamma/mu) = N x + A'u,  u = F_U (b - A x) - lambda/mu
// where N = V V' (column counts) and F_U = (I + U U')^{-1} (U U' = squared
// row norms).  Hence one iteration is
//   column pass (CSC):  p = N x + A'u;  x = F_V (p + z + delta/mu - c/mu);
//                       z = proj_K(x - delta/mu);  delta += mu (z - x)
//   row pass    (CSR):  q = A x;  e = F_U (b - q);  lambda -= mu e;
//                       u = e - lambda/mu
// The first column pass after a start (x0, lambda0) needs
// V(y0 + gamma0/mu) with y0 = V'x0, gamma0 = -U'lambda0, which is N x0 + A'u
// with u = -lambda0/mu; a start therefore only sets x and u.
//
// Residual checks (Section V-B, SCS form; see uvadmm.h) reduce in FP64 into
// per-workgroup partials that one workgroup then adds in a fixed order, so
// every run is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/uvadmm.h"
#include "common.hpp"
#include "setup.hpp"
#include "spmv.hpp"

using uv::kWG;

namespace {

// Device-side status, copied to pinned host memory after every call.
struct DevStatus {
    double r_prim, r_dual, r_gap, kkt, pobj, dobj, res_ax_b;
    double bnorm2, cnorm2;
    double prim_inf, dual_inf, scale_p, scale_d;  // infinity-norm measures
    double binf, cinf;
    double pobj_x, gap_x;  // c'x and |c'x + b'lambda| (the POGS-form test)
    long long iter;        // iterations done
    long long check_iter;  // iteration count at the last residual evaluation
    long long hist_n;      // checks recorded in the residual history since the start
    unsigned long long clock0;  // GPU wall clock at the start
    int done;              // 1 = stop: every sweep kernel returns at once
    int status;            // UV_STATUS_*
    int skip_col;          // 1: the last check's primal part failed, its column part is skipped
};

// One record of the residual history (a check of the iteration), as kept on
// the device: the iteration, the GPU wall clock and the residuals.
struct HistRec {
    long long iter;
    unsigned long long clock;
    double r_prim, r_dual, r_gap, kkt, pobj, dobj, res_ax_b, gap_x;
};

// Ring of the last `cap` records (rec null: no history kept).
struct HistRing {
    HistRec *rec;
    int cap;
};

constexpr int kSocTile = 256;  // columns per SOC tile when cones are small

// ||b||^2 and ||c||^2 in FP64 (one workgroup, fixed order).
__global__ void __launch_bounds__(kWG)
k_norms(int m, const double *__restrict__ b, int n, const double *__restrict__ c, DevStatus *st)
{
    double v[2] = {0.0, 0.0}, w[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < m; i += kWG) {
        v[0] += b[i] * b[i];
        w[0] = fmax(w[0], fabs(b[i]));
    }
    for (int j = threadIdx.x; j < n; j += kWG) {
        v[1] += c[j] * c[j];
        w[1] = fmax(w[1], fabs(c[j]));
    }
    double out[4];
    uv::block_sum_max<2, 2>(v, w, out, 1);
    if (threadIdx.x == 0) {
        st->bnorm2 = out[0];
        st->cnorm2 = out[1];
        st->binf = out[2];
        st->cinf = out[3];
    }
}

// Start: u = -lambda/mu (see the header comment), iteration state reset.
template <typename T>
__global__ void __launch_bounds__(kWG)
k_start(int m, const double *__restrict__ lam, T *__restrict__ u, double inv_mu, DevStatus *st)
{
    int i = blockIdx.x * kWG + threadIdx.x;
    if (i < m) u[i] = (T)(-lam[i] * inv_mu);
    if (i == 0) {
        st->iter = 0;
        st->check_iter = -1;
        st->hist_n = 0;
        st->clock0 = wall_clock64();
        st->done = 0;
        st->status = UV_STATUS_RUNNING;
        st->skip_col = 0;
    }
}

// ---------------------------------------------------------------------------
// Sweep kernels
// ---------------------------------------------------------------------------

// Dot product of one sparse row/column segment [beg, end) with a gathered
// vector: L lanes cooperate, lane-strided, and each lane issues E index and
// value loads and then E gathers before it accumulates, so E gathers per
// lane are in flight at once (the sweep is bound by gather latency, not by
// arithmetic).  Slots past the segment's end reload its last entry (a cache
// hit) and add zero, which keeps the loop free of divergent branches.  The
// streamed index and value arrays are read with non-temporal loads so they
// do not evict the gathered vector from the caches.
template <int L, int E, typename T, typename TV>
__device__ __forceinline__ T seg_dot(int beg, int end, int lane, const int *__restrict__ idx,
                                     const TV *__restrict__ val, const T *__restrict__ vec)
{
    T acc = 0;
    for (int base = beg + lane; base < end; base += L * E) {
        int j[E];
        TV v[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int k = base + e * L;
            const int kk = k < end ? k : end - 1;
            j[e] = __builtin_nontemporal_load(idx + kk);
            v[e] = __builtin_nontemporal_load(val + kk);
        }
        T g[E];
#pragma unroll
        for (int e = 0; e < E; ++e) g[e] = vec[j[e]];
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (base + e * L < end) acc += (T)v[e] * g[e];
    }
    return uv::group_sum<L>(acc);
}

// Row pass.  MODE 0: iterate.  MODE 1: iterate and gather z for the
// residual partials (||A z - b||^2, b'lambda, ||A x - b||^2) of the new
// lambda.  MODE 2 (resume): u = F_U (b - A x) - lambda/mu with lambda kept,
// which is the u an iteration leaves behind at this (x, lambda).
template <typename T, int L, int E, int MODE>
__global__ void __launch_bounds__(kWG)
k_row(int m, const int *__restrict__ rp, const int *__restrict__ ci, const T *__restrict__ va,
      const T *__restrict__ x, const T *__restrict__ z, const T *__restrict__ b, const T *__restrict__ fu,
      double *__restrict__ lam, T *__restrict__ u, double mu, double inv_mu, double *__restrict__ part,
      int pstride, DevStatus *st)
{
    if (MODE != 2 && st->done) return;
    const int lane = threadIdx.x & (L - 1);
    const int row = blockIdx.x * (kWG / L) + threadIdx.x / L;
    double acc[3] = {0.0, 0.0, 0.0}, mx[2] = {0.0, 0.0};
    if (row < m) {
        // epilogue operands first: independent of the gathers below
        const T bi = b[row], fi = fu[row];
        const double l0 = lam[row];
        const int beg = rp[row], end = rp[row + 1];
        const T q = seg_dot<L, E>(beg, end, lane, ci, va, x);
        T qz = 0;
        if (MODE == 1) qz = seg_dot<L, E>(beg, end, lane, ci, va, z);
        if (lane == 0) {
            const T e = fi * (bi - q);
            const double li = (MODE == 2) ? l0 : l0 - mu * (double)e;
            if (MODE != 2) lam[row] = li;
            u[row] = (T)((double)e - li * inv_mu);
            if (MODE == 1) {
                double rz = (double)qz - (double)bi, rx = (double)q - (double)bi;
                acc[0] = rz * rz;
                acc[1] = (double)bi * li;
                acc[2] = rx * rx;
                mx[0] = fabs(rz);
                mx[1] = fabs((double)qz);
            }
        }
    }
    if (MODE != 2 && blockIdx.x == 0 && threadIdx.x == 0) st->iter += 1;
    if (MODE == 1) uv::block_sum_max<3, 2>(acc, mx, part + blockIdx.x, pstride);
}

// Residual-only row pass with FP64 values of A (same partial layout as the
// MODE 1 row pass, with the row pass's lane count).
template <typename T, int L>
__global__ void __launch_bounds__(kWG)
k_res_row(int m, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ va,
          const T *__restrict__ x, const T *__restrict__ z, const double *__restrict__ b,
          const double *__restrict__ lam, double *__restrict__ part, int pstride)
{
    const int lane = threadIdx.x & (L - 1);
    const int row = blockIdx.x * (kWG / L) + threadIdx.x / L;
    double acc[3] = {0.0, 0.0, 0.0}, mx[2] = {0.0, 0.0};
    if (row < m) {
        const double bi = b[row], li = lam[row];
        const int beg = rp[row], end = rp[row + 1];
        double qx = 0.0, qz = 0.0;
        constexpr int E = 4;  // entries per lane with their gathers in flight
        for (int base = beg + lane; base < end; base += L * E) {
            int j[E];
            double v[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = base + e * L;
                const int kk = k < end ? k : end - 1;
                j[e] = ci[kk];
                v[e] = va[kk];
            }
            T gx[E], gz[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                gx[e] = x[j[e]];
                gz[e] = z[j[e]];
            }
#pragma unroll
            for (int e = 0; e < E; ++e) {
                if (base + e * L < end) {
                    qx += v[e] * (double)gx[e];
                    qz += v[e] * (double)gz[e];
                }
            }
        }
        qx = uv::group_sum<L>(qx);
        qz = uv::group_sum<L>(qz);
        if (lane == 0) {
            acc[0] = (qz - bi) * (qz - bi);
            acc[1] = bi * li;
            acc[2] = (qx - bi) * (qx - bi);
            mx[0] = fabs(qz - bi);
            mx[1] = fabs(qz);
        }
    }
    uv::block_sum_max<3, 2>(acc, mx, part + blockIdx.x, pstride);
}

// x-step (Block 1) for one column from p = N x + A'u, and the projected
// point v = x - delta/mu.
template <typename T>
__device__ __forceinline__ T x_step(int cnt, T xo, T zo, T atu, T dm, T cj, double inv_mu)
{
    const T p = (T)cnt * xo + atu;
    return (p + zo + dm - cj * (T)inv_mu) / (T)(1 + cnt);
}

// A'u for column col: the L-lane segment product over the column (S == 1)
// or the tree sum of the S slab partials P[s * n + col] (S > 1).
template <int L, int E, int S, typename T>
__device__ __forceinline__ T col_atu(int col, int beg, int end, int lane, const int *__restrict__ ri,
                                     const T *__restrict__ vc, const T *__restrict__ u, const T *__restrict__ P,
                                     int n)
{
    if (S == 1) return seg_dot<L, E>(beg, end, lane, ri, vc, u);
    return slab_tree_sum<S>(P, n, col);
}

// x-step, projection onto the orthant and delta update of one column.
template <typename T>
__device__ __forceinline__ void orth_step(int col, int cnt, T xo, T zo, T cj, double d, T atu, T *__restrict__ x,
                                          T *__restrict__ z, double *__restrict__ delta, double mu, double inv_mu)
{
    const T dm = (T)(d * inv_mu);
    const T xn = x_step<T>(cnt, xo, zo, atu, dm, cj, inv_mu);
    const T v = xn - dm;
    const T zn = v > (T)0 ? v : (T)0;
    x[col] = xn;
    z[col] = zn;
    delta[col] = d + mu * ((double)zn - (double)xn);
}

// Column pass over the orthant columns [0, n_orth).
template <typename T, int L, int E, int S>
__global__ void __launch_bounds__(kWG)
k_col_orth(int n_orth, const int *__restrict__ cp, const int *__restrict__ ri, const T *__restrict__ vc,
           const T *__restrict__ u, T *__restrict__ x, T *__restrict__ z, double *__restrict__ delta,
           const T *__restrict__ c, double mu, double inv_mu, const T *__restrict__ P, int n, const DevStatus *st)
{
    if (st->done) return;
    const int lane = threadIdx.x & (L - 1);
    const int col = blockIdx.x * (kWG / L) + threadIdx.x / L;
    if (col >= n_orth) return;   // whole L-lane groups leave together
    const T xo = x[col], zo = z[col], cj = c[col];
    const double d = delta[col];
    const int beg = cp[col], end = cp[col + 1];
    const T atu = col_atu<L, E, S>(col, beg, end, lane, ri, vc, u, P, n);
    if (lane == 0) orth_step<T>(col, end - beg, xo, zo, cj, d, atu, x, z, delta, mu, inv_mu);
}

// Column pass over second-order cones.  Workgroup t owns whole cones
// [tcone[t], tcone[t+1]) = columns [tcol[t], tcol[t+1]) (at most TC
// columns): phase 1 computes x and v = x - delta/mu per column into LDS,
// phase 2 takes each cone's tail norm (a wavefront per cone) and its
// projection case (eq. proj), phase 3 writes x, z and delta.
template <typename T, int L, int E, int TC, int S>
__global__ void __launch_bounds__(kWG)
k_col_soc(const int *__restrict__ tcol, const int *__restrict__ tcone, const int *__restrict__ soc_off,
          const int *__restrict__ cp, const int *__restrict__ ri, const T *__restrict__ vc,
          const T *__restrict__ u, T *__restrict__ x, T *__restrict__ z, double *__restrict__ delta,
          const T *__restrict__ c, double mu, double inv_mu, const T *__restrict__ P, int n, const DevStatus *st)
{
    if (st->done) return;
    __shared__ T sx[TC];
    __shared__ T sv[TC];
    __shared__ double sd[TC];
    __shared__ short sown[TC];
    __shared__ double sa1[TC];
    __shared__ double sbeta[TC];
    __shared__ short shead[TC];

    const int t = blockIdx.x;
    const int c0 = tcol[t], ncols = tcol[t + 1] - c0;
    const int q0 = tcone[t], ncones = tcone[t + 1] - q0;
    const int lane = threadIdx.x & (L - 1);

    for (int jj = threadIdx.x / L; jj < ncols; jj += kWG / L) {
        const int col = c0 + jj;
        const T xo = x[col], zo = z[col], cj = c[col];
        const double d = delta[col];
        const int beg = cp[col], end = cp[col + 1];
        const T atu = col_atu<L, E, S>(col, beg, end, lane, ri, vc, u, P, n);
        if (lane == 0) {
            const T dm = (T)(d * inv_mu);
            const T xn = x_step<T>(end - beg, xo, zo, atu, dm, cj, inv_mu);
            sx[jj] = xn;
            sv[jj] = xn - dm;
            sd[jj] = d;
        }
    }
    __syncthreads();
    // a wavefront per cone: the lanes take the tail's squares 64 apart, then
    // a fixed butterfly adds the lanes' sums
    const int wl = threadIdx.x & 63;
    for (int qi = threadIdx.x >> 6; qi < ncones; qi += kWG / 64) {
        const int s0 = soc_off[q0 + qi] - c0, s1 = soc_off[q0 + qi + 1] - c0;
        double a2 = 0.0;
        for (int j = s0 + 1 + wl; j < s1; j += 64) a2 += (double)sv[j] * (double)sv[j];
        for (int j = s0 + wl; j < s1; j += 64) sown[j] = (short)qi;
        a2 = uv::group_sum<64>(a2);
        if (wl == 0) {
            const double w1 = (double)sv[s0];
            const double alpha = sqrt(a2);
            double a1, beta;
            if (alpha <= -w1) { a1 = 0.0; beta = 0.0; }
            else if (alpha <= w1) { a1 = w1; beta = 1.0; }
            else { a1 = 0.5 * (w1 + alpha); beta = 0.5 * (1.0 + w1 / alpha); }
            sa1[qi] = a1;
            sbeta[qi] = beta;
            shead[qi] = (short)s0;
        }
    }
    __syncthreads();
    for (int jj = threadIdx.x; jj < ncols; jj += kWG) {
        const int qi = sown[jj];
        const T zn = (jj == shead[qi]) ? (T)sa1[qi] : (T)(sbeta[qi] * (double)sv[jj]);
        const T xn = sx[jj];
        const int col = c0 + jj;
        x[col] = xn;
        z[col] = zn;
        delta[col] = sd[jj] + mu * ((double)zn - (double)xn);
    }
}

// Column pass over second-order cones of at most 64 coordinates: a
// wavefront per tile of whole cones (at most 64 columns, one lane per
// column), with no LDS and no workgroup barrier.  Each lane forms x and
// v = x - delta/mu for its column; a segmented scan over the lanes (cone by
// cone, a fixed pattern) leaves each cone's tail sum of squares at its last
// lane, and every lane takes its cone's case of eq. proj from the cone's
// head value and tail norm.  info[j - off0] = (position of column j in its
// cone) | (cone size << 16).
template <typename T, int E, int S>
__global__ void __launch_bounds__(kWG)
k_col_soc_wave(int ntiles, const int *__restrict__ tcol, const int *__restrict__ info, int off0,
               const int *__restrict__ cp, const int *__restrict__ ri, const T *__restrict__ vc,
               const T *__restrict__ u, T *__restrict__ x, T *__restrict__ z, double *__restrict__ delta,
               const T *__restrict__ c, double mu, double inv_mu, const T *__restrict__ P, int n, const DevStatus *st)
{
    if (st->done) return;
    const int t = blockIdx.x * (kWG / 64) + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (t >= ntiles) return;  // the whole wavefront leaves
    const int c0 = tcol[t], w = tcol[t + 1] - c0;
    const int col = c0 + lane;
    const bool act = lane < w;
    T xn = 0, v = 0;
    double d = 0.0;
    int pos = 0, size = 1;
    if (act) {
        const T xo = x[col], zo = z[col], cj = c[col];
        d = delta[col];
        const int beg = cp[col], end = cp[col + 1];
        const T atu = col_atu<1, E, S>(col, beg, end, 0, ri, vc, u, P, n);
        const T dm = (T)(d * inv_mu);
        xn = x_step<T>(end - beg, xo, zo, atu, dm, cj, inv_mu);
        v = xn - dm;
        const int in = info[col - off0];
        pos = in & 0xffff;
        size = in >> 16;
    }
    const int head = lane - pos, last = head + size - 1;
    double sq = pos > 0 ? (double)v * (double)v : 0.0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {  // inclusive scan within each cone
        const double o = __shfl_up(sq, off);
        const int oh = __shfl_up(head, off);
        if (lane >= off && oh == head) sq += o;
    }
    const double alpha = sqrt(__shfl(sq, last));
    const double w1 = (double)__shfl(v, head);
    double a1, beta;
    if (alpha <= -w1) { a1 = 0.0; beta = 0.0; }
    else if (alpha <= w1) { a1 = w1; beta = 1.0; }
    else { a1 = 0.5 * (w1 + alpha); beta = 0.5 * (1.0 + w1 / alpha); }
    if (act) {
        const T zn = pos == 0 ? (T)a1 : (T)(beta * (double)v);
        x[col] = xn;
        z[col] = zn;
        delta[col] = d + mu * ((double)zn - (double)xn);
    }
}

// XCD-local slab passes.  The gathered vector (x in the row pass, u in the
// column pass) is cut into S contiguous slabs and the matrix into the
// matching slab-major copies; workgroup w works on slab w % S, so with the
// round-robin workgroup-to-XCD dispatch each XCD only gathers from 1/S of
// the vector (at most a few MiB, resident in its L2), and writes one partial
// per row (column) and slab.  The update kernels add the S partials in slab
// order, so the result is deterministic.
template <typename T, int L, int E, int S, bool CHECK>
__global__ void __launch_bounds__(kWG)
k_row_slab(int m, const int *__restrict__ srp, const int *__restrict__ sci, const T *__restrict__ sva,
           const T *__restrict__ x, const T *__restrict__ z, T *__restrict__ P, int ignore_done,
           const DevStatus *st)
{
    if (!ignore_done && st->done) return;
    const int sl = blockIdx.x % S, t = blockIdx.x / S;
    const int lane = threadIdx.x & (L - 1);
    const int row = t * (kWG / L) + threadIdx.x / L;
    if (row >= m) return;
    const int beg = srp[(size_t)sl * m + row], end = srp[(size_t)sl * m + row + 1];
    const T q = seg_dot<L, E>(beg, end, lane, sci, sva, x);
    T qz = 0;
    if (CHECK) qz = seg_dot<L, E>(beg, end, lane, sci, sva, z);
    if (lane == 0) {
        P[(size_t)sl * m + row] = q;
        if (CHECK) P[(size_t)(S + sl) * m + row] = qz;
    }
}

// Block-2 update of one row from q = (A x)_row: e = F_U (b - q), lambda and
// u; MODE 1 adds the row residual terms from qd (A x in FP64) and the FP64
// partials of A z.
template <typename T, int S, int MODE>
__device__ __forceinline__ void row_step(int row, int m, T q, double qd, const double *__restrict__ Pz,
                                         const T *__restrict__ b,
                                         const double *__restrict__ b64, const T *__restrict__ fu,
                                         double *__restrict__ lam, T *__restrict__ u, double mu, double inv_mu,
                                         double (&acc)[3], double (&mx)[2])
{
    const T bi = b[row], fi = fu[row];
    const double l0 = lam[row];
    const T e = fi * (bi - q);
    const double li = (MODE == 2) ? l0 : l0 - mu * (double)e;
    if (MODE != 2) lam[row] = li;
    u[row] = (T)((double)e - li * inv_mu);
    if (MODE == 1) {
        double qz = 0.0;
#pragma unroll
        for (int sl = 0; sl < S; ++sl) qz += Pz[(size_t)sl * m + row];
        const double bd = b64[row];
        const double rz = qz - bd, rx = qd - bd;
        acc[0] = rz * rz;
        acc[1] = bd * li;
        acc[2] = rx * rx;
        mx[0] = fabs(rz);
        mx[1] = fabs(qz);
    }
}

// Row update from slab partials P (type TP); the MODEs of k_row.  MODE 1
// also forms the row residual partials: a check's products of A x and A z
// are both FP64 (FP64 values of A, FP64 sums, TP = double in both
// precisions), and the mixed form's iteration goes on from A x rounded to
// FP32.
template <typename T, typename TP, int S, int MODE>
__global__ void __launch_bounds__(kWG)
k_row_combine(int m, const TP *__restrict__ P, const double *__restrict__ Pz, const T *__restrict__ b,
              const double *__restrict__ b64, const T *__restrict__ fu, double *__restrict__ lam, T *__restrict__ u,
              double mu, double inv_mu, double *__restrict__ part, int pstride, DevStatus *st)
{
    if (MODE != 2 && st->done) return;
    const int row = blockIdx.x * kWG + threadIdx.x;
    double acc[3] = {0.0, 0.0, 0.0}, mx[2] = {0.0, 0.0};
    if (row < m) {
        const TP q = slab_tree_sum<S>(P, m, row);
        row_step<T, S, MODE>(row, m, (T)q, (double)q, Pz, b, b64, fu, lam, u, mu, inv_mu, acc, mx);
    }
    if (MODE != 2 && blockIdx.x == 0 && threadIdx.x == 0) st->iter += 1;
    if (MODE == 1) uv::block_sum_max<3, 2>(acc, mx, part + blockIdx.x, pstride);
}

template <typename T, int L, int E, int S>
__global__ void __launch_bounds__(kWG)
k_col_slab(int n, const int *__restrict__ scp, const int *__restrict__ sri, const T *__restrict__ svc,
           const T *__restrict__ u, T *__restrict__ P, const DevStatus *st)
{
    if (st->done) return;
    const int sl = blockIdx.x % S, t = blockIdx.x / S;
    const int lane = threadIdx.x & (L - 1);
    const int col = t * (kWG / L) + threadIdx.x / L;
    if (col >= n) return;
    const T a = seg_dot<L, E>(scp[(size_t)sl * n + col], scp[(size_t)sl * n + col + 1], lane, sri, svc, u);
    if (lane == 0) P[(size_t)sl * n + col] = a;
}

// Residual-only column pass: ||A'lambda + c - delta||^2, c'z and c'x
// partials, FP64 values of A.
template <typename T, int L>
__global__ void __launch_bounds__(kWG)
k_res_col(int n, const int *__restrict__ cp, const int *__restrict__ ri, const double *__restrict__ vc,
          const double *__restrict__ lam, const double *__restrict__ c, const double *__restrict__ delta,
          const T *__restrict__ z, const T *__restrict__ x, double *__restrict__ part, int pstride, const int *skip)
{
    if (skip && *skip) return;  // the check's column half is ruled out (uniform)
    const int lane = threadIdx.x & (L - 1);
    const int col = blockIdx.x * (kWG / L) + threadIdx.x / L;
    double acc[3] = {0.0, 0.0, 0.0}, mx[2] = {0.0, 0.0};
    if (col < n) {
        const double cj = c[col], dj = delta[col], zj = (double)z[col], xj = (double)x[col];
        const double a = seg_dot<L, 4>(cp[col], cp[col + 1], lane, ri, vc, lam);
        if (lane == 0) {
            const double r = a + cj - dj;
            acc[0] = r * r;
            acc[1] = cj * zj;
            acc[2] = cj * xj;
            mx[0] = fabs(r);
            mx[1] = fabs(a);
        }
    }
    uv::block_sum_max<3, 2>(acc, mx, part + blockIdx.x, pstride);
}

// Column residual partials from the slab partials of A'lambda (FP64 slab
// copy): the layout of k_res_col, one thread per column.
template <typename T, int S>
__global__ void __launch_bounds__(kWG)
k_res_col_slab(int n, const double *__restrict__ P, const double *__restrict__ c, const double *__restrict__ delta,
               const T *__restrict__ z, const T *__restrict__ x, double *__restrict__ part, int pstride,
               const int *skip)
{
    if (skip && *skip) return;  // the check's column half is ruled out (uniform)
    const int col = blockIdx.x * kWG + threadIdx.x;
    double acc[3] = {0.0, 0.0, 0.0}, mx[2] = {0.0, 0.0};
    if (col < n) {
        double a = 0.0;
#pragma unroll
        for (int sl = 0; sl < S; ++sl) a += P[(size_t)sl * n + col];
        const double cj = c[col];
        const double r = a + cj - delta[col];
        acc[0] = r * r;
        acc[1] = cj * (double)z[col];
        acc[2] = cj * (double)x[col];
        mx[0] = fabs(r);
        mx[1] = fabs(a);
    }
    uv::block_sum_max<3, 2>(acc, mx, part + blockIdx.x, pstride);
}

// The stopping test of a check from its sums and maxima: s[0] ||Az-b||^2,
// s[1] b'lambda, s[2] ||Ax-b||^2, s[3] ||A'lambda+c-delta||^2, s[4] c'z,
// s[5] c'x, s[6] ||Az-b||_inf, s[7] ||Az||_inf, s[8]
// ||A'lambda+c-delta||_inf, s[9] ||A'lambda||_inf; nrm: ||b||^2, ||c||^2,
// ||b||_inf, ||c||_inf; it: the iteration count they belong to.  Records
// the residuals in st and, with decide, the status and the stop flag (and a
// record in the residual history); returns whether the run stops here.  One
// thread.
__device__ bool finish_check(const double (&s)[10], const double (&nrm)[4], long long it, double eps,
                             double eps_abs, double eps_gap, int crit, int decide, DevStatus *st, HistRing hist)
{
    const double rp = sqrt(s[0]) / (1.0 + sqrt(nrm[0]));
    const double rd = sqrt(s[3]) / (1.0 + sqrt(nrm[1]));
    const double cz = s[4], bl = s[1], cx = s[5];
    const double rg = fabs(cz + bl) / (1.0 + fabs(cz) + fabs(bl));
    const double kkt = uv::kkt_of(rp, rd, rg);
    const double res_ax_b = sqrt(s[2]), gap_x = fabs(cx + bl);
    st->r_prim = rp;
    st->r_dual = rd;
    st->r_gap = rg;
    st->kkt = kkt;
    st->pobj = cz;
    st->dobj = -bl;
    st->res_ax_b = res_ax_b;
    st->prim_inf = s[6];
    st->dual_inf = s[8];
    const double scale_p = fmax(s[7], nrm[2]), scale_d = fmax(s[9], nrm[3]);
    st->scale_p = scale_p;
    st->scale_d = scale_d;
    st->pobj_x = cx;
    st->gap_x = gap_x;
    st->check_iter = it;
    if (!decide) return false;
    if (hist.rec) {  // the checks of the iteration go into the residual history
        HistRec &h = hist.rec[st->hist_n % hist.cap];
        h.iter = it;
        h.clock = wall_clock64();
        h.r_prim = rp;
        h.r_dual = rd;
        h.r_gap = rg;
        h.kkt = kkt;
        h.pobj = cz;
        h.dobj = -bl;
        h.res_ax_b = res_ax_b;
        h.gap_x = gap_x;
        st->hist_n += 1;
    }
    // crit 1 adds the gap condition when eps_gap > 0; crit 2 is the POGS
    // form (strict inequalities as printed)
    bool conv;
    if (crit == 1)
        conv = s[6] <= eps_abs + eps * scale_p && s[8] <= eps_abs + eps * scale_d &&
               (eps_gap <= 0.0 || gap_x < eps_gap);
    else if (crit == 2)
        conv = res_ax_b < eps_abs && gap_x < eps_gap;
    else
        conv = kkt <= eps;
    if (!isfinite(kkt)) {
        st->status = UV_STATUS_NUMERIC;
        st->done = 1;
        return true;
    }
    if (conv) {
        st->status = UV_STATUS_CONVERGED;
        st->done = 1;
        return true;
    }
    return false;
}

// Adds the partials in a fixed order (eight independent loads in flight
// per thread), forms the residuals and decides whether to stop.  Partials
// are stored component-major: prow[k * nrow + block], rows: sums of
// (Az-b)^2, b'lambda, (Ax-b)^2, then maxima of |Az-b|, |Az|; columns: sums of
// (A'lambda+c-delta)^2, c'z, c'x, then maxima of |A'lambda+c-delta|,
// |A'lambda|.  crit 0: relative KKT (SCS form) <= eps; crit 1: infinity-norm
// test ||Az-b|| <= eps_abs + eps max(||Az||, ||b||) and
// ||A'lambda+c-delta|| <= eps_abs + eps max(||A'lambda||, ||c||), and
// |c'x + b'lambda| < eps_gap when eps_gap > 0; crit 2 (POGS form):
// ||Ax-b||_2 < eps_abs and |c'x + b'lambda| < eps_gap.
// decide 0 only records the values (a residual query between checks): the
// status and the stop flag change at the checks of the iteration alone.
__global__ void __launch_bounds__(kWG)
k_finalize(int nrow, const double *__restrict__ prow, int ncol, const double *__restrict__ pcol,
           double eps, double eps_abs, double eps_gap, int crit, int decide, int gated, DevStatus *st,
           HistRing hist)
{
    if (decide && gated && st->skip_col) return;  // a check that k_row_gate ruled out (uniform)
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, w[4] = {0.0, 0.0, 0.0, 0.0};
    for (int base = threadIdx.x; base < nrow; base += 8 * kWG) {
        double a[5][8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int i = base + r * kWG;
#pragma unroll
            for (int k = 0; k < 5; ++k) a[k][r] = i < nrow ? prow[k * nrow + i] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            v[0] += a[0][r];
            v[1] += a[1][r];
            v[2] += a[2][r];
            w[0] = fmax(w[0], a[3][r]);
            w[1] = fmax(w[1], a[4][r]);
        }
    }
    for (int base = threadIdx.x; base < ncol; base += 8 * kWG) {
        double a[5][8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int i = base + r * kWG;
#pragma unroll
            for (int k = 0; k < 5; ++k) a[k][r] = i < ncol ? pcol[k * ncol + i] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            v[3] += a[0][r];
            v[4] += a[1][r];
            v[5] += a[2][r];
            w[2] = fmax(w[2], a[3][r]);
            w[3] = fmax(w[3], a[4][r]);
        }
    }
    double s[10];
    uv::block_sum_max<6, 4>(v, w, s, 1);
    if (threadIdx.x != 0) return;
    // a check replayed after the run stopped (the rest of a graph launch)
    // repeats the stopping check: it leaves the status, the values and the
    // history as they are
    if (decide && st->done) return;
    const double nrm[4] = {st->bnorm2, st->cnorm2, st->binf, st->cinf};
    finish_check(s, nrm, st->iter, eps, eps_abs, eps_gap, crit, decide, st, hist);
}

// The primal half of a check, before its column half: the row partials
// summed exactly as k_finalize sums them (the same loop and reduction, so
// the values agree bit for bit) and the primal part of the stopping test --
// r_prim <= eps for the KKT test, ||Az-b||_inf <= eps_abs + eps scale_p for
// the infinity-norm test, ||Ax-b|| < eps_abs for the POGS form.  When it
// fails and the row sums are finite the check cannot stop the run, so its
// column half (the A'lambda product, the dual residual, c'z and the gap) is
// skipped: skip_col = 1, which the column kernels and k_finalize read.  A
// check replayed after the run stopped is skipped too.
__global__ void __launch_bounds__(kWG)
k_row_gate(int nrow, const double *__restrict__ prow, double eps, double eps_abs, int crit, DevStatus *st)
{
    double v[3] = {0.0, 0.0, 0.0}, w[2] = {0.0, 0.0};
    for (int base = threadIdx.x; base < nrow; base += 8 * kWG) {
        double a[5][8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int i = base + r * kWG;
#pragma unroll
            for (int k = 0; k < 5; ++k) a[k][r] = i < nrow ? prow[k * nrow + i] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            v[0] += a[0][r];
            v[1] += a[1][r];
            v[2] += a[2][r];
            w[0] = fmax(w[0], a[3][r]);
            w[1] = fmax(w[1], a[4][r]);
        }
    }
    double s[5];
    uv::block_sum_max<3, 2>(v, w, s, 1);
    if (threadIdx.x != 0) return;
    if (st->done) {
        st->skip_col = 1;
        return;
    }
    bool fails;
    if (crit == 1) fails = !(s[3] <= eps_abs + eps * fmax(s[4], st->binf));
    else if (crit == 2) fails = !(sqrt(s[2]) < eps_abs);
    else fails = !(sqrt(s[0]) / (1.0 + sqrt(st->bnorm2)) <= eps);
    const bool finite = isfinite(s[0]) && isfinite(s[1]) && isfinite(s[2]) && isfinite(s[3]) && isfinite(s[4]);
    st->skip_col = fails && finite ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Resident path: a small orthant problem held whole in one workgroup's LDS
// ---------------------------------------------------------------------------

// Byte offsets in the dynamic LDS of k_resident: FP64 delta and lambda, the
// sweep-type iterates x, z, u, the CSC and CSR values, the offsets and the
// 16-bit row and column numbers (m, n < 65536).
struct ResLayout {
    int d, l, x, z, u, vc, va, cp, rp, ri, ci;
    int bytes;
};

constexpr int kResThreads = 1024;
constexpr int kResLdsMax = 160 * 1024 - 2048;  // a CU's LDS less the kernel's static slots

template <typename T>
ResLayout resident_layout(int m, int n, int nnz)
{
    ResLayout L{};
    size_t o = 0;
    auto put = [&](int &field, size_t bytes) {
        field = (int)o;
        o = (o + bytes + 15) / 16 * 16;
    };
    put(L.d, 8 * (size_t)n);
    put(L.l, 8 * (size_t)m);
    put(L.x, sizeof(T) * (size_t)n);
    put(L.z, sizeof(T) * (size_t)n);
    put(L.u, sizeof(T) * (size_t)m);
    put(L.vc, sizeof(T) * (size_t)nnz);
    put(L.va, sizeof(T) * (size_t)nnz);
    put(L.cp, 4 * ((size_t)n + 1));
    put(L.rp, 4 * ((size_t)m + 1));
    put(L.ri, 2 * (size_t)nnz);
    put(L.ci, 2 * (size_t)nnz);
    L.bytes = o > (size_t)INT32_MAX ? INT32_MAX : (int)o;
    return L;
}

// Sum over the entries k0..k1-1 of a row or column held in LDS, split over
// the L lanes of a group (this lane: `lane`), four entries in flight per
// lane, then across the group (the total in every lane).  A fixed order.
template <typename T, typename TV, typename G>
__device__ __forceinline__ T lds_dot(int k0, int k1, int lane, int L, const unsigned short *idx, const TV *val,
                                     const G *vec)
{
    T a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int k = k0 + lane;
    for (; k + 3 * L < k1; k += 4 * L) {
        const int j0 = idx[k], j1 = idx[k + L], j2 = idx[k + 2 * L], j3 = idx[k + 3 * L];
        a0 += (T)val[k] * (T)vec[j0];
        a1 += (T)val[k + L] * (T)vec[j1];
        a2 += (T)val[k + 2 * L] * (T)vec[j2];
        a3 += (T)val[k + 3 * L] * (T)vec[j3];
    }
    for (; k < k1; k += L) a0 += (T)val[k] * (T)vec[idx[k]];
    return uv::lane_sum<T>((a0 + a1) + (a2 + a3), L);
}

// Two sums of lds_dot over the same entries (A z and A x of a check row):
// the indices and values are read once.
template <typename TV, typename G>
__device__ __forceinline__ void lds_dot2(int k0, int k1, int lane, int L, const unsigned short *idx, const TV *val,
                                         const G *v1, const G *v2, double &s1, double &s2)
{
    double a0 = 0.0, a1 = 0.0, b0 = 0.0, b1 = 0.0;
    int k = k0 + lane;
    for (; k + L < k1; k += 2 * L) {
        const int j0 = idx[k], j1 = idx[k + L];
        const double w0 = (double)val[k], w1 = (double)val[k + L];
        a0 += w0 * (double)v1[j0];
        b0 += w0 * (double)v2[j0];
        a1 += w1 * (double)v1[j1];
        b1 += w1 * (double)v2[j1];
    }
    for (; k < k1; k += L) {
        const int j = idx[k];
        const double w = (double)val[k];
        a0 += w * (double)v1[j];
        b0 += w * (double)v2[j];
    }
    s1 = uv::lane_sum<double>(a0 + a1, L);
    s2 = uv::lane_sum<double>(b0 + b1, L);
}

// The FP64 residual check of the resident kernel (every thread calls it):
// per-thread sums over its rows and columns, then a fixed-order workgroup
// reduction; thread 0 gets the sums and maxima of finish_check in sv.
template <typename T>
__device__ __forceinline__ void res_check(int m, int n, int Lr, int Lc, const int *rps, const unsigned short *cis,
                                          const int *cps, const unsigned short *ris, const double *cva,
                                          const double *cvc, const T *xs, const T *zs, const double *ds,
                                          const double *ls, const double *__restrict__ b64,
                                          const double *__restrict__ c64, double (*red)[kResThreads / 64],
                                          double (&sv)[10], const double *gate, int *s_skip)
{
    constexpr int NT = kResThreads;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const int gc = tid / Lc, lc = tid % Lc, gr = tid / Lr, lr = tid % Lr;
    double v[10] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = gr; i < m; i += NT / Lr) {
        double qz, qx;
        lds_dot2(rps[i], rps[i + 1], lr, Lr, cis, cva, zs, xs, qz, qx);
        if (lr == 0) {
            const double bi = b64[i], rz = qz - bi, rx = qx - bi;
            v[0] += rz * rz;
            v[1] += bi * ls[i];
            v[2] += rx * rx;
            v[6] = fmax(v[6], fabs(rz));
            v[7] = fmax(v[7], fabs(qz));
        }
    }
    if (gate) {
        // primal half first (gate: eps, eps_abs, crit, ||b||^2, ||b||_inf):
        // the row values folded as below, bit for bit; when the primal part
        // of the test fails with finite sums the check cannot stop the run
        // and its column half is skipped (*s_skip = 1, sv left unset)
        double g[5] = {uv::wave_fold0<false>(v[0]), uv::wave_fold0<false>(v[1]), uv::wave_fold0<false>(v[2]),
                       uv::wave_fold0<true>(v[6]), uv::wave_fold0<true>(v[7])};
        if (lane == 0)
#pragma unroll
            for (int k = 0; k < 5; ++k) red[k][w] = g[k];
        __syncthreads();
        if (w == 0) {
            double a = 0.0;
            if (lane < 5) {
                a = red[lane][0];
                for (int q = 1; q < NT / 64; ++q) a = lane < 3 ? a + red[lane][q] : fmax(a, red[lane][q]);
            }
            double f[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) f[k] = __shfl(a, k, 64);
            if (lane == 0) {
                const int crit = (int)gate[2];
                bool fails;
                if (crit == 1) fails = !(f[3] <= gate[1] + gate[0] * fmax(f[4], gate[4]));
                else if (crit == 2) fails = !(sqrt(f[2]) < gate[1]);
                else fails = !(sqrt(f[0]) / (1.0 + sqrt(gate[3])) <= gate[0]);
                *s_skip = fails && isfinite(f[0]) && isfinite(f[1]) && isfinite(f[2]) && isfinite(f[3]) &&
                          isfinite(f[4]);
            }
        }
        __syncthreads();
        if (*s_skip) return;
    }
    for (int j = gc; j < n; j += NT / Lc) {
        const double a = lds_dot<double>(cps[j], cps[j + 1], lc, Lc, ris, cvc, ls);
        if (lc == 0) {
            const double cj = c64[j], r = a + cj - ds[j];
            v[3] += r * r;
            v[4] += cj * (double)zs[j];
            v[5] += cj * (double)xs[j];
            v[8] = fmax(v[8], fabs(r));
            v[9] = fmax(v[9], fabs(a));
        }
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = uv::wave_fold0<false>(v[k]);
#pragma unroll
    for (int k = 6; k < 10; ++k) v[k] = uv::wave_fold0<true>(v[k]);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 10; ++k) red[k][w] = v[k];
    __syncthreads();
    if (w == 0) {  // lane k < 10 of the first wavefront folds value k over the wavefronts, in order
        double a = 0.0;
        if (lane < 10) {
            a = red[lane][0];
            for (int q = 1; q < NT / 64; ++q) a = lane < 6 ? a + red[lane][q] : fmax(a, red[lane][q]);
        }
#pragma unroll
        for (int k = 0; k < 10; ++k) sv[k] = __shfl(a, k, 64);
    }
}

// Up to `iters` iterations of a small orthant problem in one workgroup: the
// state and both copies of A are staged in LDS once, then every iteration
// runs the column pass (Lc lanes per column: A'u from LDS, then the x-step,
// projection and delta update), a barrier, the row pass (Lr lanes per row:
// A x, the lambda and u updates) and a barrier, with the FP64 residual
// check of the other paths every check_every iterations (FP64 values of A:
// the staged ones in FP64, from global memory in the mixed form; then a
// fixed-order workgroup reduction) and its stop decision; with gated the
// check's column half is skipped when its primal half fails the stopping
// test (res_check); the state goes back to global memory at the end.  Same
// per-entry arithmetic as the sweep kernels.  eval_only: no iteration, the
// residuals of the current state are recorded without a stop decision (a
// residual query).
template <typename T>
__global__ void __launch_bounds__(kResThreads)
k_resident(int m, int n, ResLayout L, int Lr, int Lc, const int *__restrict__ rp, const int *__restrict__ ci,
           const T *__restrict__ va, const int *__restrict__ cp, const int *__restrict__ ri,
           const T *__restrict__ vc, const double *__restrict__ va64, const double *__restrict__ vc64,
           const T *__restrict__ b, const double *__restrict__ b64, const T *__restrict__ c,
           const double *__restrict__ c64, const T *__restrict__ fu, T *__restrict__ x, T *__restrict__ z,
           T *__restrict__ u, double *__restrict__ lam, double *__restrict__ delta, double mu, long long iters,
           int eval_only, int check_every, double eps, double eps_abs, double eps_gap, int crit, DevStatus *st,
           HistRing hist, int gated)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ double red[10][kResThreads / 64];
    __shared__ int stop, skip;
    if (!eval_only && st->done) return;
    constexpr int NT = kResThreads;
    const int tid = threadIdx.x;
    double *ds = (double *)(lds_raw + L.d), *ls = (double *)(lds_raw + L.l);
    T *xs = (T *)(lds_raw + L.x), *zs = (T *)(lds_raw + L.z), *us = (T *)(lds_raw + L.u);
    T *vcs = (T *)(lds_raw + L.vc), *vas = (T *)(lds_raw + L.va);
    int *cps = (int *)(lds_raw + L.cp), *rps = (int *)(lds_raw + L.rp);
    unsigned short *ris = (unsigned short *)(lds_raw + L.ri), *cis = (unsigned short *)(lds_raw + L.ci);
    const int nnz = rp[m];
    for (int j = tid; j < n; j += NT) {
        xs[j] = x[j];
        zs[j] = z[j];
        ds[j] = delta[j];
    }
    for (int i = tid; i < m; i += NT) {
        us[i] = u[i];
        ls[i] = lam[i];
    }
    for (int j = tid; j <= n; j += NT) cps[j] = cp[j];
    for (int i = tid; i <= m; i += NT) rps[i] = rp[i];
    for (int k = tid; k < nnz; k += NT) {
        ris[k] = (unsigned short)ri[k];
        vcs[k] = vc[k];
        cis[k] = (unsigned short)ci[k];
        vas[k] = va[k];
    }
    if (tid == 0) stop = 0;
    __syncthreads();
    const long long it0 = st->iter;
    const double nrm[4] = {st->bnorm2, st->cnorm2, st->binf, st->cinf};
    const double gate[5] = {eps, eps_abs, (double)crit, nrm[0], nrm[2]};
    // FP64 values of A for the checks: the staged ones in FP64, global ones in the mixed form
    const double *cva = sizeof(T) == sizeof(double) ? (const double *)vas : va64;
    const double *cvc = sizeof(T) == sizeof(double) ? (const double *)vcs : vc64;
    if (eval_only) {
        double sv[10];
        res_check<T>(m, n, Lr, Lc, rps, cis, cps, ris, cva, cvc, xs, zs, ds, ls, b64, c64, red, sv, nullptr, &skip);
        if (tid == 0) finish_check(sv, nrm, it0, eps, eps_abs, eps_gap, crit, 0, st, hist);
        return;
    }
    const double inv_mu = 1.0 / mu;
    const int gc = tid / Lc, lc = tid % Lc, gr = tid / Lr, lr = tid % Lr;
    long long done = 0;
    int to_check = check_every - (int)(it0 % check_every);  // iterations left to the next check
    for (long long t = 0; t < iters; ++t) {
        for (int j = gc; j < n; j += NT / Lc) {
            const int k0 = cps[j], k1 = cps[j + 1];
            const T a = lds_dot<T>(k0, k1, lc, Lc, ris, vcs, us);
            if (lc == 0) {
                const double d = ds[j];
                const T dm = (T)(d * inv_mu);
                const T xn = x_step<T>(k1 - k0, xs[j], zs[j], a, dm, c[j], inv_mu);
                const T v = xn - dm;
                const T zn = v > (T)0 ? v : (T)0;
                xs[j] = xn;
                zs[j] = zn;
                ds[j] = d + mu * ((double)zn - (double)xn);
            }
        }
        __syncthreads();
        for (int i = gr; i < m; i += NT / Lr) {
            const T q = lds_dot<T>(rps[i], rps[i + 1], lr, Lr, cis, vas, xs);
            if (lr == 0) {
                const T e = fu[i] * (b[i] - q);
                const double li = ls[i] - mu * (double)e;
                ls[i] = li;
                us[i] = (T)((double)e - li * inv_mu);
            }
        }
        __syncthreads();
        done = t + 1;
        const long long itn = it0 + done;
        if (--to_check != 0) continue;
        to_check = check_every;
        double sv[10];
        res_check<T>(m, n, Lr, Lc, rps, cis, cps, ris, cva, cvc, xs, zs, ds, ls, b64, c64, red, sv,
                     gated ? gate : nullptr, &skip);
        if (gated && skip) continue;
        if (tid == 0) {
            st->iter = itn;
            stop = finish_check(sv, nrm, itn, eps, eps_abs, eps_gap, crit, 1, st, hist) ? 1 : 0;
        }
        __syncthreads();
        if (stop) break;
    }
    for (int j = tid; j < n; j += NT) {
        x[j] = xs[j];
        z[j] = zs[j];
        delta[j] = ds[j];
    }
    for (int i = tid; i < m; i += NT) {
        u[i] = us[i];
        lam[i] = ls[i];
    }
    if (tid == 0) st->iter = it0 + done;
}

}  // namespace

// ---------------------------------------------------------------------------
// Solver handle
// ---------------------------------------------------------------------------
struct uv_solver {
    int32_t m = 0, n = 0;
    int64_t nnz = 0;
    int32_t n_orth = 0, n_soc = 0;
    uv_opts o{};
    hipStream_t stream = nullptr, cap = nullptr;
    bool own_stream = false;
    std::vector<void *> allocs;

    int *rp = nullptr, *ci = nullptr, *cp = nullptr, *ri = nullptr;
    double *va64 = nullptr, *vc64 = nullptr;  // FP64 values (CSR, CSC)
    void *va = nullptr, *vc = nullptr;        // sweep values (alias of the FP64 ones in FP64 mode)
    double *b64 = nullptr, *c64 = nullptr;
    void *b = nullptr, *c = nullptr, *fu = nullptr;
    void *x = nullptr, *z = nullptr, *u = nullptr;
    double *lam = nullptr, *delta = nullptr;
    double *scratch = nullptr;                // max(m, n) doubles
    double *part_row = nullptr, *part_col = nullptr;
    int nblk_row = 0, nblk_rescol = 0;
    int *tcol = nullptr, *tcone = nullptr, *soc_off = nullptr;
    int ntiles = 0, tile_cap = kSocTile;
    int *wtcol = nullptr, *winfo = nullptr;   // wavefront tiles (all cones <= 64)
    int nwtiles = 0;
    DevStatus *st = nullptr;
    DevStatus *st_host = nullptr;             // pinned
    int L_row = 8, L_col = 4;   // lanes per row / column
    int E_row = 4, E_col = 4;   // gathers in flight per lane
    int S_row = 1, S_col = 1;   // XCD slabs of x (row pass) and of u (column pass)
    bool chunked = true;        // slab passes by 64-segment chunks (else lane groups)
    bool batch8 = true;         // chunk batches of eight 64-entry steps (else four)
    int *srp = nullptr, *sci = nullptr;  // row-pass slab copy (S_row * m + 1 offsets)
    void *sva = nullptr;
    int *scp = nullptr, *sri = nullptr;  // column-pass slab copy (S_col * n + 1 offsets)
    void *svc = nullptr;
    void *P_row = nullptr, *P_col = nullptr;  // slab partials (2 S_row m, S_col n)
    double *sva64 = nullptr, *svc64 = nullptr;  // FP64 values of the slab copies
    double *P_res = nullptr;    // FP64 slab partials of the mixed form's checks
    int nblk_row_fused = 0;     // row-residual partial blocks written by the check row pass
    bool resident = false;      // iterate with k_resident (the whole problem in one workgroup's LDS)
    bool need_start = false;    // b changed (solver_set_rhs): no iteration before a new start
    const int *res_skip = nullptr;  // skip flag of the column residual kernels being launched
    ResLayout rlay{};
    int res_lr = 1, res_lc = 1;  // lanes per row and per column of k_resident
    HistRec *hist = nullptr;     // residual history ring (opts.history records)
    double clock_khz = 0.0;      // rate of the GPU wall clock
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t host_iter = 0;
};

namespace {

template <typename T>
T *dalloc(uv_solver *s, size_t count)
{
    void *p = nullptr;
    if (uv::dev_malloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return nullptr;
    s->allocs.push_back(p);
    return (T *)p;
}

#define UV_TRY(expr)                               \
    do {                                           \
        if ((expr) != hipSuccess) return UV_EHIP;  \
    } while (0)

int pick_lanes(double avg)
{
    // about two entries per lane (with two gathers in flight per lane, one
    // pass covers a typical row), whole power-of-two groups
    int L = 1;
    while (L < 64 && L * 2 < avg) L <<= 1;
    return L;
}

bool lanes_ok(int L) { return L == 0 || (L >= 1 && L <= 64 && (L & (L - 1)) == 0); }

bool unroll_ok(int E) { return E == 0 || E == 1 || E == 2 || E == 4 || E == 8; }

bool slabs_ok(int S) { return S == 0 || S == 1 || S == 2 || S == 4 || S == 8; }


// ---- launch helpers (dispatch on precision, lanes L and unroll E) ----

// Chunked slab product with the batch depth chosen at create time.
template <typename T, int S, typename G = T>
void seg_chunk_launch(const uv_solver *s, unsigned grid, hipStream_t st, int nseg, const int *ptr, const int *idx,
                      const T *val, const G *vec, T *out, const int *skip)
{
    if (s->batch8) k_seg_chunk<T, T, S, 8, G><<<grid, kWG, 0, st>>>(nseg, ptr, idx, val, vec, out, skip);
    else k_seg_chunk<T, T, S, 4, G><<<grid, kWG, 0, st>>>(nseg, ptr, idx, val, vec, out, skip);
}

// FP64 partials of a check's A x (S m values; those of A z follow them):
// the sweep's own partial buffer in FP64, a buffer of their own in the
// mixed form.
template <typename T>
double *check_px(const uv_solver *s)
{
    return sizeof(T) == sizeof(double) ? (double *)s->P_row : s->P_res;
}

template <typename T, int S>
double *row_pz(const uv_solver *s)
{
    return check_px<T>(s) + (size_t)S * s->m;
}

template <typename T, int L, int E, int S>
void row_slab_launch(uv_solver *s, hipStream_t st, int mode)
{
    const unsigned g = S * blocks_for(s->m, kWG / L), gc = blocks_for(s->m, kWG);
    const double mu = s->o.mu, im = 1.0 / s->o.mu;
    if (s->chunked && mode == 1) {
        // a check: A z and A x with FP64 values of A and FP64 sums (the mixed
        // form gathers its FP32 iterates), then the update from A x
        const unsigned gk = S * blocks_for(s->m, kWG);
        double *px = check_px<T>(s);
        seg_chunk_launch<double, S, T>(s, gk, st, s->m, s->srp, s->sci, s->sva64, (const T *)s->z, row_pz<T, S>(s),
                                       &s->st->done);
        seg_chunk_launch<double, S, T>(s, gk, st, s->m, s->srp, s->sci, s->sva64, (const T *)s->x, px,
                                       &s->st->done);
        k_row_combine<T, double, S, 1><<<gc, kWG, 0, st>>>(s->m, px, row_pz<T, S>(s), (const T *)s->b, s->b64,
                                                           (const T *)s->fu, s->lam, (T *)s->u, mu, im,
                                                           s->part_row, s->nblk_row_fused, s->st);
        return;
    }
    if (s->chunked) {
        const unsigned gk = S * blocks_for(s->m, kWG);
        const bool ign = mode == 2;
        seg_chunk_launch<T, S>(s, gk, st, s->m, s->srp, s->sci, (const T *)s->sva, (const T *)s->x, (T *)s->P_row,
                               ign ? nullptr : &s->st->done);
    }
#define UV_SLAB_ARGS s->m, s->srp, s->sci, (const T *)s->sva, (const T *)s->x, (const T *)s->z, (T *)s->P_row
#define UV_COMB_ARGS                                                                                       \
    s->m, (const T *)s->P_row, row_pz<T, S>(s), (const T *)s->b, s->b64, (const T *)s->fu, s->lam,         \
        (T *)s->u, mu, im, s->part_row, s->nblk_row_fused, s->st
    if (mode == 1) {  // lane-group slab passes (FP64 only)
        k_row_slab<T, L, E, S, true><<<g, kWG, 0, st>>>(UV_SLAB_ARGS, 0, s->st);
        k_row_combine<T, T, S, 1><<<gc, kWG, 0, st>>>(UV_COMB_ARGS);
    } else if (mode == 2) {
        if (!s->chunked) k_row_slab<T, L, E, S, false><<<g, kWG, 0, st>>>(UV_SLAB_ARGS, 1, s->st);
        k_row_combine<T, T, S, 2><<<gc, kWG, 0, st>>>(UV_COMB_ARGS);
    } else {
        if (!s->chunked) k_row_slab<T, L, E, S, false><<<g, kWG, 0, st>>>(UV_SLAB_ARGS, 0, s->st);
        k_row_combine<T, T, S, 0><<<gc, kWG, 0, st>>>(UV_COMB_ARGS);
    }
#undef UV_SLAB_ARGS
#undef UV_COMB_ARGS
}

template <typename T, int L, int E>
struct RowLaunch {
    static void run(uv_solver *s, hipStream_t st, int mode)
    {
        if (s->S_row == 2) return row_slab_launch<T, L, E, 2>(s, st, mode);
        if (s->S_row == 4) return row_slab_launch<T, L, E, 4>(s, st, mode);
        if (s->S_row == 8) return row_slab_launch<T, L, E, 8>(s, st, mode);
        const unsigned g = blocks_for(s->m, kWG / L);
        const double mu = s->o.mu, im = 1.0 / s->o.mu;
#define UV_ROW_ARGS                                                                                        \
    s->m, s->rp, s->ci, (const T *)s->va, (const T *)s->x, (const T *)s->z, (const T *)s->b,              \
        (const T *)s->fu, s->lam, (T *)s->u, mu, im, s->part_row, s->nblk_row, s->st
        if (mode == 1) k_row<T, L, E, 1><<<g, kWG, 0, st>>>(UV_ROW_ARGS);
        else if (mode == 2) k_row<T, L, E, 2><<<g, kWG, 0, st>>>(UV_ROW_ARGS);
        else k_row<T, L, E, 0><<<g, kWG, 0, st>>>(UV_ROW_ARGS);
#undef UV_ROW_ARGS
    }
};

// Column update (x-step, projection, delta) over all cones; LL/EE/S: lanes,
// unroll and slab count of the A'u it uses.
template <typename T, int LL, int EE, int S>
void col_update_launch(uv_solver *s, hipStream_t st)
{
    const double mu = s->o.mu, im = 1.0 / s->o.mu;
    if (s->n_orth > 0) {
        const unsigned g = blocks_for(s->n_orth, kWG / LL);
        k_col_orth<T, LL, EE, S><<<g, kWG, 0, st>>>(s->n_orth, s->cp, s->ri, (const T *)s->vc, (const T *)s->u,
                                                    (T *)s->x, (T *)s->z, s->delta, (const T *)s->c, mu, im,
                                                    (const T *)s->P_col, s->n, s->st);
    }
    if (s->nwtiles > 0) {
        k_col_soc_wave<T, EE, S><<<blocks_for(s->nwtiles, kWG / 64), kWG, 0, st>>>(
            s->nwtiles, s->wtcol, s->winfo, s->n_orth, s->cp, s->ri, (const T *)s->vc, (const T *)s->u, (T *)s->x,
            (T *)s->z, s->delta, (const T *)s->c, mu, im, (const T *)s->P_col, s->n, s->st);
    } else if (s->ntiles > 0) {
#define UV_SOC_ARGS                                                                                        \
    s->tcol, s->tcone, s->soc_off, s->cp, s->ri, (const T *)s->vc, (const T *)s->u, (T *)s->x, (T *)s->z, \
        s->delta, (const T *)s->c, mu, im, (const T *)s->P_col, s->n, s->st
        if (s->tile_cap <= kSocTile) k_col_soc<T, LL, EE, kSocTile, S><<<s->ntiles, kWG, 0, st>>>(UV_SOC_ARGS);
        else k_col_soc<T, LL, EE, UV_MAX_CONE, S><<<s->ntiles, kWG, 0, st>>>(UV_SOC_ARGS);
#undef UV_SOC_ARGS
    }
}

template <typename T, int L, int E, int S>
void col_slab_launch(uv_solver *s, hipStream_t st)
{
    if (s->chunked) {
        seg_chunk_launch<T, S>(s, S * blocks_for(s->n, kWG), st, s->n, s->scp, s->sri, (const T *)s->svc,
                               (const T *)s->u, (T *)s->P_col, &s->st->done);
    } else {
        const unsigned g = S * blocks_for(s->n, kWG / L);
        k_col_slab<T, L, E, S><<<g, kWG, 0, st>>>(s->n, s->scp, s->sri, (const T *)s->svc, (const T *)s->u,
                                                  (T *)s->P_col, s->st);
    }
    col_update_launch<T, 1, 1, S>(s, st);
}

template <typename T, int L, int E>
struct ColLaunch {
    static void run(uv_solver *s, hipStream_t st, int)
    {
        if (s->S_col == 2) return col_slab_launch<T, L, E, 2>(s, st);
        if (s->S_col == 4) return col_slab_launch<T, L, E, 4>(s, st);
        if (s->S_col == 8) return col_slab_launch<T, L, E, 8>(s, st);
        col_update_launch<T, L, E, 1>(s, st);
    }
};

template <typename T, int L, int E>
struct ResRowLaunch {
    static void run(uv_solver *s, hipStream_t st, int)
    {
        const unsigned g = blocks_for(s->m, kWG / L);
        k_res_row<T, L><<<g, kWG, 0, st>>>(s->m, s->rp, s->ci, s->va64, (const T *)s->x, (const T *)s->z,
                                           s->b64, s->lam, s->part_row, s->nblk_row);
    }
};

template <typename T, int L, int E>
struct ResColLaunch {
    static void run(uv_solver *s, hipStream_t st, int)
    {
        const unsigned g = blocks_for(s->n, kWG / L);
        k_res_col<T, L><<<g, kWG, 0, st>>>(s->n, s->cp, s->ri, s->vc64, s->lam, s->c64, s->delta,
                                           (const T *)s->z, (const T *)s->x, s->part_col, s->nblk_rescol,
                                           s->res_skip);
    }
};

template <template <typename, int, int> class F, typename T, int L>
void dispatch_e(int E, uv_solver *s, hipStream_t st, int mode)
{
    switch (E) {
    case 1: F<T, L, 1>::run(s, st, mode); break;
    case 2: F<T, L, 2>::run(s, st, mode); break;
    case 4: F<T, L, 4>::run(s, st, mode); break;
    default: F<T, L, 8>::run(s, st, mode); break;
    }
}

template <template <typename, int, int> class F, typename T>
void dispatch_le(int L, int E, uv_solver *s, hipStream_t st, int mode)
{
    switch (L) {
    case 1: dispatch_e<F, T, 1>(E, s, st, mode); break;
    case 2: dispatch_e<F, T, 2>(E, s, st, mode); break;
    case 4: dispatch_e<F, T, 4>(E, s, st, mode); break;
    case 8: dispatch_e<F, T, 8>(E, s, st, mode); break;
    case 16: dispatch_e<F, T, 16>(E, s, st, mode); break;
    case 32: dispatch_e<F, T, 32>(E, s, st, mode); break;
    default: dispatch_e<F, T, 64>(E, s, st, mode); break;
    }
}

template <template <typename, int, int> class F>
void dispatch(uv_solver *s, hipStream_t st, int L, int E, int mode)
{
    if (s->o.precision == UV_MIXED) dispatch_le<F, float>(L, E, s, st, mode);
    else dispatch_le<F, double>(L, E, s, st, mode);
}

template <template <typename, int, int> class F>
void dispatch_le_res(uv_solver *s, hipStream_t st, int L)
{
    const bool mixed = s->o.precision == UV_MIXED;
    switch (L) {
#define UV_RES_CASE(LL)                                   \
    case LL:                                              \
        if (mixed) F<float, LL, 4>::run(s, st, 0);        \
        else F<double, LL, 4>::run(s, st, 0);             \
        break;
        UV_RES_CASE(1) UV_RES_CASE(2) UV_RES_CASE(4) UV_RES_CASE(8) UV_RES_CASE(16) UV_RES_CASE(32)
    default:
        if (mixed) F<float, 64, 4>::run(s, st, 0);
        else F<double, 64, 4>::run(s, st, 0);
        break;
#undef UV_RES_CASE
    }
}

void launch_col(uv_solver *s, hipStream_t st) { dispatch<ColLaunch>(s, st, s->L_col, s->E_col, 0); }

// The row pass of a check also forms the row residual partials: in FP64
// always, in the mixed form when its FP64 A z goes through the chunked slab
// product (else a separate residual pass follows).
bool fused_row_check(const uv_solver *s)
{
    return s->o.precision == UV_FP64 || (s->S_row > 1 && s->chunked);
}

// Column residuals by the chunked slab product of A'lambda over the FP64
// values of the column slab copy.
bool slab_col_check(const uv_solver *s) { return s->S_col > 1 && s->chunked; }

// mode: 0 iterate, 1 iterate + residual partials, 2 resume
void launch_row(uv_solver *s, hipStream_t st, int mode)
{
    if (mode == 1 && !fused_row_check(s)) mode = 0;
    dispatch<RowLaunch>(s, st, s->L_row, s->E_row, mode);
}

// Residual evaluation of the current state.  In FP64 mode right after a
// MODE 1 row pass only the column residuals remain.  The residual kernels
// take one fixed unroll; their lane counts follow the sweep's so the
// partial arrays are sized once.
template <int S>
void res_col_slab_launch(uv_solver *s, hipStream_t st)
{
    const unsigned g = blocks_for(s->n, kWG);
    const bool mixed = s->o.precision == UV_MIXED;
    double *P = mixed ? s->P_res : (double *)s->P_col;
    seg_chunk_launch<double, S>(s, S * g, st, s->n, s->scp, s->sri, s->svc64, s->lam, P, s->res_skip);
    if (mixed)
        k_res_col_slab<float, S><<<g, kWG, 0, st>>>(s->n, P, s->c64, s->delta, (const float *)s->z,
                                                    (const float *)s->x, s->part_col, (int)g, s->res_skip);
    else
        k_res_col_slab<double, S><<<g, kWG, 0, st>>>(s->n, P, s->c64, s->delta, (const double *)s->z,
                                                     (const double *)s->x, s->part_col, (int)g, s->res_skip);
}

void launch_residuals(uv_solver *s, hipStream_t st, bool row_done, bool decide)
{
    if (!row_done) dispatch_le_res<ResRowLaunch>(s, st, s->L_row);
    const int nrow = row_done ? s->nblk_row_fused : s->nblk_row;
    // primal half first: a check of the iteration whose primal part fails
    // cannot stop the run, and then skips its column half (not with a
    // residual history, which records every check whole, nor when every
    // check is asked for whole)
    const bool gated = decide && s->o.full_checks == 0 && !s->hist;
    if (gated)
        k_row_gate<<<1, kWG, 0, st>>>(nrow, s->part_row, s->o.eps_kkt, s->o.eps_abs, s->o.criterion, s->st);
    s->res_skip = gated ? &s->st->skip_col : nullptr;
    // with column slabs and chunked passes A'lambda goes through the slab copy
    // (FP64 values in both precisions), else the plain column residual pass
    const bool slab = slab_col_check(s);
    if (slab) {
        if (s->S_col == 2) res_col_slab_launch<2>(s, st);
        else if (s->S_col == 4) res_col_slab_launch<4>(s, st);
        else res_col_slab_launch<8>(s, st);
    } else {
        dispatch_le_res<ResColLaunch>(s, st, s->L_col);
    }
    const int ncol = slab ? (int)blocks_for(s->n, kWG) : s->nblk_rescol;
    k_finalize<<<1, kWG, 0, st>>>(nrow, s->part_row, ncol, s->part_col, s->o.eps_kkt, s->o.eps_abs,
                                  s->o.eps_gap, s->o.criterion, decide ? 1 : 0, gated ? 1 : 0, s->st,
                                  HistRing{s->hist, s->o.history});
    s->res_skip = nullptr;
}

// One iteration; with check, the residuals of the new iterate follow it.
void launch_iteration(uv_solver *s, hipStream_t st, bool check)
{
    launch_col(s, st);
    const bool fused = check && fused_row_check(s);
    launch_row(s, st, fused ? 1 : 0);
    if (check) launch_residuals(s, st, fused, true);
}

int build_graph(uv_solver *s)
{
    if (hipStreamBeginCapture(s->cap, hipStreamCaptureModeRelaxed) != hipSuccess) return UV_EHIP;
    for (int i = 0; i < s->o.check_every; ++i) launch_iteration(s, s->cap, i == s->o.check_every - 1);
    if (hipStreamEndCapture(s->cap, &s->graph) != hipSuccess) return UV_EHIP;
    if (hipGraphInstantiate(&s->exec, s->graph, nullptr, nullptr, 0) != hipSuccess) return UV_EHIP;
    return UV_OK;
}

// Lanes per segment of k_resident: the most (a power of two, at most 64)
// that keeps every segment of the pass on a lane group at once.
int resident_lanes(int segs)
{
    int L = 1;
    while (L < 64 && (int64_t)segs * L * 2 <= kResThreads) L <<= 1;
    return L;
}

// Device operands of k_resident.
struct ResArgs {
    int m, n;
    ResLayout L;
    int Lr, Lc;
    const int *rp, *ci, *cp, *ri;
    const void *va, *vc, *b, *c, *fu;  // sweep type
    const double *va64, *vc64, *b64, *c64;
    void *x, *z, *u;                   // sweep type
    double *lam, *delta;
    DevStatus *st;
    HistRing hist;
    bool mixed;
    double mu, eps, eps_abs, eps_gap;
    int check_every, crit;
    int gated;  // checks primal half first (no history, opts.full_checks = 0)
};

// Up to `iters` iterations on the resident path in launches of at most 2^16
// iterations (a launch returns at once once a check has stopped the run),
// or with eval_only one launch that records the residuals of the state.
void resident_launch(const ResArgs &a, hipStream_t st, int64_t iters, bool eval_only)
{
    constexpr int64_t kChunk = (int64_t)1 << 16;
    int64_t left = eval_only ? 1 : iters;
    while (left > 0) {
        const long long q = eval_only ? 0 : (long long)std::min(left, kChunk);
#define UV_RES_ARGS(T)                                                                                         \
    a.m, a.n, a.L, a.Lr, a.Lc, a.rp, a.ci, (const T *)a.va, a.cp, a.ri, (const T *)a.vc, a.va64, a.vc64,         \
        (const T *)a.b, a.b64, (const T *)a.c, a.c64, (const T *)a.fu, (T *)a.x, (T *)a.z, (T *)a.u, a.lam,        \
        a.delta, a.mu, q, eval_only ? 1 : 0, a.check_every, a.eps, a.eps_abs, a.eps_gap, a.crit, a.st, a.hist,  \
        a.gated
        if (a.mixed) k_resident<float><<<1, kResThreads, a.L.bytes, st>>>(UV_RES_ARGS(float));
        else k_resident<double><<<1, kResThreads, a.L.bytes, st>>>(UV_RES_ARGS(double));
#undef UV_RES_ARGS
        left -= eval_only ? 1 : kChunk;
    }
}

ResArgs res_args(const uv_solver *s)
{
    ResArgs a{};
    a.m = s->m;
    a.n = s->n;
    a.L = s->rlay;
    a.Lr = s->res_lr;
    a.Lc = s->res_lc;
    a.rp = s->rp;
    a.ci = s->ci;
    a.cp = s->cp;
    a.ri = s->ri;
    a.va = s->va;
    a.vc = s->vc;
    a.b = s->b;
    a.c = s->c;
    a.fu = s->fu;
    a.va64 = s->va64;
    a.vc64 = s->vc64;
    a.b64 = s->b64;
    a.c64 = s->c64;
    a.x = s->x;
    a.z = s->z;
    a.u = s->u;
    a.lam = s->lam;
    a.delta = s->delta;
    a.st = s->st;
    a.hist = HistRing{s->hist, s->o.history};
    a.gated = s->o.full_checks == 0 && !s->hist ? 1 : 0;
    a.mixed = s->o.precision == UV_MIXED;
    a.mu = s->o.mu;
    a.eps = s->o.eps_kkt;
    a.eps_abs = s->o.eps_abs;
    a.eps_gap = s->o.eps_gap;
    a.check_every = s->o.check_every;
    a.crit = s->o.criterion;
    return a;
}

int sync_status(uv_solver *s)
{
    UV_TRY(hipMemcpyAsync(s->st_host, s->st, sizeof(DevStatus), hipMemcpyDeviceToHost, s->stream));
    UV_TRY(hipStreamSynchronize(s->stream));
    s->host_iter = s->st_host->iter;
    return UV_OK;
}

int validate(const uv_csr *A, const double *b, const double *c, const uv_cones *K, const uv_opts *o)
{
    if (!A || !b || !c || !K || !o) return UV_EINVAL;
    if (A->m < 1 || A->n < 1 || A->nnz < 0) return UV_EINVAL;
    if (!(o->mu > 0.0) || !std::isfinite(o->mu)) return UV_EINVAL;
    if (o->precision != UV_FP64 && o->precision != UV_MIXED) return UV_EINVAL;
    if (o->check_every < 1 || !(o->eps_kkt >= 0.0) || o->max_iter < 0) return UV_EINVAL;
    if (o->criterion < 0 || o->criterion > 2 || !(o->eps_abs >= 0.0) || !(o->eps_gap >= 0.0)) return UV_EINVAL;
    if (!lanes_ok(o->lanes_row) || !lanes_ok(o->lanes_col)) return UV_EINVAL;
    if (!unroll_ok(o->unroll_row) || !unroll_ok(o->unroll_col)) return UV_EINVAL;
    if (!slabs_ok(o->slabs_row) || !slabs_ok(o->slabs_col)) return UV_EINVAL;
    if (o->slab_kernel < 0 || o->slab_kernel > 3) return UV_EINVAL;
    if (o->resident < 0 || o->resident > 2) return UV_EINVAL;
    if (o->history < 0 || o->history > (1 << 24)) return UV_EINVAL;
    if (o->full_checks < 0 || o->full_checks > 1) return UV_EINVAL;
    if (A->nnz > 0 && (!A->col_idx || !A->val)) return UV_EINVAL;
    if (!A->row_ptr) return UV_EINVAL;
    if (A->nnz >= ((int64_t)1 << 31)) return UV_ETOOBIG;
    if (A->row_ptr[0] != 0 || A->row_ptr[A->m] != A->nnz) return UV_EBADCSR;
    for (int32_t i = 0; i < A->m; ++i) {
        const int64_t b0 = A->row_ptr[i], b1 = A->row_ptr[i + 1];
        if (b1 < b0 || b1 > A->nnz) return UV_EBADCSR;
        for (int64_t k = b0; k < b1; ++k) {
            const int32_t j = A->col_idx[k];
            if (j < 0 || j >= A->n) return UV_EBADCSR;
            if (k > b0 && j <= A->col_idx[k - 1]) return UV_EBADCSR;
        }
    }
    if (K->n_orthant < 0 || K->n_soc < 0 || (K->n_soc > 0 && !K->soc_sizes)) return UV_ECONE;
    int64_t tot = K->n_orthant;
    for (int32_t q = 0; q < K->n_soc; ++q) {
        if (K->soc_sizes[q] < 1 || K->soc_sizes[q] > UV_MAX_CONE) return UV_ECONE;
        tot += K->soc_sizes[q];
    }
    if (tot != A->n) return UV_ECONE;
    return UV_OK;
}

int setup(uv_solver *s, const uv_csr *A, const double *b, const double *c, const uv_cones *K)
{
    const int m = s->m, n = s->n;
    const int nnz = (int)s->nnz;
    const bool mixed = s->o.precision == UV_MIXED;
    const size_t ts = mixed ? sizeof(float) : sizeof(double);

    if (s->o.hip_stream) {
        s->stream = (hipStream_t)s->o.hip_stream;
    } else {
        UV_TRY(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
        s->own_stream = true;
    }
    UV_TRY(hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking));
    hipStream_t st = s->stream;

    s->rp = dalloc<int>(s, m + 1);
    s->ci = dalloc<int>(s, nnz);
    s->va64 = dalloc<double>(s, nnz);
    s->cp = dalloc<int>(s, n + 1);
    s->ri = dalloc<int>(s, nnz);
    s->vc64 = dalloc<double>(s, nnz);
    s->b64 = dalloc<double>(s, m);
    s->c64 = dalloc<double>(s, n);
    s->lam = dalloc<double>(s, m);
    s->delta = dalloc<double>(s, n);
    s->scratch = dalloc<double>(s, std::max(m, n));
    s->x = dalloc<char>(s, ts * n);
    s->z = dalloc<char>(s, ts * n);
    s->u = dalloc<char>(s, ts * m);
    s->fu = dalloc<char>(s, ts * m);
    if (mixed) {
        s->va = dalloc<float>(s, nnz);
        s->vc = dalloc<float>(s, nnz);
        s->b = dalloc<float>(s, m);
        s->c = dalloc<float>(s, n);
    } else {
        s->va = s->va64;
        s->vc = s->vc64;
        s->b = s->b64;
        s->c = s->c64;
    }
    s->nblk_row = (int)blocks_for(m, kWG / s->L_row);
    s->nblk_row_fused = s->S_row > 1 ? (int)blocks_for(m, kWG) : s->nblk_row;
    s->nblk_rescol = (int)blocks_for(n, kWG / s->L_col);
    s->part_row = dalloc<double>(s, 5 * (size_t)std::max(s->nblk_row, s->nblk_row_fused));
    s->part_col = dalloc<double>(s, 5 * std::max((size_t)s->nblk_rescol, (size_t)blocks_for(n, kWG)));
    s->st = dalloc<DevStatus>(s, 1);
    if (s->o.history > 0) {
        s->hist = dalloc<HistRec>(s, (size_t)s->o.history);
        if (!s->hist) return UV_ENOMEM;
        int dev = 0, khz = 0;
        UV_TRY(hipGetDevice(&dev));
        UV_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
        s->clock_khz = khz;
    }
    const size_t ncnt = std::max({(size_t)n, (size_t)s->S_row * m, (size_t)s->S_col * n});
    int *cnt = dalloc<int>(s, ncnt);
    int *bsum = dalloc<int>(s, blocks_for(ncnt, 4 * kWG));
    for (void *p : {(void *)s->rp, (void *)s->ci, (void *)s->va64, (void *)s->cp, (void *)s->ri,
                    (void *)s->vc64, (void *)s->b64, (void *)s->c64, (void *)s->lam, (void *)s->delta,
                    (void *)s->scratch, s->x, s->z, s->u, s->fu, s->va, s->vc, s->b, s->c,
                    (void *)s->part_row, (void *)s->part_col, (void *)s->st, (void *)cnt, (void *)bsum})
        if (!p) return UV_ENOMEM;
    if (uv::host_malloc(&s->st_host, sizeof(DevStatus), hipHostMallocDefault) != hipSuccess) {
        s->st_host = nullptr;
        return UV_ENOMEM;
    }

    // SOC tiles: whole cones, at most tile_cap columns per workgroup.
    if (K->n_soc > 0) {
        int maxc = 0;
        for (int q = 0; q < K->n_soc; ++q) maxc = std::max(maxc, (int)K->soc_sizes[q]);
        s->tile_cap = maxc <= kSocTile ? kSocTile : UV_MAX_CONE;
        std::vector<int> off(K->n_soc + 1), tcol, tcone;
        off[0] = K->n_orthant;
        for (int q = 0; q < K->n_soc; ++q) off[q + 1] = off[q] + K->soc_sizes[q];
        tcol.push_back(off[0]);
        tcone.push_back(0);
        for (int q = 0; q < K->n_soc; ++q) {
            if (off[q + 1] - tcol.back() > s->tile_cap) {
                tcol.push_back(off[q]);
                tcone.push_back(q);
            }
        }
        tcol.push_back(off[K->n_soc]);
        tcone.push_back(K->n_soc);
        s->ntiles = (int)tcol.size() - 1;
        s->tcol = dalloc<int>(s, tcol.size());
        s->tcone = dalloc<int>(s, tcone.size());
        s->soc_off = dalloc<int>(s, off.size());
        if (!s->tcol || !s->tcone || !s->soc_off) return UV_ENOMEM;
        UV_TRY(hipMemcpy(s->tcol, tcol.data(), tcol.size() * 4, hipMemcpyHostToDevice));
        UV_TRY(hipMemcpy(s->tcone, tcone.data(), tcone.size() * 4, hipMemcpyHostToDevice));
        UV_TRY(hipMemcpy(s->soc_off, off.data(), off.size() * 4, hipMemcpyHostToDevice));
        if (maxc <= 64) {  // wavefront tiles of whole cones, at most 64 columns each
            std::vector<int> wt(1, off[0]), info((size_t)(off[K->n_soc] - off[0]));
            for (int q = 0; q < K->n_soc; ++q) {
                if (off[q + 1] - wt.back() > 64) wt.push_back(off[q]);
                for (int j = off[q]; j < off[q + 1]; ++j) info[j - off[0]] = (j - off[q]) | (K->soc_sizes[q] << 16);
            }
            wt.push_back(off[K->n_soc]);
            s->nwtiles = (int)wt.size() - 1;
            s->wtcol = dalloc<int>(s, wt.size());
            s->winfo = dalloc<int>(s, info.size());
            if (!s->wtcol || !s->winfo) return UV_ENOMEM;
            UV_TRY(hipMemcpy(s->wtcol, wt.data(), wt.size() * 4, hipMemcpyHostToDevice));
            UV_TRY(hipMemcpy(s->winfo, info.data(), info.size() * 4, hipMemcpyHostToDevice));
        }
    }

    // Upload (row_ptr narrowed to 32-bit; nnz < 2^31 was checked).
    {
        std::vector<int> rp32(m + 1);
        for (int i = 0; i <= m; ++i) rp32[i] = (int)A->row_ptr[i];
        UV_TRY(hipMemcpy(s->rp, rp32.data(), (m + 1) * sizeof(int), hipMemcpyHostToDevice));
    }
    if (nnz > 0) {
        UV_TRY(hipMemcpy(s->ci, A->col_idx, (size_t)nnz * 4, hipMemcpyHostToDevice));
        UV_TRY(hipMemcpy(s->va64, A->val, (size_t)nnz * 8, hipMemcpyHostToDevice));
    }
    UV_TRY(hipMemcpy(s->b64, b, (size_t)m * 8, hipMemcpyHostToDevice));
    UV_TRY(hipMemcpy(s->c64, c, (size_t)n * 8, hipMemcpyHostToDevice));

    // Column-major copy of A.
    if (!build_csc(m, n, nnz, s->rp, s->ci, s->va64, s->cp, s->ri, s->vc64, cnt, bsum, st)) return UV_EHIP;

    // XCD slab copies: row pass split by column ranges, column pass by row ranges.
    for (int pass = 0; pass < 2; ++pass) {
        const int S = pass == 0 ? s->S_row : s->S_col;
        if (S == 1) continue;
        const int nr = pass == 0 ? m : n, width = pass == 0 ? n : m;
        int *off = dalloc<int>(s, (size_t)S * nr + 1);
        int *sidx = dalloc<int>(s, nnz);
        double *sval64 = dalloc<double>(s, nnz);
        void *part = dalloc<char>(s, ts * (size_t)(pass == 0 ? 2 * S : S) * nr);
        if (!off || !sidx || !sval64 || !part) return UV_ENOMEM;
        const int w = (width + S - 1) / S;
        const bool ok = pass == 0
                            ? build_slabs(m, nnz, s->rp, s->ci, s->va64, S, w, off, sidx, sval64, cnt, bsum, st)
                            : build_slabs(n, nnz, s->cp, s->ri, s->vc64, S, w, off, sidx, sval64, cnt, bsum, st);
        if (!ok) return UV_EHIP;
        void *sval = sval64;
        if (mixed) {
            sval = dalloc<float>(s, nnz);
            if (!sval) return UV_ENOMEM;
            if (nnz > 0) k_narrow<float><<<blocks_for(nnz, kWG), kWG, 0, st>>>(nnz, sval64, (float *)sval);
        }
        if (pass == 0) { s->srp = off; s->sci = sidx; s->sva = sval; s->sva64 = sval64; s->P_row = part; }
        else { s->scp = off; s->sri = sidx; s->svc = sval; s->svc64 = sval64; s->P_col = part; }
    }
    if (mixed && (s->S_row > 1 || s->S_col > 1)) {
        // FP64 partials of the checks' A z and A'lambda
        const size_t pr = s->S_row > 1 ? 2 * (size_t)s->S_row * m : 0;
        const size_t pc = s->S_col > 1 ? (size_t)s->S_col * n : 0;
        s->P_res = dalloc<double>(s, std::max(pr, pc));
        if (!s->P_res) return UV_ENOMEM;
    }

    // F_U, narrowed copies, norms.
    if (mixed) {
        k_row_factor<float><<<blocks_for(m, kWG), kWG, 0, st>>>(m, s->rp, s->va64, (float *)s->fu);
        if (nnz > 0) {
            k_narrow<float><<<blocks_for(nnz, kWG), kWG, 0, st>>>(nnz, s->va64, (float *)s->va);
            k_narrow<float><<<blocks_for(nnz, kWG), kWG, 0, st>>>(nnz, s->vc64, (float *)s->vc);
        }
        k_narrow<float><<<blocks_for(m, kWG), kWG, 0, st>>>(m, s->b64, (float *)s->b);
        k_narrow<float><<<blocks_for(n, kWG), kWG, 0, st>>>(n, s->c64, (float *)s->c);
    } else {
        k_row_factor<double><<<blocks_for(m, kWG), kWG, 0, st>>>(m, s->rp, s->va64, (double *)s->fu);
    }
    k_norms<<<1, kWG, 0, st>>>(m, s->b64, n, s->c64, s->st);
    UV_TRY(hipGetLastError());
    UV_TRY(hipStreamSynchronize(st));
    return UV_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void uv_test_fail_alloc(int64_t after)
{
    uv::g_alloc_fail_after.store(after < 0 ? -1 : (long long)after);
}

void uv_default_opts(uv_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->mu = 1.0;
    o->precision = UV_FP64;
    o->check_every = 10;
    o->eps_kkt = 1e-4;
    o->max_iter = 0;
    o->hip_stream = nullptr;
    o->lanes_row = 0;
    o->lanes_col = 0;
    o->use_graph = 1;
    o->unroll_row = 0;
    o->unroll_col = 0;
    o->slabs_row = 0;
    o->slabs_col = 0;
    o->criterion = 0;
    o->eps_abs = 0.0;
    o->slab_kernel = 0;
    o->eps_gap = 0.0;
    o->resident = 0;
    o->history = 0;
    o->full_checks = 0;
}

const char *solver_strerror(int code)
{
    switch (code) {
    case UV_OK: return "ok";
    case UV_EINVAL: return "invalid argument (null pointer, mu <= 0, m or n < 1, or a bad option)";
    case UV_EBADCSR: return "malformed CSR (row_ptr, column range or column order within a row)";
    case UV_ECONE: return "bad cone specification (sizes must be >= 1, <= UV_MAX_CONE and sum to n)";
    case UV_ENOMEM: return "out of device or pinned host memory";
    case UV_EHIP: return "HIP runtime error";
    case UV_ENUMERIC: return "NaN or Inf in a residual check";
    case UV_ETOOBIG: return "nnz must be below 2^31";
    case UV_ENOSCRATCH:
        return "the problem does not fit the no-allocation entry point (orthant cones only, m, n < 65536, "
               "small enough for one CU's LDS and the fixed device scratch)";
    default: return "unknown error code";
    }
}

void solver_destroy(uv_solver *s)
{
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    if (s->exec) (void)hipGraphExecDestroy(s->exec);
    if (s->graph) (void)hipGraphDestroy(s->graph);
    for (void *p : s->allocs) (void)hipFree(p);
    if (s->st_host) (void)hipHostFree(s->st_host);
    if (s->cap) (void)hipStreamDestroy(s->cap);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

int solver_create(const uv_csr *A, const double *b, const double *c, const uv_cones *K, const uv_opts *opts,
                  uv_solver **out)
{
    if (!out) return UV_EINVAL;
    *out = nullptr;
    uv_opts o;
    uv_default_opts(&o);
    if (opts) o = *opts;
    int rc = validate(A, b, c, K, &o);
    if (rc != UV_OK) return rc;
    uv_solver *s = new (std::nothrow) uv_solver();
    if (!s) return UV_ENOMEM;
    s->m = A->m;
    s->n = A->n;
    s->nnz = A->nnz;
    s->n_orth = K->n_orthant;
    s->n_soc = K->n_soc;
    s->o = o;
    {
        const size_t ts = o.precision == UV_MIXED ? 4 : 8;
        s->S_row = o.slabs_row ? o.slabs_row : pick_slabs_row(ts * (size_t)A->n);
        s->S_col = o.slabs_col ? o.slabs_col : pick_slabs_col(ts * (size_t)A->m);
        // a slab needs at least one index, and slab offsets are 32-bit
        while (s->S_row > 1 && (s->S_row > A->n || (int64_t)s->S_row * A->m >= INT32_MAX)) s->S_row >>= 1;
        while (s->S_col > 1 && (s->S_col > A->m || (int64_t)s->S_col * A->n >= INT32_MAX)) s->S_col >>= 1;
    }
    // lanes from the entries a lane group actually sums (a slab holds 1/S of a row)
    s->L_row = o.lanes_row ? o.lanes_row : pick_lanes((double)A->nnz / A->m / s->S_row);
    s->L_col = o.lanes_col ? o.lanes_col : pick_lanes((double)A->nnz / A->n / s->S_col);
    s->E_row = o.unroll_row ? o.unroll_row : 2;
    s->E_col = o.unroll_col ? o.unroll_col : 2;
    s->chunked = o.slab_kernel != 2;
    s->batch8 = o.slab_kernel != 3;
    {
        // the resident path when every cone has size 1, the row and column
        // numbers fit 16 bits and the whole problem fits one CU's LDS
        const bool mixed = o.precision == UV_MIXED;
        s->rlay = mixed ? resident_layout<float>(A->m, A->n, (int)A->nnz)
                        : resident_layout<double>(A->m, A->n, (int)A->nnz);
        const bool fits = K->n_soc == 0 && A->m < 65536 && A->n < 65536 && s->rlay.bytes <= kResLdsMax;
        if (o.resident == 2 && !fits) {
            solver_destroy(s);
            return UV_EINVAL;
        }
        // automatic only when no launch shape of the sweep kernels is forced
        const bool forced = o.lanes_row || o.lanes_col || o.unroll_row || o.unroll_col || o.slabs_row ||
                            o.slabs_col || o.slab_kernel;
        s->resident = fits && (o.resident == 2 || (o.resident == 0 && !forced));
        s->res_lr = resident_lanes(A->m);
        s->res_lc = resident_lanes(A->n);
        if (s->resident) {
            const hipError_t e = mixed ? hipFuncSetAttribute((const void *)k_resident<float>,
                                                             hipFuncAttributeMaxDynamicSharedMemorySize, kResLdsMax)
                                       : hipFuncSetAttribute((const void *)k_resident<double>,
                                                             hipFuncAttributeMaxDynamicSharedMemorySize, kResLdsMax);
            if (e != hipSuccess) {
                solver_destroy(s);
                return UV_EHIP;
            }
        }
    }
    rc = setup(s, A, b, c, K);
    if (rc == UV_OK) rc = solver_set_start(s, nullptr, nullptr, nullptr, nullptr);
    if (rc == UV_OK && s->o.use_graph && !s->resident) rc = build_graph(s);
    if (rc != UV_OK) {
        solver_destroy(s);
        return rc;
    }
    *out = s;
    return UV_OK;
}

}  // extern "C"

namespace {

// Uploads (x, z, delta, lambda) (NULL = zero) and resets the status; u is
// set by the caller's kernel.
int upload_state(uv_solver *s, const double *x, const double *z, const double *delta, const double *lambda)
{
    hipStream_t st = s->stream;
    const bool mixed = s->o.precision == UV_MIXED;
    const size_t ts = mixed ? 4 : 8;
    const int m = s->m, n = s->n;
    auto put_t = [&](void *dst, const double *src, int len) -> int {
        if (!src) return hipMemsetAsync(dst, 0, ts * len, st) == hipSuccess ? UV_OK : UV_EHIP;
        if (!mixed) return hipMemcpyAsync(dst, src, 8 * (size_t)len, hipMemcpyHostToDevice, st) == hipSuccess
                               ? UV_OK : UV_EHIP;
        if (hipMemcpyAsync(s->scratch, src, 8 * (size_t)len, hipMemcpyHostToDevice, st) != hipSuccess)
            return UV_EHIP;
        k_narrow<float><<<blocks_for(len, kWG), kWG, 0, st>>>(len, s->scratch, (float *)dst);
        // the scratch buffer is reused by the next upload: wait for this one
        return hipStreamSynchronize(st) == hipSuccess ? UV_OK : UV_EHIP;
    };
    int rc;
    if ((rc = put_t(s->x, x, n)) != UV_OK) return rc;
    if ((rc = put_t(s->z, z, n)) != UV_OK) return rc;
    if (delta) UV_TRY(hipMemcpyAsync(s->delta, delta, 8 * (size_t)n, hipMemcpyHostToDevice, st));
    else UV_TRY(hipMemsetAsync(s->delta, 0, 8 * (size_t)n, st));
    if (lambda) UV_TRY(hipMemcpyAsync(s->lam, lambda, 8 * (size_t)m, hipMemcpyHostToDevice, st));
    else UV_TRY(hipMemsetAsync(s->lam, 0, 8 * (size_t)m, st));
    const double im = 1.0 / s->o.mu;
    // k_start also sets u = -lambda/mu (the start mapping); resume overwrites it
    if (mixed) k_start<float><<<blocks_for(m, kWG), kWG, 0, st>>>(m, s->lam, (float *)s->u, im, s->st);
    else k_start<double><<<blocks_for(m, kWG), kWG, 0, st>>>(m, s->lam, (double *)s->u, im, s->st);
    UV_TRY(hipGetLastError());
    return UV_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Fixed device scratch of the no-allocation entry point
// ---------------------------------------------------------------------------
namespace {

// Every device buffer of solver_solve_noalloc is carved from this array, so
// the call allocates nothing.  Each GPU holds its own copy until the process
// ends; host code reaches it only through the address hipGetSymbolAddress
// returns on that device (the array's name is not a device address there).
constexpr size_t kScratchBytes = (size_t)2 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kScratchDevices] = {};

// The scratch array's address on the current device (looked up once per
// device, with that device current).
int scratch_address(unsigned char **out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return UV_EHIP;
    if (dev < 0 || dev >= kScratchDevices) return UV_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return UV_EHIP;
        g_scratch_ptr[dev] = (unsigned char *)p;
    }
    *out = g_scratch_ptr[dev];
    return UV_OK;
}

// Buffers carved in order from a region of `cap` bytes, 256-byte aligned;
// run once without a base to size the request.
struct Carve {
    unsigned char *base;
    size_t off, cap;
    bool ok;
    template <typename T>
    T *take(size_t count)
    {
        off = (off + 255) / 256 * 256;
        const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
        if (off + bytes > cap) ok = false;
        T *p = ok && base ? (T *)(base + off) : nullptr;
        off += bytes;
        return p;
    }
};

// int64 row offsets (m + 1, validated below 2^31) to the 32-bit device form.
__global__ void __launch_bounds__(kWG) k_narrow_offsets(int len, const int64_t *__restrict__ src, int *__restrict__ dst)
{
    const int i = blockIdx.x * kWG + threadIdx.x;
    if (i < len) dst[i] = (int)src[i];
}

// Device buffers of one no-allocation solve.
struct NoAlloc {
    DevStatus *st;
    int64_t *rp64;
    int *rp, *ci, *cp, *ri, *cnt, *bsum;
    double *va64, *vc64, *b64, *c64, *lam, *delta, *wide;
    void *va, *vc, *b, *c, *fu, *x, *z, *u;
};

bool carve_noalloc(Carve &cv, int m, int n, int nnz, bool mixed, NoAlloc &d)
{
    const size_t ts = mixed ? 4 : 8;
    d.st = cv.take<DevStatus>(1);
    d.rp64 = cv.take<int64_t>((size_t)m + 1);
    d.rp = cv.take<int>((size_t)m + 1);
    d.ci = cv.take<int>(nnz);
    d.cp = cv.take<int>((size_t)n + 1);
    d.ri = cv.take<int>(nnz);
    d.cnt = cv.take<int>(n);
    d.bsum = cv.take<int>(blocks_for(n, 4 * kWG));
    d.va64 = cv.take<double>(nnz);
    d.vc64 = cv.take<double>(nnz);
    d.b64 = cv.take<double>(m);
    d.c64 = cv.take<double>(n);
    d.lam = cv.take<double>(m);
    d.delta = cv.take<double>(n);
    d.wide = cv.take<double>(n);
    d.va = mixed ? (void *)cv.take<float>(nnz) : (void *)d.va64;
    d.vc = mixed ? (void *)cv.take<float>(nnz) : (void *)d.vc64;
    d.b = mixed ? (void *)cv.take<float>(m) : (void *)d.b64;
    d.c = mixed ? (void *)cv.take<float>(n) : (void *)d.c64;
    d.fu = cv.take<char>(ts * m);
    d.x = cv.take<char>(ts * n);
    d.z = cv.take<char>(ts * n);
    d.u = cv.take<char>(ts * m);
    return cv.ok;
}

}  // namespace

extern "C" {

int solver_set_start(uv_solver *s, const double *x, const double *z, const double *delta, const double *lambda)
{
    if (!s) return UV_EINVAL;
    int rc = upload_state(s, x, z, delta, lambda);
    if (rc != UV_OK) return rc;
    s->need_start = false;
    return sync_status(s);
}

int solver_set_rhs(uv_solver *s, const double *b)
{
    if (!s || !b) return UV_EINVAL;
    for (int i = 0; i < s->m; ++i)
        if (!std::isfinite(b[i])) return UV_EINVAL;
    hipStream_t st = s->stream;
    UV_TRY(hipMemcpyAsync(s->b64, b, 8 * (size_t)s->m, hipMemcpyHostToDevice, st));
    if (s->o.precision == UV_MIXED)
        k_narrow<float><<<blocks_for(s->m, kWG), kWG, 0, st>>>(s->m, s->b64, (float *)s->b);
    k_norms<<<1, kWG, 0, st>>>(s->m, s->b64, s->n, s->c64, s->st);
    UV_TRY(hipGetLastError());
    int rc = sync_status(s);
    if (rc != UV_OK) return rc;
    // the residuals of the last check belong to the old b
    s->st_host->check_iter = -1;
    UV_TRY(hipMemcpyAsync(s->st, s->st_host, sizeof(DevStatus), hipMemcpyHostToDevice, st));
    UV_TRY(hipStreamSynchronize(st));
    s->need_start = true;
    return UV_OK;
}

int solver_resume(uv_solver *s, const double *x, const double *z, const double *delta, const double *lambda)
{
    if (!s) return UV_EINVAL;
    int rc = upload_state(s, x, z, delta, lambda);
    if (rc != UV_OK) return rc;
    s->need_start = false;
    launch_row(s, s->stream, 2);
    UV_TRY(hipGetLastError());
    return sync_status(s);
}

int solver_iterate(uv_solver *s, int64_t k, int32_t *done)
{
    if (!s || k < 0 || s->need_start) return UV_EINVAL;
    if (done) *done = 0;
    if (!s->st_host->done) {
        int64_t left = k;
        if (s->o.max_iter > 0) left = std::min<int64_t>(left, s->o.max_iter - s->host_iter);
        int64_t it = s->host_iter, since = 0;
        const int ce = s->o.check_every;
        const int64_t look = 50 * (int64_t)ce;  // read the stop flag every 50 checks
        if (s->resident && left > 0) {
            resident_launch(res_args(s), s->stream, left, false);
            left = 0;
        }
        while (left > 0) {
            if (s->exec && it % ce == 0 && left >= ce) {
                UV_TRY(hipGraphLaunch(s->exec, s->stream));
                it += ce;
                left -= ce;
                since += ce;
            } else {
                launch_iteration(s, s->stream, (it + 1) % ce == 0);
                it += 1;
                left -= 1;
                since += 1;
            }
            if (left > 0 && since >= look) {  // stop launching once a check has stopped the run
                UV_TRY(hipGetLastError());
                int rc = sync_status(s);
                if (rc != UV_OK) return rc;
                if (s->st_host->done) break;
                since = 0;
            }
        }
        UV_TRY(hipGetLastError());
        int rc = sync_status(s);
        if (rc != UV_OK) return rc;
    }
    DevStatus *h = s->st_host;
    if (!h->done && s->o.max_iter > 0 && s->host_iter >= s->o.max_iter) {
        h->status = UV_STATUS_MAX_ITER;
        h->done = 1;
        UV_TRY(hipMemcpyAsync(s->st, h, sizeof(DevStatus), hipMemcpyHostToDevice, s->stream));
        UV_TRY(hipStreamSynchronize(s->stream));
    }
    if (done) *done = h->done;
    return h->status == UV_STATUS_NUMERIC ? UV_ENUMERIC : UV_OK;
}

int solver_residuals(uv_solver *s, uv_residuals *r)
{
    if (!s || !r) return UV_EINVAL;
    if (s->st_host->check_iter != s->st_host->iter) {
        if (s->resident) resident_launch(res_args(s), s->stream, 0, true);
        else launch_residuals(s, s->stream, false, false);
        UV_TRY(hipGetLastError());
        int rc = sync_status(s);
        if (rc != UV_OK) return rc;
    }
    const DevStatus *h = s->st_host;
    r->r_prim = h->r_prim;
    r->r_dual = h->r_dual;
    r->r_gap = h->r_gap;
    r->kkt = h->kkt;
    r->pobj = h->pobj;
    r->dobj = h->dobj;
    r->res_ax_b = h->res_ax_b;
    r->prim_inf = h->prim_inf;
    r->dual_inf = h->dual_inf;
    r->scale_p = h->scale_p;
    r->scale_d = h->scale_d;
    r->iter = h->iter;
    r->status = h->status;
    r->pobj_x = h->pobj_x;
    r->gap_x = h->gap_x;
    return UV_OK;
}

int solver_solution(uv_solver *s, double *x, double *z, double *lambda, double *delta)
{
    if (!s) return UV_EINVAL;
    hipStream_t st = s->stream;
    const bool mixed = s->o.precision == UV_MIXED;
    auto get_t = [&](double *dst, const void *src, int len) -> int {
        if (!dst) return UV_OK;
        if (mixed) {
            k_widen<float><<<blocks_for(len, kWG), kWG, 0, st>>>(len, (const float *)src, s->scratch);
            src = s->scratch;
        }
        if (hipMemcpyAsync(dst, src, 8 * (size_t)len, hipMemcpyDeviceToHost, st) != hipSuccess) return UV_EHIP;
        return hipStreamSynchronize(st) == hipSuccess ? UV_OK : UV_EHIP;
    };
    int rc;
    if ((rc = get_t(x, s->x, s->n)) != UV_OK) return rc;
    if ((rc = get_t(z, s->z, s->n)) != UV_OK) return rc;
    if (lambda) UV_TRY(hipMemcpyAsync(lambda, s->lam, 8 * (size_t)s->m, hipMemcpyDeviceToHost, st));
    if (delta) UV_TRY(hipMemcpyAsync(delta, s->delta, 8 * (size_t)s->n, hipMemcpyDeviceToHost, st));
    UV_TRY(hipStreamSynchronize(st));
    return UV_OK;
}

int solver_history(uv_solver *s, int32_t max, uv_history *out, int32_t *count)
{
    if (!s || max < 0 || (max > 0 && !out) || !count) return UV_EINVAL;
    *count = 0;
    if (!s->hist || max == 0) return UV_OK;
    UV_TRY(hipMemcpyAsync(s->st_host, s->st, sizeof(DevStatus), hipMemcpyDeviceToHost, s->stream));
    UV_TRY(hipStreamSynchronize(s->stream));
    const long long written = s->st_host->hist_n, cap = s->o.history;
    const long long kept = std::min(written, cap), take = std::min<long long>(kept, max);
    const double per_s = s->clock_khz > 0 ? 1.0 / (s->clock_khz * 1e3) : 0.0;
    // the latest `take` records, oldest first: at most two runs of the ring
    std::vector<HistRec> h((size_t)take);
    const long long first = (written - take) % cap, run1 = std::min(take, cap - first);
    if (run1 > 0)
        UV_TRY(hipMemcpy(h.data(), s->hist + first, sizeof(HistRec) * (size_t)run1, hipMemcpyDeviceToHost));
    if (take > run1)
        UV_TRY(hipMemcpy(h.data() + run1, s->hist, sizeof(HistRec) * (size_t)(take - run1),
                         hipMemcpyDeviceToHost));
    for (long long q = 0; q < take; ++q) {
        const HistRec &r = h[(size_t)q];
        uv_history &o = out[q];
        o.iter = r.iter;
        o.seconds = (double)(r.clock - s->st_host->clock0) * per_s;
        o.r_prim = r.r_prim;
        o.r_dual = r.r_dual;
        o.r_gap = r.r_gap;
        o.kkt = r.kkt;
        o.pobj = r.pobj;
        o.dobj = r.dobj;
        o.res_ax_b = r.res_ax_b;
        o.gap_x = r.gap_x;
    }
    *count = (int32_t)take;
    return UV_OK;
}

int solver_solve(const uv_csr *A, const double *b, const double *c, const uv_cones *K, const uv_opts *opts,
                 int64_t iters, double *x, double *z, double *lambda, double *delta, uv_residuals *r)
{
    if (iters < 0) return UV_EINVAL;
    uv_solver *s = nullptr;
    int rc = solver_create(A, b, c, K, opts, &s);
    if (rc != UV_OK) return rc;
    int32_t done = 0;
    rc = solver_iterate(s, iters, &done);
    if (rc == UV_OK || rc == UV_ENUMERIC) {
        int rc2 = solver_solution(s, x, z, lambda, delta);
        if (rc2 == UV_OK && r) rc2 = solver_residuals(s, r);
        if (rc2 != UV_OK) rc = rc2;
    }
    solver_destroy(s);
    return rc;
}

int solver_solve_noalloc(const uv_csr *A, const double *b, const double *c, const uv_cones *K, const uv_opts *opts,
                         int64_t iters, double *x, double *z, double *lambda, double *delta, uv_residuals *r)
{
    if (iters < 0) return UV_EINVAL;
    uv_opts o;
    uv_default_opts(&o);
    if (opts) o = *opts;
    int rc = validate(A, b, c, K, &o);
    if (rc != UV_OK) return rc;
    if (o.resident == 1) return UV_EINVAL;  // this entry point is the resident path
    const bool mixed = o.precision == UV_MIXED;
    const int m = A->m, n = A->n, nnz = (int)A->nnz;
    const ResLayout L = mixed ? resident_layout<float>(m, n, nnz) : resident_layout<double>(m, n, nnz);
    if (K->n_soc != 0 || m >= 65536 || n >= 65536 || L.bytes > kResLdsMax) return UV_ENOSCRATCH;
    NoAlloc d{};
    Carve size{nullptr, 0, kScratchBytes, true};
    if (!carve_noalloc(size, m, n, nnz, mixed, d)) return UV_ENOSCRATCH;
    unsigned char *base = nullptr;
    if ((rc = scratch_address(&base)) != UV_OK) return rc;
    Carve cv{base, 0, kScratchBytes, true};
    carve_noalloc(cv, m, n, nnz, mixed, d);
    const hipError_t fe = mixed ? hipFuncSetAttribute((const void *)k_resident<float>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, kResLdsMax)
                                : hipFuncSetAttribute((const void *)k_resident<double>,
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, kResLdsMax);
    if (fe != hipSuccess) return UV_EHIP;
    hipStream_t st = (hipStream_t)o.hip_stream;
    const size_t ts = mixed ? 4 : 8;
    // inputs and the setup of solver_create
    UV_TRY(hipMemcpyAsync(d.rp64, A->row_ptr, 8 * ((size_t)m + 1), hipMemcpyHostToDevice, st));
    k_narrow_offsets<<<blocks_for(m + 1, kWG), kWG, 0, st>>>(m + 1, d.rp64, d.rp);
    if (nnz > 0) {
        UV_TRY(hipMemcpyAsync(d.ci, A->col_idx, 4 * (size_t)nnz, hipMemcpyHostToDevice, st));
        UV_TRY(hipMemcpyAsync(d.va64, A->val, 8 * (size_t)nnz, hipMemcpyHostToDevice, st));
    }
    UV_TRY(hipMemcpyAsync(d.b64, b, 8 * (size_t)m, hipMemcpyHostToDevice, st));
    UV_TRY(hipMemcpyAsync(d.c64, c, 8 * (size_t)n, hipMemcpyHostToDevice, st));
    if (!build_csc(m, n, nnz, d.rp, d.ci, d.va64, d.cp, d.ri, d.vc64, d.cnt, d.bsum, st)) return UV_EHIP;
    if (mixed) {
        k_row_factor<float><<<blocks_for(m, kWG), kWG, 0, st>>>(m, d.rp, d.va64, (float *)d.fu);
        if (nnz > 0) {
            k_narrow<float><<<blocks_for(nnz, kWG), kWG, 0, st>>>(nnz, d.va64, (float *)d.va);
            k_narrow<float><<<blocks_for(nnz, kWG), kWG, 0, st>>>(nnz, d.vc64, (float *)d.vc);
        }
        k_narrow<float><<<blocks_for(m, kWG), kWG, 0, st>>>(m, d.b64, (float *)d.b);
        k_narrow<float><<<blocks_for(n, kWG), kWG, 0, st>>>(n, d.c64, (float *)d.c);
    } else {
        k_row_factor<double><<<blocks_for(m, kWG), kWG, 0, st>>>(m, d.rp, d.va64, (double *)d.fu);
    }
    k_norms<<<1, kWG, 0, st>>>(m, d.b64, n, d.c64, d.st);
    // the zero start (everything the last call left in the scratch is overwritten)
    UV_TRY(hipMemsetAsync(d.x, 0, ts * n, st));
    UV_TRY(hipMemsetAsync(d.z, 0, ts * n, st));
    UV_TRY(hipMemsetAsync(d.delta, 0, 8 * (size_t)n, st));
    UV_TRY(hipMemsetAsync(d.lam, 0, 8 * (size_t)m, st));
    const double im = 1.0 / o.mu;
    if (mixed) k_start<float><<<blocks_for(m, kWG), kWG, 0, st>>>(m, d.lam, (float *)d.u, im, d.st);
    else k_start<double><<<blocks_for(m, kWG), kWG, 0, st>>>(m, d.lam, (double *)d.u, im, d.st);
    UV_TRY(hipGetLastError());
    ResArgs a{};
    a.m = m;
    a.n = n;
    a.L = L;
    a.Lr = resident_lanes(m);
    a.Lc = resident_lanes(n);
    a.rp = d.rp;
    a.ci = d.ci;
    a.cp = d.cp;
    a.ri = d.ri;
    a.va = d.va;
    a.vc = d.vc;
    a.b = d.b;
    a.c = d.c;
    a.fu = d.fu;
    a.va64 = d.va64;
    a.vc64 = d.vc64;
    a.b64 = d.b64;
    a.c64 = d.c64;
    a.x = d.x;
    a.z = d.z;
    a.u = d.u;
    a.lam = d.lam;
    a.delta = d.delta;
    a.st = d.st;
    a.hist = HistRing{nullptr, 0};
    a.gated = o.full_checks == 0 ? 1 : 0;
    a.mixed = mixed;
    a.mu = o.mu;
    a.eps = o.eps_kkt;
    a.eps_abs = o.eps_abs;
    a.eps_gap = o.eps_gap;
    a.check_every = o.check_every;
    a.crit = o.criterion;
    int64_t left = iters;
    if (o.max_iter > 0) left = std::min<int64_t>(left, o.max_iter);
    resident_launch(a, st, left, false);
    UV_TRY(hipGetLastError());
    DevStatus h{};
    UV_TRY(hipMemcpyAsync(&h, d.st, sizeof(DevStatus), hipMemcpyDeviceToHost, st));
    UV_TRY(hipStreamSynchronize(st));
    if (r && h.check_iter != h.iter) {  // residuals of the final iterate (no decision)
        resident_launch(a, st, 0, true);
        UV_TRY(hipGetLastError());
        const int status = h.status, stopped = h.done;
        UV_TRY(hipMemcpyAsync(&h, d.st, sizeof(DevStatus), hipMemcpyDeviceToHost, st));
        UV_TRY(hipStreamSynchronize(st));
        h.status = status;
        h.done = stopped;
    }
    if (!h.done && o.max_iter > 0 && h.iter >= o.max_iter) {
        h.status = UV_STATUS_MAX_ITER;
        h.done = 1;
    }
    // outputs
    auto get_t = [&](double *dst, const void *src) -> int {
        if (!dst) return UV_OK;
        if (mixed) {
            k_widen<float><<<blocks_for(n, kWG), kWG, 0, st>>>(n, (const float *)src, d.wide);
            src = d.wide;
        }
        if (hipMemcpyAsync(dst, src, 8 * (size_t)n, hipMemcpyDeviceToHost, st) != hipSuccess) return UV_EHIP;
        return hipStreamSynchronize(st) == hipSuccess ? UV_OK : UV_EHIP;
    };
    if ((rc = get_t(x, d.x)) != UV_OK) return rc;
    if ((rc = get_t(z, d.z)) != UV_OK) return rc;
    if (lambda) UV_TRY(hipMemcpyAsync(lambda, d.lam, 8 * (size_t)m, hipMemcpyDeviceToHost, st));
    if (delta) UV_TRY(hipMemcpyAsync(delta, d.delta, 8 * (size_t)n, hipMemcpyDeviceToHost, st));
    UV_TRY(hipStreamSynchronize(st));
    if (r) {
        r->r_prim = h.r_prim;
        r->r_dual = h.r_dual;
        r->r_gap = h.r_gap;
        r->kkt = h.kkt;
        r->pobj = h.pobj;
        r->dobj = h.dobj;
        r->res_ax_b = h.res_ax_b;
        r->prim_inf = h.prim_inf;
        r->dual_inf = h.dual_inf;
        r->scale_p = h.scale_p;
        r->scale_d = h.scale_d;
        r->iter = h.iter;
        r->status = h.status;
        r->pobj_x = h.pobj_x;
        r->gap_x = h.gap_x;
    }
    return h.status == UV_STATUS_NUMERIC ? UV_ENUMERIC : UV_OK;
}

int solver_time_kernels(uv_solver *s, int32_t iters, double *ms_col, double *ms_row)
{
    if (!s || iters < 1 || !ms_col || !ms_row) return UV_EINVAL;
    if (s->st_host->done || s->need_start) return UV_EINVAL;   // a stopped solver launches nothing to time
    std::vector<hipEvent_t> ev(3 * (size_t)iters, nullptr);
    int rc = UV_OK;
    for (auto &e : ev)
        if (hipEventCreate(&e) != hipSuccess) { rc = UV_EHIP; break; }
    if (rc == UV_OK) {
        for (int i = 0; i < iters; ++i) {
            (void)hipEventRecord(ev[3 * i], s->stream);
            launch_col(s, s->stream);
            (void)hipEventRecord(ev[3 * i + 1], s->stream);
            launch_row(s, s->stream, 0);
            (void)hipEventRecord(ev[3 * i + 2], s->stream);
        }
        if (hipStreamSynchronize(s->stream) != hipSuccess) rc = UV_EHIP;
    }
    double tc = 0.0, tr = 0.0;
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
        rc = sync_status(s);
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

int solver_launch_shape(const uv_solver *s, int32_t *shape)
{
    if (!s || !shape) return UV_EINVAL;
    shape[0] = s->L_row;
    shape[1] = s->E_row;
    shape[2] = s->L_col;
    shape[3] = s->E_col;
    shape[4] = s->S_row;
    shape[5] = s->S_col;
    shape[6] = s->resident ? 1 : 0;
    return UV_OK;
}

}  // extern "C"
