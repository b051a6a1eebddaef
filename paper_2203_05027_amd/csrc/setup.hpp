// setup.hpp -- setup kernels shared by the single-problem and batched solvers
// (the set-up of Algorithm 1: the UV decomposition is implicit in the CSR and
// CSC copies of A; F_U and F_V are diagonal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace {

using uv::kWG;

// F_U[i] = 1 / (1 + sum_j A_ij^2)   (U U' is diagonal: squared row norms)
template <typename T>
__global__ void __launch_bounds__(kWG)
k_row_factor(int m, const int *__restrict__ rp, const double *__restrict__ va, T *__restrict__ fu)
{
    int i = blockIdx.x * kWG + threadIdx.x;
    if (i >= m) return;
    double d = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) d += va[k] * va[k];
    fu[i] = (T)(1.0 / (1.0 + d));
}

// Column-major copy of A (the pattern of V): count, scan, scatter, then a
// per-column sort by row so the layout is deterministic.
__global__ void __launch_bounds__(kWG)
k_col_count(int nnz, const int *__restrict__ ci, int *__restrict__ cnt)
{
    int k = blockIdx.x * kWG + threadIdx.x;
    if (k < nnz) atomicAdd(&cnt[ci[k]], 1);
}

// Inclusive scan of 4*kWG items per workgroup; block totals to bsum.
__global__ void __launch_bounds__(kWG)
k_scan_local(int n, const int *__restrict__ in, int *__restrict__ out, int *__restrict__ bsum)
{
    __shared__ int s[kWG];
    const int base = blockIdx.x * 4 * kWG + threadIdx.x * 4;
    int v[4], t = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        v[r] = (base + r < n) ? in[base + r] : 0;
        t += v[r];
        v[r] = t;
    }
    s[threadIdx.x] = t;
    __syncthreads();
    for (int off = 1; off < kWG; off <<= 1) {
        int a = (threadIdx.x >= off) ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += a;
        __syncthreads();
    }
    int excl = s[threadIdx.x] - t;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (base + r < n) out[base + r] = v[r] + excl;
    if (threadIdx.x == kWG - 1) bsum[blockIdx.x] = s[kWG - 1];
}

// Exclusive scan of the block totals, one workgroup, chunk by chunk.
__global__ void __launch_bounds__(kWG) k_scan_blocks(int nb, int *__restrict__ bsum)
{
    __shared__ int s[kWG];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += kWG) {
        int i = base + threadIdx.x;
        int v = (i < nb) ? bsum[i] : 0;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < kWG; off <<= 1) {
            int a = (threadIdx.x >= off) ? s[threadIdx.x - off] : 0;
            __syncthreads();
            s[threadIdx.x] += a;
            __syncthreads();
        }
        if (i < nb) bsum[i] = carry + s[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == kWG - 1) carry += s[kWG - 1];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kWG)
k_scan_add(int n, int *__restrict__ out, const int *__restrict__ bsum)
{
    int i = blockIdx.x * kWG + threadIdx.x;
    if (i < n) out[i] += bsum[i / (4 * kWG)];
}

__global__ void __launch_bounds__(kWG)
k_col_scatter(int m, const int *__restrict__ rp, const int *__restrict__ ci, const double *__restrict__ va,
              const int *__restrict__ cp, int *__restrict__ fill, int *__restrict__ ri, double *__restrict__ vc)
{
    int i = blockIdx.x * kWG + threadIdx.x;
    if (i >= m) return;
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
        int j = ci[k];
        int pos = cp[j] + atomicAdd(&fill[j], 1);
        ri[pos] = i;
        vc[pos] = va[k];
    }
}

__device__ void sift_down(int *key, double *val, int root, int len)
{
    for (;;) {
        int child = 2 * root + 1;
        if (child >= len) return;
        if (child + 1 < len && key[child + 1] > key[child]) ++child;
        if (key[root] >= key[child]) return;
        int tk = key[root]; key[root] = key[child]; key[child] = tk;
        double tv = val[root]; val[root] = val[child]; val[child] = tv;
        root = child;
    }
}

// Sorts each column's (row, value) pairs by row: insertion sort for short
// columns, heapsort otherwise (rows within a column are distinct).
__global__ void __launch_bounds__(kWG)
k_col_sort(int n, const int *__restrict__ cp, int *__restrict__ ri, double *__restrict__ vc)
{
    int j = blockIdx.x * kWG + threadIdx.x;
    if (j >= n) return;
    int *key = ri + cp[j];
    double *val = vc + cp[j];
    int len = cp[j + 1] - cp[j];
    if (len <= 32) {
        for (int a = 1; a < len; ++a) {
            int kk = key[a];
            double vv = val[a];
            int p = a - 1;
            while (p >= 0 && key[p] > kk) { key[p + 1] = key[p]; val[p + 1] = val[p]; --p; }
            key[p + 1] = kk;
            val[p + 1] = vv;
        }
        return;
    }
    for (int r = len / 2 - 1; r >= 0; --r) sift_down(key, val, r, len);
    for (int e = len - 1; e > 0; --e) {
        int tk = key[0]; key[0] = key[e]; key[e] = tk;
        double tv = val[0]; val[0] = val[e]; val[e] = tv;
        sift_down(key, val, 0, e);
    }
}

template <typename T>
__global__ void __launch_bounds__(kWG) k_narrow(int64_t len, const double *__restrict__ src, T *__restrict__ dst)
{
    int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i < len) dst[i] = (T)src[i];
}

template <typename T>
__global__ void __launch_bounds__(kWG) k_widen(int64_t len, const T *__restrict__ src, double *__restrict__ dst)
{
    int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i < len) dst[i] = (double)src[i];
}

// Slab split of a compressed-row-like matrix (nr rows, ptr, idx): entry k
// of row r belongs to slab min(idx[k] / w, S - 1) (S <= 8 contiguous index
// ranges).  cnt[s * nr + r] = entries of row r in slab s.
__global__ void __launch_bounds__(kWG)
k_slab_count(int nr, const int *__restrict__ ptr, const int *__restrict__ idx, int S, int w, int *__restrict__ cnt)
{
    const int r = blockIdx.x * kWG + threadIdx.x;
    if (r >= nr) return;
    int c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = ptr[r]; k < ptr[r + 1]; ++k) c[min(idx[k] / w, S - 1)]++;
    for (int s = 0; s < S; ++s) cnt[(int64_t)s * nr + r] = c[s];
}

// Scatter into the slab-major copy: off (S * nr + 1 entries, exclusive
// prefix sums of cnt) gives where row r of slab s starts.  Entries keep
// their order within a row, so the copy is deterministic.
__global__ void __launch_bounds__(kWG)
k_slab_scatter(int nr, const int *__restrict__ ptr, const int *__restrict__ idx, const double *__restrict__ val,
               int S, int w, const int *__restrict__ off, int *__restrict__ sidx, double *__restrict__ sval)
{
    const int r = blockIdx.x * kWG + threadIdx.x;
    if (r >= nr) return;
    int pos[8];
    for (int s = 0; s < S; ++s) pos[s] = off[(int64_t)s * nr + r];
    for (int k = ptr[r]; k < ptr[r + 1]; ++k) {
        const int p = pos[min(idx[k] / w, S - 1)]++;
        sidx[p] = idx[k];
        sval[p] = val[k];
    }
}

inline unsigned blocks_for(int64_t items, int per_block)
{
    return (unsigned)((items + per_block - 1) / per_block);
}

// out[0] = 0, out[i + 1] = in[0] + ... + in[i] for i < len; bsum needs
// ceil(len / (4 * kWG)) ints.
inline bool scan_exclusive(int len, const int *in, int *out, int *bsum, hipStream_t st)
{
    const int nscan = (int)blocks_for(len, 4 * kWG);
    if (hipMemsetAsync(out, 0, 4, st) != hipSuccess) return false;
    k_scan_local<<<nscan, kWG, 0, st>>>(len, in, out + 1, bsum);
    k_scan_blocks<<<1, kWG, 0, st>>>(nscan, bsum);
    k_scan_add<<<blocks_for(len, kWG), kWG, 0, st>>>(len, out + 1, bsum);
    return hipGetLastError() == hipSuccess;
}

// Slab-major copy of a compressed-row-like matrix (see k_slab_count):
// off (S * nr + 1), sidx and sval (nnz each); cnt (S * nr ints) and bsum
// (ceil(S * nr / (4 * kWG)) ints) are scratch.
inline bool build_slabs(int nr, int nnz, const int *ptr, const int *idx, const double *val, int S, int w, int *off,
                        int *sidx, double *sval, int *cnt, int *bsum, hipStream_t st)
{
    k_slab_count<<<blocks_for(nr, kWG), kWG, 0, st>>>(nr, ptr, idx, S, w, cnt);
    if (!scan_exclusive(S * nr, cnt, off, bsum, st)) return false;
    if (nnz > 0) k_slab_scatter<<<blocks_for(nr, kWG), kWG, 0, st>>>(nr, ptr, idx, val, S, w, off, sidx, sval);
    return hipGetLastError() == hipSuccess;
}

// Column-major copy (cp, ri, vc) of the CSR matrix (rp, ci, va): counting
// sort by column, then each column sorted by row.  cnt needs n ints and
// bsum ceil(n / (4 * kWG)) ints of scratch.  Returns false if a launch or
// memset failed.
inline bool build_csc(int m, int n, int nnz, const int *rp, const int *ci, const double *va, int *cp, int *ri,
                      double *vc, int *cnt, int *bsum, hipStream_t st)
{
    const int nscan = (int)blocks_for(n, 4 * kWG);
    if (hipMemsetAsync(cnt, 0, (size_t)n * 4, st) != hipSuccess) return false;
    if (hipMemsetAsync(cp, 0, 4, st) != hipSuccess) return false;
    if (nnz > 0) k_col_count<<<blocks_for(nnz, kWG), kWG, 0, st>>>(nnz, ci, cnt);
    k_scan_local<<<nscan, kWG, 0, st>>>(n, cnt, cp + 1, bsum);
    k_scan_blocks<<<1, kWG, 0, st>>>(nscan, bsum);
    k_scan_add<<<blocks_for(n, kWG), kWG, 0, st>>>(n, cp + 1, bsum);
    if (hipMemsetAsync(cnt, 0, (size_t)n * 4, st) != hipSuccess) return false;
    k_col_scatter<<<blocks_for(m, kWG), kWG, 0, st>>>(m, rp, ci, va, cp, cnt, ri, vc);
    k_col_sort<<<blocks_for(n, kWG), kWG, 0, st>>>(n, cp, ri, vc);
    return hipGetLastError() == hipSuccess;
}

}  // namespace
