// common.hpp -- shared device helpers of the gfx950 solver library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace uv {

constexpr int kWG = 256;      // threads per workgroup for every sweep kernel
constexpr int kWave = 64;     // CDNA wavefront width

// Sum over the L consecutive lanes of a group (L a power of two <= 64); the
// butterfly leaves the total in every lane of the group.  A fixed pattern,
// so results are bitwise reproducible.
template <int L, typename T>
__device__ __forceinline__ T group_sum(T v)
{
#pragma unroll
    for (int off = L / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, L);
    return v;
}

// Workgroup sum of K doubles, deterministic (wave butterfly, then thread 0
// adds the per-wave totals in wave order).  Thread 0 writes component k to
// out[k * stride].
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double *out, int stride)
{
    __shared__ double s[K][kWG / kWave];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = group_sum<kWave>(v[k]);
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) s[k][w] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double t = 0.0;
#pragma unroll
            for (int i = 0; i < kWG / kWave; ++i) t += s[k][i];
            out[k * stride] = t;
        }
    }
}

}  // namespace uv
