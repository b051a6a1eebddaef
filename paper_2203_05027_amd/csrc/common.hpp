// common.hpp -- shared device helpers of the gfx950 solver library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <atomic>

namespace uv {

// Allocation-failure test hook (uv_test_fail_alloc): while armed (>= 0) it
// counts down on every device or pinned-host allocation made through the two
// helpers below, and the allocation that finds it at zero fails as if the
// memory were exhausted; the hook then disarms itself.
inline std::atomic<long long> g_alloc_fail_after{-1};

inline bool alloc_hook_fires()
{
    long long k = g_alloc_fail_after.load();
    while (k >= 0) {
        if (g_alloc_fail_after.compare_exchange_weak(k, k - 1)) return k == 0;
    }
    return false;
}

template <typename T>
inline hipError_t dev_malloc(T **p, size_t bytes)
{
    if (alloc_hook_fires()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipMalloc((void **)p, bytes);
}

template <typename T>
inline hipError_t host_malloc(T **p, size_t bytes, unsigned flags)
{
    if (alloc_hook_fires()) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    return hipHostMalloc((void **)p, bytes, flags);
}

// Relative KKT residual: the largest of the three relative residuals, and
// NaN when any of them is NaN (fmax alone would drop a NaN operand and hide
// a numeric failure behind the other two).
__device__ __forceinline__ double kkt_of(double rp, double rd, double rg)
{
    const double k = fmax(rp, fmax(rd, rg));
    return (isnan(rp) || isnan(rd) || isnan(rg)) ? __builtin_nan("") : k;
}

constexpr int kWG = 256;      // threads per workgroup for every sweep kernel
constexpr int kWave = 64;     // CDNA wavefront width

// v of lane ^ 1 (CTRL 0xB1) or lane ^ 2 (CTRL 0x4E): a DPP quad permutation,
// a register move with no LDS traffic.
template <int CTRL>
__device__ __forceinline__ float dpp_quad(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF,
                                                                   false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_quad(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the L consecutive lanes of a group (L a power of two <= 64, a
// run-time value; every lane of a group active or none); the butterfly,
// widest offset first, leaves the total in every lane of the group.  The
// offsets 2 and 1 are DPP quad moves, the wider ones cross-lane permutes:
// the same pairs and order either way, so results are bitwise reproducible.
template <typename T>
__device__ __forceinline__ T lane_sum(T v, int L)
{
    for (int off = L >> 1; off >= 4; off >>= 1) v += __shfl_xor(v, off, L);
    if (L >= 4) v += dpp_quad<0x4E>(v);
    if (L >= 2) v += dpp_quad<0xB1>(v);
    return v;
}

template <int L, typename T>
__device__ __forceinline__ T group_sum(T v)
{
    return lane_sum<T>(v, L);
}

// A wavefront's sum (MAX = false) or maximum of a double, in lane 0: pairs
// within quads, then the other quad of each half row and the other half of
// each row of 16 lanes (DPP moves, no LDS traffic), then the four row totals
// read across the wavefront and combined as (r0 + r1) + (r2 + r3).  A fixed
// order, so results are bitwise reproducible (not the same order as
// group_sum<64>).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ __forceinline__ double read_lane(double v, int lane)
{
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane), hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}

template <bool MAX>
__device__ __forceinline__ double wave_fold0(double v)
{
    auto op = [](double a, double b) { return MAX ? fmax(a, b) : a + b; };
    v = op(v, dpp_move<0xB1>(v));   // quad_perm 1,0,3,2: lane ^ 1
    v = op(v, dpp_move<0x4E>(v));   // quad_perm 2,3,0,1: lane ^ 2
    v = op(v, dpp_move<0x141>(v));  // row_half_mirror: the other quad of the half row
    v = op(v, dpp_move<0x140>(v));  // row_mirror: the other half of the row
    return op(op(read_lane(v, 0), read_lane(v, 16)), op(read_lane(v, 32), read_lane(v, 48)));
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

// Workgroup reduction of KS sums and KM maxima (deterministic); thread 0
// writes sum k to out[k * stride] and maximum k to out[(KS + k) * stride].
template <int KS, int KM>
__device__ __forceinline__ void block_sum_max(double (&vs)[KS], double (&vm)[KM], double *out, int stride)
{
    __shared__ double s[KS + KM][kWG / kWave];
#pragma unroll
    for (int k = 0; k < KS; ++k) vs[k] = group_sum<kWave>(vs[k]);
#pragma unroll
    for (int k = 0; k < KM; ++k)
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1) vm[k] = fmax(vm[k], __shfl_xor(vm[k], off, kWave));
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < KS; ++k) s[k][w] = vs[k];
#pragma unroll
        for (int k = 0; k < KM; ++k) s[KS + k][w] = vm[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < KS + KM; ++k) {
            double t = s[k][0];
#pragma unroll
            for (int i = 1; i < kWG / kWave; ++i) t = k < KS ? t + s[k][i] : fmax(t, s[k][i]);
            out[k * stride] = t;
        }
    }
}

}  // namespace uv
