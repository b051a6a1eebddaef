// spmv.hpp -- the sparse product kernel of the slab passes, shared by the
// UV-decomposition solver and the standard-ADMM baseline.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace {

using uv::kWG;

// Chunked segment sums for the slab passes: out[s * nseg + g] = sum over the
// entries k of segment g in slab s of val[k] * vec[idx[k]].  A wavefront owns
// 64 consecutive segments (one per lane for the final sum): it streams their
// contiguous entries with coalesced loads, four 64-entry steps in flight per
// round, parks the products in LDS, and each lane then adds its own
// segment's products in entry order.  Unlike one lane group per segment this
// needs no per-segment pointer before the stream starts and keeps every lane
// busy however short the segments are.  Deterministic.  With S = 1 the
// arguments are a plain compressed-row (or -column) matrix.  The grid is
// S * ceil(nseg / kWG) workgroups; workgroup w works on slab w % S.
constexpr int kChunkCap = 512;  // LDS products per wavefront and round

// One workgroup's share of the chunked product: wavefront w of workgroup
// group `grp` owns segments (grp * 4 + w) * 64 + lane of slab `sl` and the
// function returns that segment's sum (0 past nseg).  No early exit, so a
// caller may synchronise the workgroup afterwards.  G is the type of the
// gathered vector (the FP64 residual products of the mixed-precision form
// gather FP32 iterates); products and sums are in T.
template <typename T, typename TV, int S, int U, typename G>
__device__ __forceinline__ T chunk_sum(int nseg, int sl, int grp, const int *__restrict__ ptr,
                                       const int *__restrict__ idx, const TV *__restrict__ val,
                                       const G *__restrict__ vec, T (*buf)[kChunkCap])
{
    static_assert(kChunkCap % (64 * U) == 0, "a round holds whole batches");
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int g0 = (grp * (kWG / 64) + w) * 64;
    T acc = 0;
    if (g0 >= nseg) return acc;  // the whole wavefront has no segment
    const int *p = ptr + (size_t)sl * nseg;  // p[nseg] is the slab's end
    const int gl = g0 + lane;
    const int beg = p[gl < nseg ? gl : nseg];
    const int e_last = p[min(g0 + 64, nseg)];
    int end = __shfl_down(beg, 1);
    if (lane == 63) end = e_last;
    const int E0 = __shfl(beg, 0), E1 = e_last;
    for (int P0 = E0; P0 < E1; P0 += kChunkCap) {
        const int P1 = min(P0 + kChunkCap, E1);
        for (int b = P0; b < P1; b += 64 * U) {  // U coalesced 64-entry steps in flight
            int j[U];
            TV v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = b + u * 64 + lane;
                const int kk = k < P1 ? k : P1 - 1;
                j[u] = __builtin_nontemporal_load(idx + kk);
                v[u] = __builtin_nontemporal_load(val + kk);
            }
            G g[U];
#pragma unroll
            for (int u = 0; u < U; ++u) g[u] = vec[j[u]];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = b + u * 64 + lane;
                if (k < P1) buf[w][k - P0] = (T)v[u] * (T)g[u];
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int a = max(beg, P0), z = min(end, P1);
        for (int k = a; k < z; ++k) acc += buf[w][k - P0];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    return acc;
}

template <typename T, typename TV, int S, int U = 4, typename G = T>
__global__ void __launch_bounds__(kWG)
k_seg_chunk(int nseg, const int *__restrict__ ptr, const int *__restrict__ idx, const TV *__restrict__ val,
            const G *__restrict__ vec, T *__restrict__ out, const int *skip)
{
    if (skip && *skip) return;  // a device flag (stop, or nothing left to do)
    __shared__ T buf[kWG / 64][kChunkCap];
    const int sl = blockIdx.x % S, grp = blockIdx.x / S;
    const T acc = chunk_sum<T, TV, S, U, G>(nseg, sl, grp, ptr, idx, val, vec, buf);
    const int gl = grp * kWG + threadIdx.x;
    if (gl < nseg) out[(size_t)sl * nseg + gl] = acc;
}

// Sum of the S slab partials of one segment in a fixed pairwise tree:
// leaves 0 + p_s (a lone -0 becomes +0, as in a running sum from zero),
// then (p0 + p1), (p2 + p3), ... and so on up; every update kernel adds the
// partials this way, so results do not depend on the kernel.
template <int S, typename T>
__device__ __forceinline__ T slab_tree_sum(const T *__restrict__ P, size_t stride, size_t i)
{
    T v[S];
#pragma unroll
    for (int q = 0; q < S; ++q) v[q] = (T)0 + P[(size_t)q * stride + i];
#pragma unroll
    for (int w = S; w > 1; w >>= 1)
#pragma unroll
        for (int k = 0; k < w / 2; ++k) v[k] = v[2 * k] + v[2 * k + 1];
    return v[0];
}

// Slabs of the gathered vector (`bytes` long) for the row pass (x gathered,
// one partial per row) and the column pass (u gathered, one partial per
// column, about twice as many).  A slab part of at most 2-4 MiB keeps the
// gathers in an XCD's L2 (random-gather probe: 150-170 G/s against 70 G/s
// from 16 MiB), and every slab adds a partial per segment; measured with the
// eight-step chunk kernel on the 1e6 x 2e6 LP and the 1e5-cone SOCP: row
// pass best in 4 slabs from x of 8 MiB (FP32) up, column pass best in 2
// slabs for u of 4-11 MiB.
inline int pick_slabs_row(size_t bytes)
{
    if (bytes <= (2u << 20)) return 1;
    return bytes <= (6u << 20) ? 2 : 4;
}

inline int pick_slabs_col(size_t bytes)
{
    if (bytes <= (2u << 20)) return 1;
    return bytes <= (16u << 20) ? 2 : 4;
}

}  // namespace
