// probe.hip -- measurement of the chip's random-gather rate, the practical
// bound of the sweep's sparse products.  A product over a random sparse
// matrix streams (index, value) pairs, which HBM serves near its peak, and
// gathers one vector entry per pair at a random address, which the cache
// hierarchy serves one request at a time.  This kernel does only that: every
// thread streams eight pairs with coalesced loads, gathers eight table
// entries and stores one sum, so its duration is a floor for a product with
// the same number of pairs, the same table and the same slab split.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/uvadmm.h"
#include "common.hpp"

namespace {

using uv::kWG;
constexpr int kPerThread = 8;

__device__ __forceinline__ uint64_t mix(uint64_t x)
{
    // splitmix64 finalizer (Steele, Lea, Flood, "Fast splittable pseudorandom number generators")
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

template <typename T>
__global__ void __launch_bounds__(kWG) k_probe_fill(int64_t nnz, int slab_len, uint64_t seed, int *idx, T *val)
{
    const int64_t k = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (k >= nnz) return;
    idx[k] = (int)(mix(seed ^ (uint64_t)k) % (uint64_t)slab_len);
    val[k] = (T)1;
}

template <typename T>
__global__ void __launch_bounds__(kWG) k_probe_table(int64_t len, T *tab)
{
    const int64_t k = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (k < len) tab[k] = (T)0.5;
}

// Workgroup w streams pairs [w * kWG * 8, (w + 1) * kWG * 8) and gathers
// from table part w % slabs (slab_len entries each).
template <typename T>
__global__ void __launch_bounds__(kWG)
k_probe_gather(int64_t nnz, const int *__restrict__ idx, const T *__restrict__ val, const T *__restrict__ tab,
               T *__restrict__ out, int slabs, int slab_len)
{
    const int64_t base = (int64_t)blockIdx.x * kWG * kPerThread + threadIdx.x;
    const T *part = tab + (int64_t)(blockIdx.x % slabs) * slab_len;
    int j[kPerThread];
    T v[kPerThread];
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) {
        int64_t k = base + (int64_t)u * kWG;
        if (k >= nnz) k = nnz - 1;
        j[u] = __builtin_nontemporal_load(idx + k);
        v[u] = __builtin_nontemporal_load(val + k);
    }
    T g[kPerThread];
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) g[u] = part[j[u]];
    T acc = 0;
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) acc += v[u] * g[u];
    out[(int64_t)blockIdx.x * kWG + threadIdx.x] = acc;
}

template <typename T>
int run(int64_t nnz, int64_t table_len, int slabs, int reps, uint64_t seed, double *ms)
{
    const int slab_len = (int)(table_len / slabs);
    const int64_t nblk = (nnz + (int64_t)kWG * kPerThread - 1) / ((int64_t)kWG * kPerThread);
    int *idx = nullptr;
    T *val = nullptr, *tab = nullptr, *out = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = UV_OK;
    if (uv::dev_malloc(&idx, 4 * nnz) != hipSuccess || uv::dev_malloc(&val, sizeof(T) * nnz) != hipSuccess ||
        uv::dev_malloc(&tab, sizeof(T) * table_len) != hipSuccess ||
        uv::dev_malloc(&out, sizeof(T) * nblk * kWG) != hipSuccess)
        rc = UV_ENOMEM;
    if (rc == UV_OK && (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
                        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = UV_EHIP;
    if (rc == UV_OK) {
        k_probe_fill<T><<<(unsigned)((nnz + kWG - 1) / kWG), kWG, 0, st>>>(nnz, slab_len, seed, idx, val);
        k_probe_table<T><<<(unsigned)((table_len + kWG - 1) / kWG), kWG, 0, st>>>(table_len, tab);
        k_probe_gather<T><<<(unsigned)nblk, kWG, 0, st>>>(nnz, idx, val, tab, out, slabs, slab_len);  // warm-up
        (void)hipEventRecord(e0, st);
        for (int r = 0; r < reps; ++r)
            k_probe_gather<T><<<(unsigned)nblk, kWG, 0, st>>>(nnz, idx, val, tab, out, slabs, slab_len);
        (void)hipEventRecord(e1, st);
        float t = 0.f;
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess)
            rc = UV_EHIP;
        else
            *ms = (double)t / reps;
    }
    if (st) (void)hipStreamSynchronize(st);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (st) (void)hipStreamDestroy(st);
    for (void *p : {(void *)idx, (void *)val, (void *)tab, (void *)out})
        if (p) (void)hipFree(p);
    return rc;
}

}  // namespace

extern "C" int probe_gather(int64_t nnz, int64_t table_len, int32_t slabs, int32_t fp64, int32_t reps,
                            uint64_t seed, double *ms)
{
    if (!ms || nnz < 1 || nnz >= ((int64_t)1 << 31) || reps < 1 || slabs < 1 || slabs > 8) return UV_EINVAL;
    if (table_len < slabs || table_len / slabs >= ((int64_t)1 << 31)) return UV_EINVAL;
    return fp64 ? run<double>(nnz, table_len, slabs, reps, seed, ms) : run<float>(nnz, table_len, slabs, reps, seed, ms);
}
