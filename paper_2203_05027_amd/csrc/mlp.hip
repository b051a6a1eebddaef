// mlp.hip -- the learned warm start's network: a multilayer perceptron
// (ReLU hidden layers, linear output) whose GEMMs run on gfx950's BF16
// matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation) from
// LDS-staged tiles, trained on a mean squared error with Adam.  Master
// weights, biases, gradients and the Adam moments are FP32; each GEMM reads
// BF16 copies of its operands.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/uvadmm.h"
#include "common.hpp"

namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (NaN stays NaN).
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

enum Epi {
    EPI_F32 = 0,        // C (FP32)
    EPI_BIAS_RELU = 1,  // relu(C + bias) -> BF16 activation
    EPI_BIAS_F32 = 2,   // C + bias -> FP32 output
    EPI_MASK = 3,       // C * [act > 0] -> FP32 and BF16 (gradient through a ReLU)
};

// How a GEMM operand tile is read from global memory: 16-byte loads of
// eight elements consecutive along k (KC) or along the tile's other
// dimension (MC: m for A, n for B), or one element at a time (EL) when
// neither stride is 1 or the addresses are not 16-byte aligned.
enum LoadMode { LD_KC = 0, LD_MC = 1, LD_EL = 2 };

constexpr int kBK = 64;           // k per staged step (two 16x16x32 MFMAs)
constexpr int kLK = kBK + 8;      // LDS row pitch in elements (144 bytes: 16-byte aligned rows)

// The loads of one operand tile (ROWS rows of the tile's m or n dimension,
// k0..k0+63) of a thread: ROWS * 8 / 256 chunks of eight elements, held in
// registers between the global loads and the LDS stores so that the next
// tile's loads are in flight while the current tile is multiplied.
// Element (r, k) of the operand is P[r * rs + k * ks]; rows >= R and k >= K
// are zero.  KC: chunks along k (row c / 8, k (c % 8) * 8); MC: chunks along
// the rows (k c % 64, rows (c / 64) * 8), so that the 64 lanes of a
// wavefront store their transposed elements to 64 consecutive k of one row
// (no LDS bank conflicts; lanes eight rows apart would all meet in one or
// two banks, whatever the 16-byte-aligned pitch).
template <int MODE, int ROWS>
struct TileLoad {
    static constexpr int kChunks = ROWS * kBK / 8 / 256;
    static_assert(kChunks >= 1 && ROWS * kBK / 8 % 256 == 0, "whole chunks per thread");
    uint4 v[kChunks];

    __device__ __forceinline__ void load(const uint16_t *__restrict__ P, int64_t rs, int64_t ks, int r0, int R,
                                         int k0, int K)
    {
#pragma unroll
        for (int q = 0; q < kChunks; ++q) {
            const int c = threadIdx.x + q * 256;
            v[q] = uint4{0u, 0u, 0u, 0u};
            if (MODE == LD_KC) {
                const int gr = r0 + (c >> 3), gk = k0 + (c & 7) * 8;
                if (gr < R && gk < K) v[q] = *(const uint4 *)(P + (int64_t)gr * rs + gk);
            } else {
                const int gk = k0 + c % kBK, gr = r0 + (c / kBK) * 8;
                if (gr < R && gk < K) v[q] = *(const uint4 *)(P + (int64_t)gk * ks + gr);
            }
        }
    }

    // into LDS as T[row][k] (k contiguous, pitch kLK)
    __device__ __forceinline__ void store(uint16_t *__restrict__ T) const
    {
#pragma unroll
        for (int q = 0; q < kChunks; ++q) {
            const int c = threadIdx.x + q * 256;
            if (MODE == LD_KC) {
                *(uint4 *)(T + (c >> 3) * kLK + (c & 7) * 8) = v[q];
            } else {
                const int kk = c % kBK, r8 = (c / kBK) * 8;
                const uint16_t *e = (const uint16_t *)&v[q];
#pragma unroll
                for (int t = 0; t < 8; ++t) T[(r8 + t) * kLK + kk] = e[t];
            }
        }
    }
};

// The element-wise form (no unit stride or unaligned operands): straight
// into LDS.
template <int ROWS>
__device__ __forceinline__ void stage_el(const uint16_t *__restrict__ P, int64_t rs, int64_t ks, int r0, int R,
                                         int k0, int K, uint16_t *__restrict__ T)
{
    for (int c = threadIdx.x; c < ROWS * kBK; c += 256) {
        const int r = c / kBK, kk = c % kBK, gr = r0 + r, gk = k0 + kk;
        T[r * kLK + kk] = (gr < R && gk < K) ? P[(int64_t)gr * rs + (int64_t)gk * ks] : (uint16_t)0;
    }
}

// C (M x N) = A (M x K) B (K x N) on BF16 operands with FP32 accumulation;
// A(i,k) = A[i*a_rs + k*a_cs], B(k,j) = B[k*b_rs + j*b_cs]; M, N, K
// multiples of 16.  A workgroup (four wavefronts, 2 x 2) owns a block of
// (32 TM) x (32 TN) entries of C, a wavefront (16 TM) x (16 TN): TM x TN
// accumulators of the 16x16x32 MFMA.  Each 64-deep k step stages the
// block's A rows and B columns in LDS, k contiguous, from coalesced 16-byte
// loads issued during the previous step's products; lane l reads its
// operands as one 16-byte LDS load each: A[l % 16][8 (l / 16) .. +7] and
// B[8 (l / 16) .. +7][l % 16] of a 32-wide half step, and holds
// C[4 (l / 16) .. +3][l % 16] of each tile.
template <int EPI, int TM, int TN, int AM, int BMODE>
__global__ void __launch_bounds__(256)
k_mfma_gemm(int M, int N, int K, const uint16_t *__restrict__ A, int64_t a_rs, int64_t a_cs,
            const uint16_t *__restrict__ B, int64_t b_rs, int64_t b_cs, float *__restrict__ Cf,
            uint16_t *__restrict__ Cb, int64_t ldc, const float *__restrict__ bias,
            const uint16_t *__restrict__ act)
{
    constexpr int BM = 32 * TM, BN = 32 * TN;
    constexpr bool PREFETCH = AM != LD_EL && BMODE != LD_EL;
    __shared__ __align__(16) uint16_t As[BM * kLK];
    __shared__ __align__(16) uint16_t Bs[BN * kLK];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int tiles_n = (N + BN - 1) / BN;
    const int m0 = (blockIdx.x / tiles_n) * BM, n0 = (blockIdx.x % tiles_n) * BN;
    const int r = lane & 15, kq = lane >> 4;
    v4f acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    // A tile: rows m (A(m, k) = A[m a_rs + k a_cs]); B tile: rows n (B(k, n) = B[n b_cs + k b_rs])
    TileLoad<AM == LD_EL ? LD_KC : AM, BM> la;
    TileLoad<BMODE == LD_EL ? LD_KC : BMODE, BN> lb;
    if (PREFETCH) {
        la.load(A, a_rs, a_cs, m0, M, 0, K);
        lb.load(B, b_cs, b_rs, n0, N, 0, K);
    }
    for (int k0 = 0; k0 < K; k0 += kBK) {
        if (PREFETCH) {
            la.store(As);
            lb.store(Bs);
        } else {
            stage_el<BM>(A, a_rs, a_cs, m0, M, k0, K, As);
            stage_el<BN>(B, b_cs, b_rs, n0, N, k0, K, Bs);
        }
        __syncthreads();
        if (PREFETCH && k0 + kBK < K) {
            la.load(A, a_rs, a_cs, m0, M, k0 + kBK, K);
            lb.load(B, b_cs, b_rs, n0, N, k0 + kBK, K);
        }
#pragma unroll
        for (int h = 0; h < kBK / 32; ++h) {
            v8bf af[TM], bf[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i)
                af[i] = *(const v8bf *)(As + (wm * 16 * TM + i * 16 + r) * kLK + h * 32 + kq * 8);
#pragma unroll
            for (int j = 0; j < TN; ++j)
                bf[j] = *(const v8bf *)(Bs + (wn * 16 * TN + j * 16 + r) * kLK + h * 32 + kq * 8);
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
            const int col = n0 + wn * 16 * TN + j * 16 + r;
            if (col >= N) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = m0 + wm * 16 * TM + i * 16 + kq * 4 + e;
                if (row >= M) continue;
                const int64_t o = (int64_t)row * ldc + col;
                float v = acc[i][j][e];
                if (EPI == EPI_F32) {
                    Cf[o] = v;
                } else if (EPI == EPI_BIAS_RELU) {
                    v += bias[col];
                    Cb[o] = f2bf(v > 0.f ? v : 0.f);
                } else if (EPI == EPI_BIAS_F32) {
                    Cf[o] = v + bias[col];
                } else {
                    v = bf2f(act[o]) > 0.f ? v : 0.f;
                    Cf[o] = v;
                    Cb[o] = f2bf(v);
                }
            }
        }
}

__global__ void __launch_bounds__(256) k_to_bf16(int64_t len, const float *__restrict__ x, uint16_t *__restrict__ y)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t < len) y[t] = f2bf(x[t]);
}

// Loss = mean((Y - T)^2) and dY = 2 (Y - T) / len, FP32 and BF16; one
// workgroup, fixed summation order.
__global__ void __launch_bounds__(256)
k_mse(int64_t len, const float *__restrict__ Y, const float *__restrict__ T, float *__restrict__ dYf,
      uint16_t *__restrict__ dYb, float *__restrict__ loss)
{
    __shared__ double s[256];
    double acc = 0.0;
    const float sc = 2.0f / (float)len;
    for (int64_t t = threadIdx.x; t < len; t += 256) {
        const float d = Y[t] - T[t];
        acc += (double)d * d;
        const float g = sc * d;
        dYf[t] = g;
        dYb[t] = f2bf(g);
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(s[0] / (double)len);
}

// db[j] = sum_i dZ[i][j]
__global__ void __launch_bounds__(256)
k_colsum(int M, int N, const float *__restrict__ dZ, float *__restrict__ db)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= N) return;
    float s = 0.f;
    for (int i = 0; i < M; ++i) s += dZ[(int64_t)i * N + j];
    db[j] = s;
}

__device__ __forceinline__ uint64_t mix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// He-uniform initialisation, U(-sqrt(6/fan_in), sqrt(6/fan_in)).
__global__ void __launch_bounds__(256)
k_init(int64_t len, int fan_in, uint64_t seed, float *__restrict__ w, uint16_t *__restrict__ wb)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= len) return;
    const double u = (double)(mix64(seed ^ mix64((uint64_t)t)) >> 11) * (1.0 / 9007199254740992.0);
    const float v = (float)((2.0 * u - 1.0) * sqrt(6.0 / fan_in));
    w[t] = v;
    wb[t] = f2bf(v);
}

// Adam (bias-corrected), FP32 state; refreshes the BF16 copy.
__global__ void __launch_bounds__(256)
k_adam(int64_t len, float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m1,
       float *__restrict__ m2, uint16_t *__restrict__ pb, float lr, float b1, float b2, float eps, float c1,
       float c2)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= len) return;
    const float gt = g[t];
    const float a = b1 * m1[t] + (1.f - b1) * gt;
    const float v = b2 * m2[t] + (1.f - b2) * gt * gt;
    m1[t] = a;
    m2[t] = v;
    const float upd = lr * (a / c1) / (sqrtf(v / c2) + eps);
    const float np = p[t] - upd;
    p[t] = np;
    if (pb) pb[t] = f2bf(np);
}

inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

struct uv_mlp {
    int L = 0;                       // layers
    std::vector<int> d;              // widths d[0..L]
    int max_batch = 0;
    hipStream_t stream = nullptr;
    std::vector<void *> allocs;
    std::vector<float *> W, b, gW, gb, mW, vW, mb, vb;
    std::vector<uint16_t *> Wb;      // BF16 weight copies
    std::vector<uint16_t *> act;     // BF16 activations a_0 (input) .. a_{L-1}
    std::vector<float *> dzf;        // FP32 gradient w.r.t. pre-activations
    std::vector<uint16_t *> dzb;     // BF16 copies
    float *y = nullptr;              // FP32 output (max_batch x d[L])
    float *loss = nullptr;
    int64_t step = 0;
};

namespace {

template <typename T>
T *malloc_d(uv_mlp *h, size_t count)
{
    void *p = nullptr;
    if (uv::dev_malloc(&p, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return nullptr;
    h->allocs.push_back(p);
    return (T *)p;
}

// Load mode of an operand whose element (r, k) is P[r * rs + k * ks]:
// 16-byte loads need a unit stride along them, the other stride a multiple
// of eight elements and a 16-byte-aligned base.
int load_mode(const uint16_t *P, int64_t rs, int64_t ks)
{
    const bool aligned = ((uintptr_t)P & 15) == 0;
    if (aligned && ks == 1 && rs % 8 == 0) return LD_KC;
    if (aligned && rs == 1 && ks % 8 == 0) return LD_MC;
    return LD_EL;
}

template <int EPI, int TM, int TN, int AM>
void gemm_launch_b(int bmode, unsigned grid, hipStream_t st, int M, int N, int K, const uint16_t *A, int64_t a_rs,
                   int64_t a_cs, const uint16_t *B, int64_t b_rs, int64_t b_cs, float *Cf, uint16_t *Cb, int64_t ldc,
                   const float *bias, const uint16_t *act)
{
#define UV_GEMM_ARGS M, N, K, A, a_rs, a_cs, B, b_rs, b_cs, Cf, Cb, ldc, bias, act
    if (bmode == LD_KC) k_mfma_gemm<EPI, TM, TN, AM, LD_KC><<<grid, 256, 0, st>>>(UV_GEMM_ARGS);
    else if (bmode == LD_MC) k_mfma_gemm<EPI, TM, TN, AM, LD_MC><<<grid, 256, 0, st>>>(UV_GEMM_ARGS);
    else k_mfma_gemm<EPI, TM, TN, AM, LD_EL><<<grid, 256, 0, st>>>(UV_GEMM_ARGS);
}

template <int EPI, int TM, int TN>
void gemm_launch(hipStream_t st, int M, int N, int K, const uint16_t *A, int64_t a_rs, int64_t a_cs,
                 const uint16_t *B, int64_t b_rs, int64_t b_cs, float *Cf, uint16_t *Cb, int64_t ldc,
                 const float *bias, const uint16_t *act)
{
    const unsigned grid = (unsigned)(((M + 32 * TM - 1) / (32 * TM)) * ((N + 32 * TN - 1) / (32 * TN)));
    const int am = load_mode(A, a_rs, a_cs), bm = load_mode(B, b_cs, b_rs);
    if (am == LD_KC) gemm_launch_b<EPI, TM, TN, LD_KC>(bm, grid, st, UV_GEMM_ARGS);
    else if (am == LD_MC) gemm_launch_b<EPI, TM, TN, LD_MC>(bm, grid, st, UV_GEMM_ARGS);
    else gemm_launch_b<EPI, TM, TN, LD_EL>(bm, grid, st, UV_GEMM_ARGS);
#undef UV_GEMM_ARGS
}

// 128 x 128 blocks when they still give every CU a block, else 64 x 64.
template <int EPI>
int gemm_any(hipStream_t st, int M, int N, int K, const uint16_t *A, int64_t a_rs, int64_t a_cs,
             const uint16_t *B, int64_t b_rs, int64_t b_cs, float *Cf, uint16_t *Cb, int64_t ldc,
             const float *bias, const uint16_t *act)
{
    const int64_t big = (int64_t)((M + 127) / 128) * ((N + 127) / 128);
    if (big >= 256) gemm_launch<EPI, 4, 4>(st, M, N, K, A, a_rs, a_cs, B, b_rs, b_cs, Cf, Cb, ldc, bias, act);
    else gemm_launch<EPI, 2, 2>(st, M, N, K, A, a_rs, a_cs, B, b_rs, b_cs, Cf, Cb, ldc, bias, act);
    return hipGetLastError() == hipSuccess ? UV_OK : UV_EHIP;
}

template <int EPI>
int mm(uv_mlp *h, int M, int N, int K, const uint16_t *A, int64_t a_rs, int64_t a_cs, const uint16_t *B,
       int64_t b_rs, int64_t b_cs, float *Cf, uint16_t *Cb, int64_t ldc, const float *bias, const uint16_t *act)
{
    return gemm_any<EPI>(h->stream, M, N, K, A, a_rs, a_cs, B, b_rs, b_cs, Cf, Cb, ldc, bias, act);
}

int forward(uv_mlp *h, int batch, const float *x)
{
    k_to_bf16<<<nb256((int64_t)batch * h->d[0]), 256, 0, h->stream>>>((int64_t)batch * h->d[0], x, h->act[0]);
    int rc = UV_OK;
    for (int l = 0; l < h->L && rc == UV_OK; ++l) {
        const int K = h->d[l], N = h->d[l + 1];
        if (l < h->L - 1)
            rc = mm<EPI_BIAS_RELU>(h, batch, N, K, h->act[l], K, 1, h->Wb[l], N, 1, nullptr, h->act[l + 1], N,
                                   h->b[l], nullptr);
        else
            rc = mm<EPI_BIAS_F32>(h, batch, N, K, h->act[l], K, 1, h->Wb[l], N, 1, h->y, nullptr, N, h->b[l],
                                  nullptr);
    }
    return rc;
}

int backward(uv_mlp *h, int batch, const float *t)
{
    const int L = h->L;
    const int64_t out_len = (int64_t)batch * h->d[L];
    k_mse<<<1, 256, 0, h->stream>>>(out_len, h->y, t, h->dzf[L - 1], h->dzb[L - 1], h->loss);
    int rc = UV_OK;
    for (int l = L - 1; l >= 0 && rc == UV_OK; --l) {
        const int K = h->d[l], N = h->d[l + 1];
        // dW_l = a_l' dz_l  (K x N), db_l = column sums of dz_l
        rc = mm<EPI_F32>(h, K, N, batch, h->act[l], 1, K, h->dzb[l], N, 1, h->gW[l], nullptr, N, nullptr, nullptr);
        k_colsum<<<nb256(N), 256, 0, h->stream>>>(batch, N, h->dzf[l], h->gb[l]);
        if (l > 0 && rc == UV_OK)  // dz_{l-1} = (dz_l W_l') * [a_l > 0]
            rc = mm<EPI_MASK>(h, batch, K, N, h->dzb[l], N, 1, h->Wb[l], 1, N, h->dzf[l - 1], h->dzb[l - 1], K,
                              nullptr, h->act[l]);
    }
    return rc == UV_OK && hipGetLastError() == hipSuccess ? UV_OK : UV_EHIP;
}

bool dims_ok(int batch, const uv_mlp *h) { return batch >= 16 && batch % 16 == 0 && batch <= h->max_batch; }

}  // namespace

extern "C" {

void mlp_destroy(uv_mlp *h)
{
    if (!h) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (void *p : h->allocs) (void)hipFree(p);
    delete h;
}

int mlp_create(int32_t nlayers, const int32_t *dims, int32_t max_batch, uint64_t seed, void *stream, uv_mlp **out)
{
    if (!out) return UV_EINVAL;
    *out = nullptr;
    if (nlayers < 1 || nlayers > 16 || !dims || max_batch < 16 || max_batch % 16) return UV_EINVAL;
    for (int l = 0; l <= nlayers; ++l)
        if (dims[l] < 16 || dims[l] % 16 || dims[l] > 65536) return UV_EINVAL;
    uv_mlp *h = new (std::nothrow) uv_mlp();
    if (!h) return UV_ENOMEM;
    h->L = nlayers;
    h->d.assign(dims, dims + nlayers + 1);
    h->max_batch = max_batch;
    h->stream = (hipStream_t)stream;
    const int L = nlayers;
    h->W.resize(L); h->b.resize(L); h->gW.resize(L); h->gb.resize(L); h->mW.resize(L); h->vW.resize(L);
    h->mb.resize(L); h->vb.resize(L); h->Wb.resize(L); h->act.resize(L); h->dzf.resize(L); h->dzb.resize(L);
    bool ok = true;
    for (int l = 0; l < L; ++l) {
        const size_t nw = (size_t)h->d[l] * h->d[l + 1], nbias = h->d[l + 1];
        ok &= (h->W[l] = malloc_d<float>(h, nw)) != nullptr;
        ok &= (h->gW[l] = malloc_d<float>(h, nw)) != nullptr;
        ok &= (h->mW[l] = malloc_d<float>(h, nw)) != nullptr;
        ok &= (h->vW[l] = malloc_d<float>(h, nw)) != nullptr;
        ok &= (h->Wb[l] = malloc_d<uint16_t>(h, nw)) != nullptr;
        ok &= (h->b[l] = malloc_d<float>(h, nbias)) != nullptr;
        ok &= (h->gb[l] = malloc_d<float>(h, nbias)) != nullptr;
        ok &= (h->mb[l] = malloc_d<float>(h, nbias)) != nullptr;
        ok &= (h->vb[l] = malloc_d<float>(h, nbias)) != nullptr;
        ok &= (h->act[l] = malloc_d<uint16_t>(h, (size_t)max_batch * h->d[l])) != nullptr;
        ok &= (h->dzf[l] = malloc_d<float>(h, (size_t)max_batch * h->d[l + 1])) != nullptr;
        ok &= (h->dzb[l] = malloc_d<uint16_t>(h, (size_t)max_batch * h->d[l + 1])) != nullptr;
    }
    ok &= (h->y = malloc_d<float>(h, (size_t)max_batch * h->d[L])) != nullptr;
    ok &= (h->loss = malloc_d<float>(h, 1)) != nullptr;
    if (!ok) {
        mlp_destroy(h);
        return UV_ENOMEM;
    }
    for (int l = 0; l < L && ok; ++l) {
        const int64_t nw = (int64_t)h->d[l] * h->d[l + 1];
        k_init<<<nb256(nw), 256, 0, h->stream>>>(nw, h->d[l], seed + 0x1000003ull * (l + 1), h->W[l], h->Wb[l]);
        ok &= hipMemsetAsync(h->b[l], 0, 4 * (size_t)h->d[l + 1], h->stream) == hipSuccess;
        ok &= hipMemsetAsync(h->mW[l], 0, 4 * nw, h->stream) == hipSuccess;
        ok &= hipMemsetAsync(h->vW[l], 0, 4 * nw, h->stream) == hipSuccess;
        ok &= hipMemsetAsync(h->mb[l], 0, 4 * (size_t)h->d[l + 1], h->stream) == hipSuccess;
        ok &= hipMemsetAsync(h->vb[l], 0, 4 * (size_t)h->d[l + 1], h->stream) == hipSuccess;
    }
    ok &= hipGetLastError() == hipSuccess && hipStreamSynchronize(h->stream) == hipSuccess;
    if (!ok) {
        mlp_destroy(h);
        return UV_EHIP;
    }
    *out = h;
    return UV_OK;
}

int mlp_get_params(uv_mlp *h, float *w, float *b)
{
    if (!h) return UV_EINVAL;
    size_t ow = 0, ob = 0;
    for (int l = 0; l < h->L; ++l) {
        const size_t nw = (size_t)h->d[l] * h->d[l + 1], nbias = h->d[l + 1];
        if (w && hipMemcpy(w + ow, h->W[l], 4 * nw, hipMemcpyDeviceToHost) != hipSuccess) return UV_EHIP;
        if (b && hipMemcpy(b + ob, h->b[l], 4 * nbias, hipMemcpyDeviceToHost) != hipSuccess) return UV_EHIP;
        ow += nw;
        ob += nbias;
    }
    return UV_OK;
}

int mlp_set_params(uv_mlp *h, const float *w, const float *b)
{
    if (!h) return UV_EINVAL;
    size_t ow = 0, ob = 0;
    for (int l = 0; l < h->L; ++l) {
        const size_t nw = (size_t)h->d[l] * h->d[l + 1], nbias = h->d[l + 1];
        if (w) {
            if (hipMemcpy(h->W[l], w + ow, 4 * nw, hipMemcpyHostToDevice) != hipSuccess) return UV_EHIP;
            k_to_bf16<<<nb256(nw), 256, 0, h->stream>>>((int64_t)nw, h->W[l], h->Wb[l]);
        }
        if (b && hipMemcpy(h->b[l], b + ob, 4 * nbias, hipMemcpyHostToDevice) != hipSuccess) return UV_EHIP;
        ow += nw;
        ob += nbias;
    }
    return hipStreamSynchronize(h->stream) == hipSuccess ? UV_OK : UV_EHIP;
}

int mlp_forward(uv_mlp *h, int32_t batch, const float *x_dev, float *y_dev)
{
    if (!h || !x_dev || !y_dev || !dims_ok(batch, h)) return UV_EINVAL;
    int rc = forward(h, batch, x_dev);
    if (rc != UV_OK) return rc;
    if (hipMemcpyAsync(y_dev, h->y, 4 * (size_t)batch * h->d[h->L], hipMemcpyDeviceToDevice, h->stream) != hipSuccess)
        return UV_EHIP;
    return hipStreamSynchronize(h->stream) == hipSuccess ? UV_OK : UV_EHIP;
}

int mlp_gradients(uv_mlp *h, int32_t batch, const float *x_dev, const float *t_dev, float *gw, float *gb,
                  float *loss)
{
    if (!h || !x_dev || !t_dev || !dims_ok(batch, h)) return UV_EINVAL;
    int rc = forward(h, batch, x_dev);
    if (rc == UV_OK) rc = backward(h, batch, t_dev);
    if (rc != UV_OK) return rc;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return UV_EHIP;
    size_t ow = 0, ob = 0;
    for (int l = 0; l < h->L; ++l) {
        const size_t nw = (size_t)h->d[l] * h->d[l + 1], nbias = h->d[l + 1];
        if (gw && hipMemcpy(gw + ow, h->gW[l], 4 * nw, hipMemcpyDeviceToHost) != hipSuccess) return UV_EHIP;
        if (gb && hipMemcpy(gb + ob, h->gb[l], 4 * nbias, hipMemcpyDeviceToHost) != hipSuccess) return UV_EHIP;
        ow += nw;
        ob += nbias;
    }
    if (loss && hipMemcpy(loss, h->loss, 4, hipMemcpyDeviceToHost) != hipSuccess) return UV_EHIP;
    return UV_OK;
}

int mlp_train_step(uv_mlp *h, int32_t batch, const float *x_dev, const float *t_dev, float lr, float *loss)
{
    if (!h || !x_dev || !t_dev || !dims_ok(batch, h) || !(lr > 0.f)) return UV_EINVAL;
    int rc = forward(h, batch, x_dev);
    if (rc == UV_OK) rc = backward(h, batch, t_dev);
    if (rc != UV_OK) return rc;
    h->step += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - (float)std::pow((double)b1, (double)h->step);
    const float c2 = 1.f - (float)std::pow((double)b2, (double)h->step);
    for (int l = 0; l < h->L; ++l) {
        const int64_t nw = (int64_t)h->d[l] * h->d[l + 1], nbias = h->d[l + 1];
        k_adam<<<nb256(nw), 256, 0, h->stream>>>(nw, h->W[l], h->gW[l], h->mW[l], h->vW[l], h->Wb[l], lr, b1, b2, eps,
                                                 c1, c2);
        k_adam<<<nb256(nbias), 256, 0, h->stream>>>(nbias, h->b[l], h->gb[l], h->mb[l], h->vb[l], nullptr, lr, b1, b2,
                                                    eps, c1, c2);
    }
    if (hipGetLastError() != hipSuccess) return UV_EHIP;
    if (loss) {
        if (hipMemcpyAsync(loss, h->loss, 4, hipMemcpyDeviceToHost, h->stream) != hipSuccess) return UV_EHIP;
        if (hipStreamSynchronize(h->stream) != hipSuccess) return UV_EHIP;
    }
    return UV_OK;
}

int mlp_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t *A, int64_t a_rs, int64_t a_cs, const uint16_t *B,
                  int64_t b_rs, int64_t b_cs, float *C, int64_t ldc, void *stream)
{
    if (M < 16 || N < 16 || K < 16 || M % 16 || N % 16 || K % 16 || !A || !B || !C) return UV_EINVAL;
    if (gemm_any<EPI_F32>((hipStream_t)stream, M, N, K, A, a_rs, a_cs, B, b_rs, b_cs, C, nullptr, ldc, nullptr,
                          nullptr) != UV_OK)
        return UV_EHIP;
    return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? UV_OK : UV_EHIP;
}

}  // extern "C"
