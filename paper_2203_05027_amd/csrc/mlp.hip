// mlp.hip -- the learned warm start's network: a multilayer perceptron
// (ReLU hidden layers, linear output) whose GEMMs run on the BF16 matrix
// cores (v_mfma_f32_16x16x16_bf16, FP32 accumulation), trained on a mean
// squared error with Adam.  Master weights, biases, gradients and the Adam
// moments are FP32; each GEMM reads BF16 copies of its operands.
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

typedef short v4s __attribute__((ext_vector_type(4)));
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

// C (M x N) = A (M x K) B (K x N) on BF16 operands with FP32 accumulation;
// A(i,k) = A[i*a_rs + k*a_cs], B(k,j) = B[k*b_rs + j*b_cs]; M, N, K
// multiples of 16.  Each wavefront owns one 16 x 16 tile of C: lane l feeds
// A[l%16][4(l/16)..+3] and B[4(l/16)..+3][l%16] and receives
// C[4(l/16)..+3][l%16] (the 16x16x16 BF16 MFMA operand layout).
template <int EPI>
__global__ void __launch_bounds__(256)
k_mfma_gemm(int M, int N, int K, const uint16_t *__restrict__ A, int64_t a_rs, int64_t a_cs,
            const uint16_t *__restrict__ B, int64_t b_rs, int64_t b_cs, float *__restrict__ Cf,
            uint16_t *__restrict__ Cb, int64_t ldc, const float *__restrict__ bias,
            const uint16_t *__restrict__ act)
{
    const int wave = blockIdx.x * 4 + threadIdx.x / 64, lane = threadIdx.x % 64;
    const int tiles_n = N / 16;
    const int ti = wave / tiles_n, tj = wave % tiles_n;
    if (ti * 16 >= M) return;
    const int r = lane % 16, kq = lane / 16;
    const int64_t arow = (int64_t)(ti * 16 + r) * a_rs, bcol = (int64_t)(tj * 16 + r) * b_cs;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        v4s a, b;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t k = k0 + kq * 4 + e;
            a[e] = (short)A[arow + k * a_cs];
            b[e] = (short)B[k * b_rs + bcol];
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    const int col = tj * 16 + r;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = ti * 16 + kq * 4 + e;
        const int64_t o = (int64_t)row * ldc + col;
        float v = acc[e];
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

template <int EPI>
int mm(uv_mlp *h, int M, int N, int K, const uint16_t *A, int64_t a_rs, int64_t a_cs, const uint16_t *B,
       int64_t b_rs, int64_t b_cs, float *Cf, uint16_t *Cb, int64_t ldc, const float *bias, const uint16_t *act)
{
    const int64_t tiles = (int64_t)(M / 16) * (N / 16);
    k_mfma_gemm<EPI><<<(unsigned)((tiles + 3) / 4), 256, 0, h->stream>>>(M, N, K, A, a_rs, a_cs, B, b_rs, b_cs, Cf,
                                                                        Cb, ldc, bias, act);
    return hipGetLastError() == hipSuccess ? UV_OK : UV_EHIP;
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
    const int64_t tiles = (int64_t)(M / 16) * (N / 16);
    k_mfma_gemm<EPI_F32><<<(unsigned)((tiles + 3) / 4), 256, 0, (hipStream_t)stream>>>(
        M, N, K, A, a_rs, a_cs, B, b_rs, b_cs, C, nullptr, ldc, nullptr, nullptr);
    if (hipGetLastError() != hipSuccess) return UV_EHIP;
    return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? UV_OK : UV_EHIP;
}

}  // extern "C"
