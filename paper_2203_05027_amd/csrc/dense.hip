// dense.hip -- dense linear algebra for the learned warm start: an FP32
// GEMM, a randomized principal-component fit built on it, and the small
// (l x l, l <= 1024) host-side factorizations the fit needs.
//
// PCA of the solution matrix Y (N samples x D features, D large):
//   mean, center Y in place, Z = Y Omega (Omega Gaussian, D x l),
//   q rounds of Z <- orth(Y (orth(Y' Z))),  Q = orth(Z),  B = Q' Y (l x D),
//   B B' = U S^2 U' (Jacobi),  basis = top-k rows of S^{-1} U' B,
// i.e. the randomized range finder with power iterations of Halko,
// Martinsson and Tropp; orth() is Cholesky QR applied twice.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/uvadmm.h"
#include "common.hpp"

namespace {

constexpr int TM = 64, TN = 64, TK = 16;

// C = alpha * A B + beta * C, A(i,k) = A[i*a_rs + k*a_cs], B(k,j) = B[k*b_rs + j*b_cs],
// C row-major with leading dimension ldc.  64x64 tile per 256-thread
// workgroup, 4x4 outputs per thread, LDS-staged 16-deep slices.
__global__ void __launch_bounds__(256)
k_gemm_f32(int M, int N, int K, const float *__restrict__ A, int64_t a_rs, int64_t a_cs,
           const float *__restrict__ B, int64_t b_rs, int64_t b_cs, float *__restrict__ C, int64_t ldc,
           float alpha, float beta)
{
    __shared__ float As[TK][TM + 4];
    __shared__ float Bs[TK][TN + 4];
    const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
    const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TN;
    float acc[4][4] = {};
    for (int k0 = 0; k0 < K; k0 += TK) {
        for (int t = threadIdx.x; t < TM * TK; t += 256) {
            const int r = t / TK, kk = t % TK;
            const int i = i0 + r, k = k0 + kk;
            As[kk][r] = (i < M && k < K) ? A[(int64_t)i * a_rs + (int64_t)k * a_cs] : 0.f;
        }
        for (int t = threadIdx.x; t < TN * TK; t += 256) {
            const int cc = t % TN, kk = t / TN;
            const int j = j0 + cc, k = k0 + kk;
            Bs[kk][cc] = (j < N && k < K) ? B[(int64_t)k * b_rs + (int64_t)j * b_cs] : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            float a[4], b[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) a[r] = As[kk][ty * 4 + r];
#pragma unroll
            for (int s = 0; s < 4; ++s) b[s] = Bs[kk][tx * 4 + s];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int s = 0; s < 4; ++s) acc[r][s] += a[r] * b[s];
        }
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = i0 + ty * 4 + r;
        if (i >= M) continue;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int j = j0 + tx * 4 + s;
            if (j >= N) continue;
            float *cptr = C + (int64_t)i * ldc + j;
            *cptr = alpha * acc[r][s] + (beta != 0.f ? beta * *cptr : 0.f);
        }
    }
}

// Column means of Y (N x D, leading dimension ld) and Y -= mean.
__global__ void __launch_bounds__(256)
k_center(int64_t N, int64_t D, float *__restrict__ Y, int64_t ld, float *__restrict__ mean)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= D) return;
    double s = 0.0;
    for (int64_t i = 0; i < N; ++i) s += Y[i * ld + j];
    const float mu = (float)(s / (double)N);
    mean[j] = mu;
    for (int64_t i = 0; i < N; ++i) Y[i * ld + j] -= mu;
}

// Gaussian matrix from a counter-based generator: splitmix64 of
// (seed, index) gives two uniforms, Box-Muller turns them into N(0,1).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__global__ void __launch_bounds__(256) k_gauss(int64_t len, uint64_t seed, float *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= len) return;
    const uint64_t r = splitmix64(seed ^ splitmix64((uint64_t)t));
    const double u1 = ((r >> 11) + 1.0) * (1.0 / 9007199254740993.0);  // (0, 1]
    const double u2 = (double)(splitmix64(r) >> 11) * (1.0 / 9007199254740992.0);
    out[t] = (float)(sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
}

// y_i += v (row-broadcast add): Y (N x D, ld).
__global__ void __launch_bounds__(256)
k_add_row(int64_t N, int64_t D, float *__restrict__ Y, int64_t ld, const float *__restrict__ v)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= N * D) return;
    const int64_t i = t / D, j = t % D;
    Y[i * ld + j] += v[j];
}

__global__ void __launch_bounds__(256)
k_mul_row(int64_t N, int64_t D, float *__restrict__ Y, int64_t ld, const float *__restrict__ v)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= N * D) return;
    const int64_t i = t / D, j = t % D;
    Y[i * ld + j] *= v[j];
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

int gemm(hipStream_t st, int M, int N, int K, const float *A, int64_t a_rs, int64_t a_cs, const float *B,
         int64_t b_rs, int64_t b_cs, float *C, int64_t ldc, float alpha, float beta)
{
    if (M <= 0 || N <= 0) return UV_OK;
    dim3 g(nblk(N, TN), nblk(M, TM));
    k_gemm_f32<<<g, 256, 0, st>>>(M, N, K, A, a_rs, a_cs, B, b_rs, b_cs, C, ldc, alpha, beta);
    return hipGetLastError() == hipSuccess ? UV_OK : UV_EHIP;
}

// ---- host-side small dense factorizations (l x l, row-major) ----

// Lower Cholesky G = L L'.  A non-positive pivot (rank loss) is replaced by
// a tiny positive one so the factor stays finite.
void chol_lower(std::vector<double> &G, int l)
{
    double scale = 0.0;
    for (int i = 0; i < l; ++i) scale = std::max(scale, G[(size_t)i * l + i]);
    const double floor_ = std::max(scale, 1e-300) * 1e-14;
    for (int j = 0; j < l; ++j) {
        double d = G[(size_t)j * l + j];
        for (int k = 0; k < j; ++k) d -= G[(size_t)j * l + k] * G[(size_t)j * l + k];
        d = std::sqrt(std::max(d, floor_));
        G[(size_t)j * l + j] = d;
        for (int i = j + 1; i < l; ++i) {
            double s = G[(size_t)i * l + j];
            for (int k = 0; k < j; ++k) s -= G[(size_t)i * l + k] * G[(size_t)j * l + k];
            G[(size_t)i * l + j] = s / d;
        }
        for (int k = j + 1; k < l; ++k) G[(size_t)j * l + k] = 0.0;
    }
}

// Inverse of a lower-triangular matrix (forward substitution per column).
std::vector<double> inv_lower(const std::vector<double> &L, int l)
{
    std::vector<double> X((size_t)l * l, 0.0);
    for (int c = 0; c < l; ++c) {
        for (int i = c; i < l; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) s -= L[(size_t)i * l + k] * X[(size_t)k * l + c];
            X[(size_t)i * l + c] = s / L[(size_t)i * l + i];
        }
    }
    return X;
}

}  // namespace

extern "C" {

// Symmetric eigen-decomposition by cyclic Jacobi rotations: S (l x l,
// row-major, destroyed) -> eigenvalues w (descending) and eigenvectors as
// the columns of V (row-major l x l).
int uvla_sym_eig(int32_t l, double *S, double *w, double *V)
{
    if (l < 1 || !S || !w || !V) return UV_EINVAL;
    for (int i = 0; i < l; ++i)
        for (int j = 0; j < l; ++j) V[(size_t)i * l + j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < l; ++i)
            for (int j = 0; j < l; ++j) {
                const double v = S[(size_t)i * l + j] * S[(size_t)i * l + j];
                tot += v;
                if (i != j) off += v;
            }
        if (off <= 1e-30 * std::max(tot, 1e-300)) break;
        for (int p = 0; p < l - 1; ++p) {
            for (int q = p + 1; q < l; ++q) {
                const double apq = S[(size_t)p * l + q];
                if (std::fabs(apq) < 1e-300) continue;
                const double app = S[(size_t)p * l + p], aqq = S[(size_t)q * l + q];
                const double theta = (aqq - app) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < l; ++k) {  // rows p, q
                    const double a = S[(size_t)p * l + k], b = S[(size_t)q * l + k];
                    S[(size_t)p * l + k] = cs * a - sn * b;
                    S[(size_t)q * l + k] = sn * a + cs * b;
                }
                for (int k = 0; k < l; ++k) {  // columns p, q
                    const double a = S[(size_t)k * l + p], b = S[(size_t)k * l + q];
                    S[(size_t)k * l + p] = cs * a - sn * b;
                    S[(size_t)k * l + q] = sn * a + cs * b;
                }
                for (int k = 0; k < l; ++k) {
                    const double a = V[(size_t)k * l + p], b = V[(size_t)k * l + q];
                    V[(size_t)k * l + p] = cs * a - sn * b;
                    V[(size_t)k * l + q] = sn * a + cs * b;
                }
            }
        }
    }
    // sort descending
    std::vector<int> idx(l);
    for (int i = 0; i < l; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return S[(size_t)a * l + a] > S[(size_t)b * l + b]; });
    std::vector<double> Vs((size_t)l * l);
    for (int c = 0; c < l; ++c) {
        w[c] = S[(size_t)idx[c] * l + idx[c]];
        for (int r = 0; r < l; ++r) Vs[(size_t)r * l + c] = V[(size_t)r * l + idx[c]];
    }
    std::memcpy(V, Vs.data(), sizeof(double) * l * l);
    return UV_OK;
}

int gemm_f32(int32_t M, int32_t N, int32_t K, const float *A, int64_t a_rs, int64_t a_cs, const float *B,
             int64_t b_rs, int64_t b_cs, float *C, int64_t ldc, float alpha, float beta, void *stream)
{
    if (M < 0 || N < 0 || K < 0 || !A || !B || !C) return UV_EINVAL;
    int rc = gemm((hipStream_t)stream, M, N, K, A, a_rs, a_cs, B, b_rs, b_cs, C, ldc, alpha, beta);
    if (rc != UV_OK) return rc;
    return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? UV_OK : UV_EHIP;
}

int add_row_vector(int64_t N, int64_t D, float *Y, int64_t ld, const float *v, void *stream)
{
    if (!Y || !v || N < 0 || D < 0) return UV_EINVAL;
    if (N * D == 0) return UV_OK;
    k_add_row<<<nblk(N * D, 256), 256, 0, (hipStream_t)stream>>>(N, D, Y, ld, v);
    if (hipGetLastError() != hipSuccess) return UV_EHIP;
    return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? UV_OK : UV_EHIP;
}

int mul_row_vector(int64_t N, int64_t D, float *Y, int64_t ld, const float *v, void *stream)
{
    if (!Y || !v || N < 0 || D < 0 || (N > 0 && ld < D)) return UV_EINVAL;
    if (N * D == 0) return UV_OK;
    k_mul_row<<<nblk(N * D, 256), 256, 0, (hipStream_t)stream>>>(N, D, Y, ld, v);
    if (hipGetLastError() != hipSuccess) return UV_EHIP;
    return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? UV_OK : UV_EHIP;
}

int pca_fit(float *Y, int64_t N, int64_t D, int64_t ld, int32_t k, int32_t oversample, int32_t power_iters,
            uint64_t seed, float *mean, float *basis, float *sv, void *stream)
{
    if (!Y || !mean || !basis || !sv || N < 1 || D < 1 || ld < D || k < 1 || oversample < 0 || power_iters < 0)
        return UV_EINVAL;
    const int l = (int)std::min<int64_t>(std::min<int64_t>(k + oversample, N), D);
    if (k > l || l > 1024 || N >= ((int64_t)1 << 31) || D >= ((int64_t)1 << 31)) return UV_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    float *Om = nullptr, *Z = nullptr, *W = nullptr, *G = nullptr, *R = nullptr, *Bm = nullptr, *Tm = nullptr;
    auto cleanup = [&]() {
        for (float *p : {Om, Z, W, G, R, Bm, Tm})
            if (p) (void)hipFree(p);
    };
    if (uv::dev_malloc(&Om, sizeof(float) * D * l) != hipSuccess || uv::dev_malloc(&Z, sizeof(float) * N * l) != hipSuccess ||
        uv::dev_malloc(&W, sizeof(float) * D * l) != hipSuccess || uv::dev_malloc(&G, sizeof(float) * l * l) != hipSuccess ||
        uv::dev_malloc(&R, sizeof(float) * l * l) != hipSuccess || uv::dev_malloc(&Bm, sizeof(float) * l * D) != hipSuccess ||
        uv::dev_malloc(&Tm, sizeof(float) * std::max(N, D) * l) != hipSuccess) {
        cleanup();
        return UV_ENOMEM;
    }
    int rc = UV_OK;
    std::vector<float> gh((size_t)l * l), rh((size_t)l * l);
    std::vector<double> gd((size_t)l * l);
    // orthonormalize the columns of X (rows x l, row-major): X <- X R^{-1}
    // with G = X'X = L L', R = L'  (Cholesky QR; applied twice)
    auto orth = [&](float *X, int64_t rows) -> int {
        for (int pass = 0; pass < 2; ++pass) {
            int r = gemm(st, l, l, (int)rows, X, 1, l, X, l, 1, G, l, 1.f, 0.f);
            if (r != UV_OK) return r;
            if (hipMemcpyAsync(gh.data(), G, sizeof(float) * l * l, hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return UV_EHIP;
            for (size_t t = 0; t < gd.size(); ++t) gd[t] = gh[t];
            chol_lower(gd, l);
            std::vector<double> Li = inv_lower(gd, l);
            for (int i = 0; i < l; ++i)  // R^{-1} = (L^{-1})'
                for (int j = 0; j < l; ++j) rh[(size_t)i * l + j] = (float)Li[(size_t)j * l + i];
            if (hipMemcpyAsync(R, rh.data(), sizeof(float) * l * l, hipMemcpyHostToDevice, st) != hipSuccess)
                return UV_EHIP;
            // X <- X R^{-1} through the scratch Tm (max(N, D) x l)
            r = gemm(st, (int)rows, l, l, X, l, 1, R, l, 1, Tm, l, 1.f, 0.f);
            if (r != UV_OK) return r;
            if (hipMemcpyAsync(X, Tm, sizeof(float) * rows * l, hipMemcpyDeviceToDevice, st) != hipSuccess)
                return UV_EHIP;
        }
        return UV_OK;
    };
    do {
        k_center<<<nblk(D, 256), 256, 0, st>>>(N, D, Y, ld, mean);
        k_gauss<<<nblk(D * l, 256), 256, 0, st>>>(D * l, seed, Om);
        if (hipGetLastError() != hipSuccess) { rc = UV_EHIP; break; }
        if ((rc = gemm(st, (int)N, l, (int)D, Y, ld, 1, Om, l, 1, Z, l, 1.f, 0.f)) != UV_OK) break;   // Z = Y Om
        for (int q = 0; q < power_iters && rc == UV_OK; ++q) {
            if ((rc = orth(Z, N)) != UV_OK) break;
            if ((rc = gemm(st, (int)D, l, (int)N, Y, 1, ld, Z, l, 1, W, l, 1.f, 0.f)) != UV_OK) break;  // W = Y'Z
            if ((rc = orth(W, D)) != UV_OK) break;
            rc = gemm(st, (int)N, l, (int)D, Y, ld, 1, W, l, 1, Z, l, 1.f, 0.f);                          // Z = Y W
        }
        if (rc != UV_OK) break;
        if ((rc = orth(Z, N)) != UV_OK) break;
        if ((rc = gemm(st, l, (int)D, (int)N, Z, 1, l, Y, ld, 1, Bm, D, 1.f, 0.f)) != UV_OK) break;   // Bm = Z'Y
        if ((rc = gemm(st, l, l, (int)D, Bm, D, 1, Bm, 1, D, G, l, 1.f, 0.f)) != UV_OK) break;        // G = Bm Bm'
        if (hipMemcpyAsync(gh.data(), G, sizeof(float) * l * l, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) { rc = UV_EHIP; break; }
        std::vector<double> S((size_t)l * l), w(l), V((size_t)l * l);
        for (size_t t = 0; t < S.size(); ++t) S[t] = gh[t];
        uvla_sym_eig(l, S.data(), w.data(), V.data());
        // basis row c = (V[:, c]' Bm) / sigma_c for the top k
        std::vector<float> P((size_t)k * l);
        for (int c = 0; c < k; ++c) {
            const double sg = std::sqrt(std::max(w[c], 0.0));
            sv[c] = (float)sg;
            const double inv = sg > 0 ? 1.0 / sg : 0.0;
            for (int r = 0; r < l; ++r) P[(size_t)c * l + r] = (float)(V[(size_t)r * l + c] * inv);
        }
        if (hipMemcpyAsync(R, P.data(), sizeof(float) * k * l, hipMemcpyHostToDevice, st) != hipSuccess) { rc = UV_EHIP; break; }
        rc = gemm(st, k, (int)D, l, R, l, 1, Bm, D, 1, basis, D, 1.f, 0.f);
        if (rc == UV_OK && hipStreamSynchronize(st) != hipSuccess) rc = UV_EHIP;
    } while (false);
    if (hipStreamSynchronize(st) != hipSuccess && rc == UV_OK) rc = UV_EHIP;
    cleanup();
    return rc;
}

}  // extern "C"
