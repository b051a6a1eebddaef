"""Binding of the learned-warm-start kernels (dense GEMM, PCA fit, BF16 MLP).

Argument marshalling only: device buffers are torch tensors on the GPU (used
as plain memory), every computation runs in the library's kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np

from .solver import _check, lib

_bound = False


def _bind():
    global _bound
    if _bound:
        return lib()
    L = lib()
    P, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    L.gemm_f32.argtypes = [i32, i32, i32, P, i64, i64, P, i64, i64, P, i64, f32, f32, P]
    L.gemm_f32.restype = ctypes.c_int
    L.add_row_vector.argtypes = [i64, i64, P, i64, P, P]
    L.add_row_vector.restype = ctypes.c_int
    L.mul_row_vector.argtypes = [i64, i64, P, i64, P, P]
    L.mul_row_vector.restype = ctypes.c_int
    L.pca_fit.argtypes = [P, i64, i64, i64, i32, i32, i32, ctypes.c_uint64, P, P, P, P]
    L.pca_fit.restype = ctypes.c_int
    L.uvla_sym_eig.argtypes = [i32, P, P, P]
    L.uvla_sym_eig.restype = ctypes.c_int
    L.mlp_create.argtypes = [i32, P, i32, ctypes.c_uint64, P, ctypes.POINTER(P)]
    L.mlp_create.restype = ctypes.c_int
    L.mlp_get_params.argtypes = [P, P, P]
    L.mlp_get_params.restype = ctypes.c_int
    L.mlp_set_params.argtypes = [P, P, P]
    L.mlp_set_params.restype = ctypes.c_int
    L.mlp_forward.argtypes = [P, i32, P, P]
    L.mlp_forward.restype = ctypes.c_int
    L.mlp_gradients.argtypes = [P, i32, P, P, P, P, P]
    L.mlp_gradients.restype = ctypes.c_int
    L.mlp_train_step.argtypes = [P, i32, P, P, f32, P]
    L.mlp_train_step.restype = ctypes.c_int
    L.mlp_destroy.argtypes = [P]
    L.mlp_destroy.restype = None
    L.mlp_gemm_bf16.argtypes = [i32, i32, i32, P, i64, i64, P, i64, i64, P, i64, P]
    L.mlp_gemm_bf16.restype = ctypes.c_int
    _bound = True
    return L


def _dp(t) -> ctypes.c_void_p:
    """Device pointer of a torch tensor (contiguous, on the GPU)."""
    assert t.is_cuda and t.is_contiguous(), "expected a contiguous GPU tensor"
    return ctypes.c_void_p(t.data_ptr())


def sym_eig(S: np.ndarray):
    """Eigenvalues (descending) and eigenvectors (columns) of a symmetric
    matrix, by the library's host Jacobi routine."""
    L = _bind()
    S = np.array(S, dtype=np.float64, order="C", copy=True)
    l = S.shape[0]
    w = np.empty(l)
    V = np.empty((l, l))
    _check(L.uvla_sym_eig(l, S.ctypes.data_as(ctypes.c_void_p), w.ctypes.data_as(ctypes.c_void_p),
                          V.ctypes.data_as(ctypes.c_void_p)), "uvla_sym_eig")
    return w, V


def gemm(A, B, C=None, alpha=1.0, beta=0.0, transA=False, transB=False):
    """C = alpha op(A) op(B) + beta C for contiguous FP32 GPU tensors."""
    import torch
    L = _bind()
    M, K = (A.shape[1], A.shape[0]) if transA else A.shape
    K2, N = (B.shape[1], B.shape[0]) if transB else B.shape
    assert K == K2
    if C is None:
        C = torch.empty((M, N), dtype=torch.float32, device=A.device)
    a_rs, a_cs = (1, A.shape[1]) if transA else (A.shape[1], 1)
    b_rs, b_cs = (1, B.shape[1]) if transB else (B.shape[1], 1)
    _check(L.gemm_f32(M, N, K, _dp(A), a_rs, a_cs, _dp(B), b_rs, b_cs, _dp(C), C.shape[1],
                      float(alpha), float(beta), None), "gemm_f32")
    return C


def add_row_vector(Y, v):
    L = _bind()
    _check(L.add_row_vector(Y.shape[0], Y.shape[1], _dp(Y), Y.shape[1], _dp(v), None), "add_row_vector")


def mul_row_vector(Y, v):
    """Y[i, j] *= v[j] on every row (contiguous FP32 GPU tensors)."""
    L = _bind()
    _check(L.mul_row_vector(Y.shape[0], Y.shape[1], _dp(Y), Y.shape[1], _dp(v), None), "mul_row_vector")


def pca_fit(Y, k: int, oversample: int = 32, power_iters: int = 2, seed: int = 0):
    """Top-k principal components of the rows of the GPU tensor Y (N x D,
    centered in place).  Returns (mean (D,), basis (k, D), singular values)."""
    import torch
    L = _bind()
    N, D = Y.shape
    mean = torch.empty(D, dtype=torch.float32, device=Y.device)
    basis = torch.empty((k, D), dtype=torch.float32, device=Y.device)
    sv = np.empty(k, dtype=np.float32)
    _check(L.pca_fit(_dp(Y), N, D, Y.shape[1], int(k), int(oversample), int(power_iters), int(seed),
                     _dp(mean), _dp(basis), sv.ctypes.data_as(ctypes.c_void_p), None), "pca_fit")
    return mean, basis, sv


def gemm_bf16(A_bits, B_bits, transA=False, transB=False):
    """FP32 C = op(A) op(B) for BF16 operands given as int16 GPU tensors of
    raw bit patterns (the MLP's matrix-core kernel)."""
    import torch
    L = _bind()
    M, K = (A_bits.shape[1], A_bits.shape[0]) if transA else A_bits.shape
    K2, N = (B_bits.shape[1], B_bits.shape[0]) if transB else B_bits.shape
    assert K == K2
    C = torch.empty((M, N), dtype=torch.float32, device=A_bits.device)
    a_rs, a_cs = (1, A_bits.shape[1]) if transA else (A_bits.shape[1], 1)
    b_rs, b_cs = (1, B_bits.shape[1]) if transB else (B_bits.shape[1], 1)
    _check(L.mlp_gemm_bf16(M, N, K, _dp(A_bits), a_rs, a_cs, _dp(B_bits), b_rs, b_cs, _dp(C), N, None),
           "mlp_gemm_bf16")
    return C


class MLP:
    """dims[0] -> ... -> dims[-1], ReLU hidden layers, linear output, BF16
    MFMA GEMMs with FP32 accumulation, Adam."""

    def __init__(self, dims, max_batch=256, seed=0):
        L = _bind()
        self.dims = [int(d) for d in dims]
        self.max_batch = int(max_batch)
        arr = (ctypes.c_int32 * len(self.dims))(*self.dims)
        h = ctypes.c_void_p()
        _check(L.mlp_create(len(self.dims) - 1, arr, self.max_batch, int(seed), None, ctypes.byref(h)),
               "mlp_create")
        self._h = h
        self.nw = sum(a * b for a, b in zip(self.dims[:-1], self.dims[1:]))
        self.nb = sum(self.dims[1:])

    def close(self):
        if getattr(self, "_h", None):
            lib().mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        w = np.empty(self.nw, dtype=np.float32)
        b = np.empty(self.nb, dtype=np.float32)
        _check(lib().mlp_get_params(self._h, w.ctypes.data_as(ctypes.c_void_p),
                                    b.ctypes.data_as(ctypes.c_void_p)), "mlp_get_params")
        return w, b

    def set_params(self, w, b):
        w = np.ascontiguousarray(w, dtype=np.float32)
        b = np.ascontiguousarray(b, dtype=np.float32)
        _check(lib().mlp_set_params(self._h, w.ctypes.data_as(ctypes.c_void_p),
                                    b.ctypes.data_as(ctypes.c_void_p)), "mlp_set_params")

    def split(self, flat_w, flat_b):
        """Per-layer views (W_l of shape dims[l] x dims[l+1], b_l)."""
        ws, bs, ow, ob = [], [], 0, 0
        for a, c in zip(self.dims[:-1], self.dims[1:]):
            ws.append(flat_w[ow: ow + a * c].reshape(a, c))
            bs.append(flat_b[ob: ob + c])
            ow += a * c
            ob += c
        return ws, bs

    def forward(self, x):
        import torch
        y = torch.empty((x.shape[0], self.dims[-1]), dtype=torch.float32, device=x.device)
        _check(lib().mlp_forward(self._h, x.shape[0], _dp(x), _dp(y)), "mlp_forward")
        return y

    def gradients(self, x, t):
        gw = np.empty(self.nw, dtype=np.float32)
        gb = np.empty(self.nb, dtype=np.float32)
        loss = ctypes.c_float()
        _check(lib().mlp_gradients(self._h, x.shape[0], _dp(x), _dp(t), gw.ctypes.data_as(ctypes.c_void_p),
                                   gb.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss)), "mlp_gradients")
        return gw, gb, loss.value

    def train_step(self, x, t, lr=1e-3) -> float:
        loss = ctypes.c_float()
        _check(lib().mlp_train_step(self._h, x.shape[0], _dp(x), _dp(t), float(lr), ctypes.byref(loss)),
               "mlp_train_step")
        return loss.value
