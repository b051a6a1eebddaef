"""GPU tests of the warm-start kernels: FP32 GEMM, BF16 MFMA GEMM (operand
lane layout), MLP forward/backward/Adam against the FP64 oracle, and the
PCA fit against numpy's SVD."""
import sys

import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu


def say(msg):
    sys.__stderr__.write(f"[gpu-test] {msg}\n")
    sys.__stderr__.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("M_,N_,K_,ta,tb", [(64, 64, 16, False, False), (70, 33, 129, False, True),
                                            (1, 300, 7, True, False), (257, 65, 64, True, True)])
def test_gemm_f32(torch_cuda, M_, N_, K_, ta, tb):
    from paper_2203_05027_amd import learn
    torch = torch_cuda
    rng = np.random.default_rng(0)
    A = rng.standard_normal((K_, M_) if ta else (M_, K_)).astype(np.float32)
    B = rng.standard_normal((N_, K_) if tb else (K_, N_)).astype(np.float32)
    C0 = rng.standard_normal((M_, N_)).astype(np.float32)
    C = torch.from_numpy(C0.copy()).cuda()
    learn.gemm(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), C, alpha=0.5, beta=2.0,
               transA=ta, transB=tb)
    ref = 0.5 * ((A.T if ta else A).astype(np.float64) @ (B.T if tb else B)) + 2.0 * C0
    np.testing.assert_allclose(C.cpu().numpy(), ref, rtol=1e-4, atol=1e-4 * np.abs(ref).max())


def _bits(t):
    return t.view(np.uint32) >> 16


@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
def test_gemm_bf16_lane_layout(torch_cuda, ta, tb):
    """The MFMA kernel against an FP64 product of the same BF16 values: a
    wrong operand or accumulator lane layout permutes entries and fails."""
    from paper_2203_05027_amd import learn
    torch = torch_cuda
    rng = np.random.default_rng(1)
    Mm, Nn, Kk = 48, 80, 64
    A = M.bf16_round(rng.standard_normal((Kk, Mm) if ta else (Mm, Kk))).astype(np.float32)
    B = M.bf16_round(rng.standard_normal((Nn, Kk) if tb else (Kk, Nn))).astype(np.float32)
    Ab = torch.from_numpy((_bits(A)).astype(np.int16)).cuda()
    Bb = torch.from_numpy((_bits(B)).astype(np.int16)).cuda()
    C = learn.gemm_bf16(Ab, Bb, transA=ta, transB=tb).cpu().numpy()
    ref = (A.T if ta else A).astype(np.float64) @ (B.T if tb else B).astype(np.float64)
    np.testing.assert_allclose(C, ref, rtol=1e-5, atol=1e-5)


def test_mlp_forward_and_gradients(torch_cuda):
    from paper_2203_05027_amd import learn
    torch = torch_cuda
    dims = [64, 128, 96, 32]
    net = learn.MLP(dims, max_batch=64, seed=3)
    w, b = net.params()
    rng = np.random.default_rng(4)
    b = rng.standard_normal(b.size).astype(np.float32) * 0.1
    net.set_params(w, b)
    ws, bs = net.split(w.astype(np.float64), b.astype(np.float64))
    x = rng.standard_normal((48, 64)).astype(np.float32)
    t = rng.standard_normal((48, 32)).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    y = net.forward(xd).cpu().numpy()
    y_bf, _ = M.forward(ws, bs, x, bf16=True)
    y_64, _ = M.forward(ws, bs, x, bf16=False)
    say(f"forward rel err vs bf16-emulating oracle {np.abs(y - y_bf).max() / np.abs(y_bf).max():.2e}, "
        f"vs fp64 {np.abs(y - y_64).max() / np.abs(y_64).max():.2e}")
    np.testing.assert_allclose(y, y_bf, rtol=1e-4, atol=1e-4 * np.abs(y_bf).max())
    gw, gb, loss = net.gradients(xd, td)
    lo, gws, gbs = M.loss_and_grads(ws, bs, x, t, bf16=True)
    lo64, gws64, gbs64 = M.loss_and_grads(ws, bs, x, t, bf16=False)
    assert loss == pytest.approx(lo, rel=1e-4)
    gwl, gbl = net.split(gw, gb)
    for l in range(3):
        e_bf = np.linalg.norm(gwl[l] - gws[l]) / np.linalg.norm(gws[l])
        e_64 = np.linalg.norm(gwl[l] - gws64[l]) / np.linalg.norm(gws64[l])
        say(f"layer {l}: dW rel err vs bf16 oracle {e_bf:.2e}, vs fp64 oracle {e_64:.2e}")
        # Against the oracle that rounds to BF16 at the same points: where both
        # sides round the same value the difference is the FP32 summation order
        # (about K * 2^-24, K <= 128 here, so below 1e-5).  A value that lands
        # within that distance of a BF16 rounding boundary (or a pre-activation
        # within it of zero, a ReLU mask) can round the other way on one side,
        # a change of one BF16 spacing (2^-7 relative) in that one element;
        # 2e-3 in norm leaves room for such flips in a few percent of the
        # gradient's weight, far above what is seen (~1e-7).  The error against
        # the unrounded FP64 gradient measures BF16 itself, not the kernels, and
        # is reported only.
        assert e_bf <= 2e-3, (l, e_bf)
        np.testing.assert_allclose(gbl[l], gbs[l], rtol=2e-3, atol=2e-3 * np.abs(gbs[l]).max())


def test_mlp_adam_step_and_training(torch_cuda):
    from paper_2203_05027_amd import learn
    torch = torch_cuda
    dims = [16, 64, 16]
    net = learn.MLP(dims, max_batch=128, seed=5)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((128, 16)).astype(np.float32)
    Wt = rng.standard_normal((16, 16)).astype(np.float32) / 4
    t = np.tanh(x @ Wt).astype(np.float32)
    xd, td = torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()
    w0, b0 = net.params()
    gw, gb, _ = net.gradients(xd, td)
    net.train_step(xd, td, lr=1e-2)
    w1, b1 = net.params()
    pw, _, _ = M.adam_step(w0.astype(np.float64), gw.astype(np.float64), 0, 0, 1, lr=1e-2)
    np.testing.assert_allclose(w1, pw, rtol=1e-5, atol=1e-6)
    # steps 2..8: the moments accumulate across steps; each step's gradient
    # is the kernels' own at the current weights, fed to the oracle's Adam
    m_w, v_w = (1 - 0.9) * gw.astype(np.float64), (1 - 0.999) * gw.astype(np.float64) ** 2
    m_b, v_b = (1 - 0.9) * gb.astype(np.float64), (1 - 0.999) * gb.astype(np.float64) ** 2
    pw, pb = w1.astype(np.float64), net.params()[1].astype(np.float64)
    for step in range(2, 9):
        gw, gb, _ = net.gradients(xd, td)
        net.train_step(xd, td, lr=1e-2)
        pw, m_w, v_w = M.adam_step(pw, gw.astype(np.float64), m_w, v_w, step, lr=1e-2)
        pb, m_b, v_b = M.adam_step(pb, gb.astype(np.float64), m_b, v_b, step, lr=1e-2)
        w_gpu, b_gpu = net.params()
        # FP32 state on the GPU: a step moves a weight by at most lr (1e-2)
        np.testing.assert_allclose(w_gpu, pw, rtol=1e-5, atol=1e-6 * step)
        np.testing.assert_allclose(b_gpu, pb, rtol=1e-5, atol=1e-6 * step)
        pw, pb = w_gpu.astype(np.float64), b_gpu.astype(np.float64)
    losses = [net.train_step(xd, td, lr=3e-3) for _ in range(400)]
    say(f"training loss {losses[0]:.4f} -> {losses[-1]:.5f}")
    assert losses[-1] < 0.05 * losses[0]


def test_pca_fit_recovers_subspace(torch_cuda):
    from paper_2203_05027_amd import learn
    torch = torch_cuda
    rng = np.random.default_rng(7)
    N, D, r = 600, 3000, 12
    U = rng.standard_normal((N, r))
    V = np.linalg.qr(rng.standard_normal((D, r)))[0]
    s = np.geomspace(100, 5, r)
    Y = (U * s) @ V.T + 0.01 * rng.standard_normal((N, D)) + rng.standard_normal(D) * 3
    Yd = torch.from_numpy(Y.astype(np.float32)).cuda()
    mean, basis, sv = learn.pca_fit(Yd, k=8, oversample=16, power_iters=2, seed=1)
    Yc = Y - Y.mean(axis=0)
    _, S, Vt = np.linalg.svd(Yc, full_matrices=False)
    np.testing.assert_allclose(mean.cpu().numpy(), Y.mean(axis=0), rtol=1e-4, atol=1e-4)
    np.testing.assert_allclose(sv, S[:8], rtol=1e-3)
    Bm = basis.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(Bm @ Bm.T, np.eye(8), atol=1e-4)
    # same subspace: singular values of Vt_k Bm' are all ~1
    cos = np.linalg.svd(Vt[:8] @ Bm.T, compute_uv=False)
    say(f"principal-angle cosines min {cos.min():.6f}")
    assert cos.min() > 0.999


@pytest.mark.parametrize("Mm,Nn,Kk", [(16, 16, 16), (48, 80, 48), (256, 512, 64), (2048, 2048, 96)])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True)])
def test_gemm_bf16_tiles_and_ragged_k(torch_cuda, Mm, Nn, Kk, ta, tb):
    """Block tiles of both sizes (64 and 128: the 2048 x 2048 case), a k that
    leaves part of the last 32-wide step empty, and both load modes of each
    operand, against an FP64 product of the same BF16 values."""
    from paper_2203_05027_amd import learn
    torch = torch_cuda
    rng = np.random.default_rng(Mm + Nn + Kk)
    A = M.bf16_round(rng.standard_normal((Kk, Mm) if ta else (Mm, Kk))).astype(np.float32)
    B = M.bf16_round(rng.standard_normal((Nn, Kk) if tb else (Kk, Nn))).astype(np.float32)
    Ab = torch.from_numpy((_bits(A)).astype(np.int16)).cuda()
    Bb = torch.from_numpy((_bits(B)).astype(np.int16)).cuda()
    C = learn.gemm_bf16(Ab, Bb, transA=ta, transB=tb).cpu().numpy()
    ref = (A.T if ta else A).astype(np.float64) @ (B.T if tb else B).astype(np.float64)
    np.testing.assert_allclose(C, ref, rtol=1e-5, atol=1e-4)


def test_gemm_bf16_unaligned_operands(torch_cuda):
    """Operands that start 2 bytes off a 16-byte boundary take the
    element-wise load path and give the same product."""
    from paper_2203_05027_amd import learn
    torch = torch_cuda
    rng = np.random.default_rng(3)
    Mm, Nn, Kk = 64, 96, 80
    A = M.bf16_round(rng.standard_normal((Mm, Kk))).astype(np.float32)
    B = M.bf16_round(rng.standard_normal((Kk, Nn))).astype(np.float32)
    Ab = torch.zeros(Mm * Kk + 1, dtype=torch.int16, device="cuda")
    Bb = torch.zeros(Kk * Nn + 1, dtype=torch.int16, device="cuda")
    Ab[1:] = torch.from_numpy(_bits(A).astype(np.int16).reshape(-1)).cuda()
    Bb[1:] = torch.from_numpy(_bits(B).astype(np.int16).reshape(-1)).cuda()
    C = learn.gemm_bf16(Ab[1:].view(Mm, Kk), Bb[1:].view(Kk, Nn)).cpu().numpy()
    np.testing.assert_allclose(C, A.astype(np.float64) @ B.astype(np.float64), rtol=1e-5, atol=1e-4)
