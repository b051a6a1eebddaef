"""Plain FP64 CPU oracle of the warm-start network (test infrastructure only).

A multilayer perceptron y = W_L' relu(... relu(W_1' x + b_1) ...) + b_L
(weights stored input-major, W_l of shape d_{l-1} x d_l) with the mean
squared error loss mean((y - t)^2), its gradients by the chain rule, and one
Adam step.  ``bf16=True`` rounds, at the points the GPU kernels store BF16
(the network input, the weights read by the GEMMs, the hidden activations and
the back-propagated pre-activation gradients), to the nearest BF16 value with
ties to even, so that the GPU and this oracle differ only by the order of the
FP32 sums.
"""
from __future__ import annotations

import numpy as np


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Nearest BF16 value (ties to even) of FP32-representable input."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def forward(ws, bs, x, bf16=False):
    """Returns the output and the list of layer inputs a_0 .. a_{L-1}."""
    r = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    a = r(x)
    acts = [a]
    L = len(ws)
    for l in range(L):
        z = a @ r(ws[l]) + np.asarray(bs[l], dtype=np.float64)
        if l < L - 1:
            a = r(np.maximum(z, 0.0))
            acts.append(a)
        else:
            a = z
    return a, acts


def loss_and_grads(ws, bs, x, t, bf16=False):
    """MSE loss and its gradients with respect to every W_l and b_l."""
    r = bf16_round if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    y, acts = forward(ws, bs, x, bf16)
    diff = y - np.asarray(t, dtype=np.float64)
    n = diff.size
    loss = float((diff * diff).sum() / n)
    dz = 2.0 * diff / n
    gws, gbs = [None] * len(ws), [None] * len(ws)
    for l in range(len(ws) - 1, -1, -1):
        dzr = r(dz)
        gws[l] = acts[l].T @ dzr
        gbs[l] = dz.sum(axis=0)
        if l > 0:
            dz = (dzr @ r(ws[l]).T) * (acts[l] > 0)
    return loss, gws, gbs


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam update; returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
