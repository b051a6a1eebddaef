"""Learned warm start for a parametric LP family (one A and c, b = b(theta)).

Pipeline, every numeric step in the library's kernels:
 1. solve the training members with the plain method (the family solver,
    cold start) and keep their primal-dual solutions [z ; lambda] on the GPU;
 2. fit a principal-component basis of those solutions (randomized range
    finder on the library's FP32 GEMM);
 3. train a BF16 MLP theta -> standardized PCA coefficients (MFMA GEMMs,
    Adam);
 4. for a new theta: coefficients -> [x ; lambda] = mean + basis' coef ->
    start z = max(x, 0), delta = max(c + A'lambda, 0) -> iterate; the
    cold-started plain method remains the fallback (a member the warm start
    leaves unconverged is re-solved cold).
"""
from __future__ import annotations

import time

import numpy as np

from . import learn
from .solver import Family


class WarmStart:
    def __init__(self, fam, k=256, hidden=(512, 512), B=256, precision="mixed", mu=1.0,
                 check_every=10, seed=0, log=print):
        import torch
        self.torch = torch
        self.fam = fam
        self.k = int(k)
        self.B = int(B)
        self.dims = [fam.p, *hidden, self.k]
        self.opts = dict(mu=mu, precision=precision, check_every=check_every)
        self.seed = seed
        self.log = log or (lambda *_: None)
        self.D = fam.n + fam.m
        self.mean = self.basis = self.sv = None
        self.net = None
        self.scale = None

    def _family(self, eps, max_iter):
        f = self.fam
        return Family(f.m, f.n, f.row_ptr, f.col_idx, f.val, f.c, B=self.B, eps=eps,
                      max_iter=max_iter, **self.opts)

    # 1. training data --------------------------------------------------
    def solve_members(self, thetas, eps=1e-3, max_iter=20_000, out=None):
        """Cold solves of every theta; rows [z ; lambda] go into the GPU
        tensor ``out`` (len(thetas) x (n + m)).  Returns per-member stats."""
        torch = self.torch
        N = len(thetas)
        if out is None:
            out = torch.empty((N, self.D), dtype=torch.float32, device="cuda")
        iters = np.zeros(N, dtype=np.int64)
        conv = np.zeros(N, dtype=bool)
        t0 = time.time()
        with self._family(eps, max_iter) as F:
            for g0 in range(0, N, self.B):
                th = thetas[g0: g0 + self.B]
                F.set_rhs(self.fam.b_many(th))
                while F.iterate(2000):
                    pass
                res = F.residuals()
                iters[g0: g0 + len(th)] = [r["iter"] for r in res]
                conv[g0: g0 + len(th)] = [r["status"] == "converged" for r in res]
                F.solution_device(out[g0:].data_ptr(), self.D)
                self.log(f"solved {g0 + len(th)}/{N}: median iters {int(np.median(iters[g0:g0 + len(th)]))}, "
                         f"{time.time() - t0:.1f} s")
        return out, {"iters": iters, "converged": conv, "seconds": time.time() - t0}

    # 2. basis ----------------------------------------------------------
    def fit_basis(self, Y, oversample=32, power_iters=2):
        """PCA of the rows of Y (centered in place); returns the standardized
        coefficients of the rows (N x k)."""
        torch = self.torch
        self.mean, self.basis, self.sv = learn.pca_fit(Y, self.k, oversample, power_iters, self.seed)
        coef = learn.gemm(Y, self.basis, transB=True)             # (Y - mean) basis'
        # standardize: each coefficient has variance sv^2 / N
        self.scale = torch.from_numpy(np.maximum(self.sv / np.sqrt(Y.shape[0]), 1e-12).astype(np.float32)).cuda()
        return coef / self.scale

    # 3. network --------------------------------------------------------
    def train(self, thetas, targets, epochs=200, batch=256, lr=1e-3, lr_min=1e-5):
        torch = self.torch
        N = len(thetas)
        X = torch.from_numpy(np.asarray(thetas, dtype=np.float32)).cuda()
        self.net = learn.MLP(self.dims, max_batch=batch, seed=self.seed + 1)
        rng = np.random.default_rng(self.seed)
        steps = epochs * (N // batch)
        hist, s = [], 0
        t0 = time.time()
        for ep in range(epochs):
            perm = torch.from_numpy(rng.permutation(N)).cuda()
            tot = 0.0
            for q in range(N // batch):
                idx = perm[q * batch:(q + 1) * batch]
                xb = X.index_select(0, idx).contiguous()
                tb = targets.index_select(0, idx).contiguous()
                cur = lr_min + 0.5 * (lr - lr_min) * (1 + np.cos(np.pi * s / max(steps, 1)))
                tot += self.net.train_step(xb, tb, lr=cur)
                s += 1
            hist.append(tot / max(N // batch, 1))
            if ep % max(epochs // 10, 1) == 0 or ep == epochs - 1:
                self.log(f"epoch {ep}: train mse {hist[-1]:.5f} ({time.time() - t0:.1f} s)")
        return hist

    def predict(self, thetas):
        """[x ; lambda] predictions (GPU, len(thetas) x (n + m))."""
        torch = self.torch
        th = np.asarray(thetas, dtype=np.float32)
        n = len(th)
        pad = (-n) % 16
        X = torch.from_numpy(np.concatenate([th, np.zeros((pad, th.shape[1]), np.float32)])).cuda()
        outs = []
        for g in range(0, len(X), self.net.max_batch):
            outs.append(self.net.forward(X[g: g + self.net.max_batch].contiguous()))
        coef = (torch.cat(outs)[:n] * self.scale).contiguous()
        Yhat = learn.gemm(coef, self.basis)                        # coef basis
        learn.add_row_vector(Yhat, self.mean)
        return Yhat

    def model_error(self, Yhat, Ytrue):
        """Relative error of predictions against solutions (per row, median)."""
        d = (Yhat - Ytrue).norm(dim=1) / Ytrue.norm(dim=1).clamp_min(1e-30)
        return float(d.median())

    # 4. warm vs cold ---------------------------------------------------
    def compare(self, thetas, eps=1e-4, max_iter=100_000, parts="both"):
        """Iterations and time to eps from cold and from learned starts for
        the same members; a warm start that fails to converge falls back to
        a cold solve (counted in its time and iterations)."""
        torch = self.torch
        N = len(thetas)
        cold_it = np.zeros(N, np.int64)
        warm_it = np.zeros(N, np.int64)
        cold_ok = np.zeros(N, bool)
        warm_ok = np.zeros(N, bool)
        t_cold = t_warm = t_pred = 0.0
        with self._family(eps, max_iter) as F:
            for g0 in range(0, N, self.B):
                th = thetas[g0: g0 + self.B]
                nb = len(th)
                b = self.fam.b_many(th)
                F.set_rhs(b)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                while F.iterate(2000):
                    pass
                t_cold += time.perf_counter() - t0
                r = F.residuals()
                cold_it[g0:g0 + nb] = [x["iter"] for x in r]
                cold_ok[g0:g0 + nb] = [x["status"] == "converged" for x in r]
                F.set_rhs(b)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                Yhat = self.predict(th)
                F.set_start_predicted(Yhat.data_ptr(), self.D, parts)
                torch.cuda.synchronize()
                t_pred += time.perf_counter() - t0
                while F.iterate(2000):
                    pass
                t_warm += time.perf_counter() - t0
                r = F.residuals()
                warm_it[g0:g0 + nb] = [x["iter"] for x in r]
                warm_ok[g0:g0 + nb] = [x["status"] == "converged" for x in r]
                if not warm_ok[g0:g0 + nb].all():           # fallback: cold solve
                    F.set_rhs(b)
                    t0 = time.perf_counter()
                    while F.iterate(2000):
                        pass
                    t_warm += time.perf_counter() - t0
                    r = F.residuals()
                    for q in np.nonzero(~warm_ok[g0:g0 + nb])[0]:
                        warm_it[g0 + q] += r[q]["iter"]
                        warm_ok[g0 + q] = r[q]["status"] == "converged"
                self.log(f"compare {g0 + nb}/{N}: cold median {int(np.median(cold_it[g0:g0+nb]))} "
                         f"warm median {int(np.median(warm_it[g0:g0+nb]))}")
        return {"cold_iters": cold_it, "warm_iters": warm_it, "cold_converged": cold_ok,
                "warm_converged": warm_ok, "cold_seconds": t_cold, "warm_seconds": t_warm,
                "predict_seconds": t_pred}
