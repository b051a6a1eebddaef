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

Members stream through the family solver's B slots: a slot whose member
stops takes the next pending member at once (family_refill), so the time to
solve a set of members follows their total iteration count rather than the
slowest member of each group of B.  Once no member is pending and only a few
still run, one group iteration (all B slots' traffic) costs more than those
few members' iterations on the single-problem solver: the remaining members
then continue their runs there, one after another, from their exact state
(family_member_state -> solver_set_rhs + solver_resume), so a slow member
does not hold the whole group.
"""
from __future__ import annotations

import time

import numpy as np

from . import learn
from .solver import Family, Solver


class _Rhs:
    """Right-hand sides b(theta) of a member list, made on demand for the
    rows asked for (a slice or a list of member indices)."""

    def __init__(self, fam, thetas):
        self.fam, self.thetas = fam, np.asarray(thetas)

    def __len__(self):
        return len(self.thetas)

    def __getitem__(self, idx):
        return np.ascontiguousarray(self.fam.b_many(self.thetas[idx]))


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
        """Cold solves of every theta, streamed through the slots; rows
        [z ; lambda] go into the GPU tensor ``out`` (len(thetas) x (n + m)).
        Returns per-member stats."""
        torch = self.torch
        N = len(thetas)
        if out is None:
            out = torch.empty((N, self.D), dtype=torch.float32, device="cuda")
        t0 = time.time()
        st = self.solve_stream(_Rhs(self.fam, thetas), eps=eps, max_iter=max_iter, keep=out)
        self.log(f"solved {N}: median iters {int(np.median(st['iters']))}, {time.time() - t0:.1f} s")
        st["seconds"] = time.time() - t0
        return out, st

    # 2. basis ----------------------------------------------------------
    def fit_basis(self, Y, oversample=32, power_iters=2):
        """PCA of the rows of Y (centered in place); returns the standardized
        coefficients of the rows (N x k)."""
        torch = self.torch
        self.mean, self.basis, self.sv = learn.pca_fit(Y, self.k, oversample, power_iters, self.seed)
        coef = learn.gemm(Y, self.basis, transB=True)             # (Y - mean) basis'
        # standardize: each coefficient has variance sv^2 / N
        scale = np.maximum(self.sv / np.sqrt(Y.shape[0]), 1e-12).astype(np.float32)
        self.scale = torch.from_numpy(scale).cuda()
        learn.mul_row_vector(coef, torch.from_numpy((1.0 / scale).astype(np.float32)).cuda())
        return coef

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
        coef = torch.cat(outs)[:n].contiguous()
        learn.mul_row_vector(coef, self.scale)
        Yhat = learn.gemm(coef, self.basis)                        # coef basis
        learn.add_row_vector(Yhat, self.mean)
        return Yhat

    def model_error(self, Yhat, Ytrue):
        """Relative error of predictions against solutions (per row, median;
        evaluated on the host)."""
        a, t = Yhat.cpu().numpy().astype(np.float64), Ytrue.cpu().numpy().astype(np.float64)
        d = np.linalg.norm(a - t, axis=1) / np.maximum(np.linalg.norm(t, axis=1), 1e-30)
        return float(np.median(d))

    # 4. warm vs cold ---------------------------------------------------
    def solve_stream(self, b_all, Yhat=None, parts="both", eps=1e-4, max_iter=100_000, chunk=50,
                     keep=None, tail_slots=16):
        """Solves every member (row of the host array b_all) through the B
        slots, refilling a slot as soon as its member stops.  With Yhat
        (device FP32 rows [x ; lambda], one per member) a member starts from
        its prediction and, if that leaves it unconverged, is queued again
        with the zero start (the cold fallback; its iterations add up).
        keep: a device FP32 tensor (len(b_all) x (n + m)) that receives each
        member's [z ; lambda] when it stops.  Returns {"iters", "converged",
        "seconds"}; the time runs from the first right-hand side to the last
        stop (predictions are made beforehand and timed by the caller).
        tail_slots: once no member is pending and at most this many still
        run, they continue on the single-problem solver (0: never).  One
        group iteration of the 256-slot family on the 5e4 x 1e5 LP takes
        0.46 ms against 17 us for an iteration of one member alone, so a
        member moved there costs 1/27 of a group iteration per iteration;
        16 leaves room for the per-member hand-over (a state copy each way).
        Also returned: "group_iters" (iterations of the B-slot group),
        "busy" (the fraction of slot-iterations that served a member),
        "tail_iters" (group iterations after the last member got a slot),
        "handed_over" (members finished on the single-problem solver, listed
        in "handed_members") and "handover_iters" (their iterations there)."""
        torch = self.torch
        N = len(b_all)
        D = self.D
        iters = np.zeros(N, np.int64)
        conv = np.zeros(N, bool)
        tail = self._tail_solver(b_all[0:1][0], eps) if tail_slots > 0 else None
        handed, handed_iters, handed_members = 0, 0, []
        with self._family(eps, max_iter) as F:
            buf = (torch.empty((self.B, D), dtype=torch.float32, device="cuda") if keep is not None else None)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            nb = min(N, self.B)
            F.set_rhs(b_all[:nb])
            if Yhat is not None:
                F.set_start_predicted(Yhat.data_ptr(), D, parts)
            owner = list(range(nb))                  # member in each slot (None: idle)
            warm = [Yhat is not None] * nb           # whether the slot's member started warm
            nxt, retry = nb, []
            group_iters, tail_iters, busy_slot_iters = 0, 0, 0
            while True:
                F.iterate(chunk)
                stat, its = F.status_iters()  # 0 running, 1 converged, 2 max_iter, 3 numeric
                group_iters += chunk
                if nxt >= N and not retry:
                    tail_iters += chunk
                free, stopped = [], []
                for sl in range(nb):
                    mem = owner[sl]
                    if mem is None:
                        free.append(sl)
                        continue
                    if stat[sl] == 0:
                        continue
                    stopped.append(sl)
                    iters[mem] += its[sl]
                    busy_slot_iters += int(its[sl])
                    ok = stat[sl] == 1
                    if not ok and warm[sl]:
                        retry.append(mem)            # the cold fallback
                    else:
                        conv[mem] = ok
                    free.append(sl)
                if keep is not None and stopped:
                    F.solution_device(buf.data_ptr(), D)
                    for sl in stopped:
                        keep[owner[sl]].copy_(buf[sl])
                for sl in stopped:
                    owner[sl] = None
                # pending members in order (contiguous prediction rows), then cold retries
                take = min(len(free), N - nxt)
                entered = bool(take) or bool(retry and free)
                if take:
                    sl_new = free[:take]
                    ptr = Yhat[nxt].data_ptr() if Yhat is not None else None
                    F.refill(sl_new, b_all[nxt:nxt + take], dev_ptr=ptr, ld=D, parts=parts)
                    for q, sl in enumerate(sl_new):
                        owner[sl], warm[sl] = nxt + q, Yhat is not None
                    nxt += take
                    free = free[take:]
                if retry and free:
                    r_take = min(len(free), len(retry))
                    mems, retry = retry[:r_take], retry[r_take:]
                    F.refill(free[:r_take], b_all[mems])
                    for sl, mem in zip(free[:r_take], mems):
                        owner[sl], warm[sl] = mem, False
                if all(o is None for o in owner) and nxt >= N and not retry:
                    break
                running = [sl for sl in range(nb) if owner[sl] is not None]
                # (not in a pass that just refilled slots: their residuals
                # above belong to the members that left)
                if tail is not None and not entered and nxt >= N and not retry and len(running) <= tail_slots:
                    for sl in running:  # the last few continue alone
                        mem = owner[sl]
                        done_here = int(its[sl])
                        busy_slot_iters += done_here
                        ok, more = self._finish_alone(tail, F, sl, b_all[mem:mem + 1][0], eps,
                                                      max_iter - done_here, warm[sl], max_iter)
                        iters[mem] += done_here + more
                        conv[mem] = ok
                        handed += 1
                        handed_iters += more
                        handed_members.append(mem)
                        if keep is not None:
                            st = tail.solution()
                            row = np.concatenate([st["z"], st["lambda"]]).astype(np.float32)
                            keep[mem].copy_(torch.from_numpy(row))
                        owner[sl] = None
                    break
            torch.cuda.synchronize()
            seconds = time.perf_counter() - t0
        if tail is not None:
            tail.close()
        return {"iters": iters, "converged": conv, "seconds": seconds, "group_iters": group_iters,
                "busy": busy_slot_iters / max(group_iters * self.B, 1), "tail_iters": tail_iters,
                "handed_over": handed, "handover_iters": handed_iters, "handed_members": handed_members}

    def _tail_solver(self, b0, eps):
        """The single-problem solver that takes over the last running
        members (same A, c, options; its b is set per member)."""
        f = self.fam
        return Solver(f.m, f.n, f.row_ptr, f.col_idx, f.val, b0, f.c, f.n, (), eps=eps, **self.opts)

    @staticmethod
    def _finish_alone(tail, F, slot, b, eps, left, warm, max_iter):
        """Continues the member in `slot` on the single-problem solver from
        its current state for at most `left` more iterations; a warm-started
        member left unconverged is re-solved cold (its iterations add up).
        Returns (converged, iterations run here)."""
        st = F.member_state(slot)
        tail.set_rhs(b)
        tail.resume(st["x"], st["z"], st["delta"], st["lambda"])
        more = 0
        if left > 0:
            tail.iterate(left)
            more = tail.residuals()["iter"]
        ok = tail.residuals()["status"] == "converged"
        if not ok and warm:  # the cold fallback
            tail.set_start()
            tail.iterate(max_iter)
            r = tail.residuals()
            more += r["iter"]
            ok = r["status"] == "converged"
        return ok, more

    def compare_stream(self, thetas, eps=1e-4, max_iter=100_000, parts=("both",), projection=False,
                       chunk=50, tail_slots=16):
        """Cold and learned starts of the same members through the same
        streaming driver and slots (see solve_stream).  Variants: "cold", one
        per entry of parts ("both", "primal" or "dual" halves of the
        prediction) and, with projection=True, "projection": the cold
        solution projected on the PCA basis (what a perfect network could
        give with this basis).  A variant's seconds include its prediction
        time (reported apart as "predict_seconds")."""
        torch = self.torch
        N = len(thetas)
        b_all = np.ascontiguousarray(self.fam.b_many(thetas))
        keep = torch.empty((N, self.D), dtype=torch.float32, device="cuda") if projection else None
        out = {"cold": self.solve_stream(b_all, eps=eps, max_iter=max_iter, chunk=chunk, keep=keep,
                                         tail_slots=tail_slots)}
        self.log(f"stream cold: {out['cold']['seconds']:.2f} s, median {int(np.median(out['cold']['iters']))}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Yhat = self.predict(thetas)
        torch.cuda.synchronize()
        t_pred = time.perf_counter() - t0
        for p in parts:
            r = self.solve_stream(b_all, Yhat=Yhat, parts=p, eps=eps, max_iter=max_iter, chunk=chunk,
                                  tail_slots=tail_slots)
            r["seconds"] += t_pred
            out[p] = r
            self.log(f"stream {p}: {r['seconds']:.2f} s, median {int(np.median(r['iters']))}")
        del Yhat
        if projection:
            mb = learn.gemm(self.mean.reshape(1, -1).contiguous(), self.basis, transB=True)
            neg_mb = torch.from_numpy(-mb.cpu().numpy().reshape(-1)).cuda()
            coef = learn.gemm(keep, self.basis, transB=True)
            learn.add_row_vector(coef, neg_mb)
            Yp = learn.gemm(coef, self.basis)
            learn.add_row_vector(Yp, self.mean)
            out["projection"] = self.solve_stream(b_all, Yhat=Yp, eps=eps, max_iter=max_iter, chunk=chunk,
                                                  tail_slots=tail_slots)
            self.log(f"stream projection: median {int(np.median(out['projection']['iters']))}")
        out["predict_seconds"] = t_pred
        return out

    def _solve_group(self, F, b, stats, g0, fallback_b=None):
        """Iterate the family solver to its stop; record iterations and
        convergence into stats[...][g0:g0+nb]; a member left unconverged is
        re-solved cold when fallback_b is given (its iterations added)."""
        torch = self.torch
        nb = len(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while F.iterate(2000):
            pass
        r = F.residuals()
        stats["iters"][g0:g0 + nb] = [x["iter"] for x in r]
        stats["converged"][g0:g0 + nb] = [x["status"] == "converged" for x in r]
        ok = stats["converged"][g0:g0 + nb]
        if fallback_b is not None and not ok.all():
            F.set_rhs(fallback_b)
            while F.iterate(2000):
                pass
            r = F.residuals()
            for q in np.nonzero(~ok)[0]:
                stats["iters"][g0 + q] += r[q]["iter"]
                stats["converged"][g0 + q] = r[q]["status"] == "converged"
        torch.cuda.synchronize()
        stats["seconds"] += time.perf_counter() - t0

    def compare(self, thetas, eps=1e-4, max_iter=100_000, parts=("both",), projection=False):
        """Iterations and time to eps for the same members from the cold
        start and from learned starts (one per entry of parts: "both",
        "primal" or "dual" halves of the prediction used); a warm start that
        fails to converge falls back to a cold solve (counted in its time and
        iterations).  projection=True adds the start a perfect network would
        give with this basis: the cold solution projected on the PCA basis.
        Returns {variant: {"iters", "converged", "seconds"}} plus
        "predict_seconds"."""
        torch = self.torch
        N = len(thetas)

        def new():
            return {"iters": np.zeros(N, np.int64), "converged": np.zeros(N, bool), "seconds": 0.0}

        out = {"cold": new()}
        for p in parts:
            out[p] = new()
        if projection:
            out["projection"] = new()
        t_pred = 0.0
        if projection:
            mb = learn.gemm(self.mean.reshape(1, -1).contiguous(), self.basis, transB=True)
            neg_mb = torch.from_numpy(-mb.cpu().numpy().reshape(-1)).cuda()
        with self._family(eps, max_iter) as F:
            Ysol = torch.empty((self.B, self.D), dtype=torch.float32, device="cuda")
            for g0 in range(0, N, self.B):
                th = thetas[g0: g0 + self.B]
                nb = len(th)
                b = self.fam.b_many(th)
                F.set_rhs(b)
                self._solve_group(F, b, out["cold"], g0)
                if projection:
                    F.solution_device(Ysol.data_ptr(), self.D)
                Yhat = None
                for p in parts:
                    F.set_rhs(b)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    if Yhat is None:
                        Yhat = self.predict(th)
                    F.set_start_predicted(Yhat.data_ptr(), self.D, p)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    t_pred += dt
                    out[p]["seconds"] += dt
                    self._solve_group(F, b, out[p], g0, fallback_b=b)
                if projection:
                    # coefficients (Y - mean) basis' = Y basis' - mean basis', then back
                    coef = learn.gemm(Ysol[:nb].contiguous(), self.basis, transB=True)
                    learn.add_row_vector(coef, neg_mb)
                    Yp = learn.gemm(coef, self.basis)
                    learn.add_row_vector(Yp, self.mean)
                    F.set_rhs(b)
                    F.set_start_predicted(Yp.data_ptr(), self.D, "both")
                    self._solve_group(F, b, out["projection"], g0, fallback_b=b)
                self.log(f"compare {g0 + nb}/{N}: " + ", ".join(
                    f"{k} median {int(np.median(v['iters'][g0:g0 + nb]))}" for k, v in out.items()))
        out["predict_seconds"] = t_pred
        return out
