"""GPU tests of the parametric-family solver (one A, many b) against the
CPU oracle run on each member alone."""
import sys

import numpy as np
import pytest

import oracle
from paper_2203_05027_amd import instances as I
from paper_2203_05027_amd.solver import Family

pytestmark = pytest.mark.gpu
KEYS = ("x", "z", "delta", "lambda")


def say(msg):
    sys.__stderr__.write(f"[gpu-test] {msg}\n")
    sys.__stderr__.flush()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def family_members(fam, thetas):
    return [fam.instance(t) for t in thetas]


@pytest.fixture(scope="module")
def small_family():
    return I.ParametricFamily(m=300, n=600, k=5, p=8, seed=7)


@pytest.mark.parametrize("B,nb", [(64, 5), (128, 70)])
def test_fp64_family_matches_oracle(small_family, B, nb):
    fam = small_family
    thetas = [fam.theta(1000 + i, p=8) for i in range(nb)]
    insts = family_members(fam, thetas)
    say(f"family B={B} nb={nb}")
    with Family(fam.m, fam.n, fam.row_ptr, fam.col_idx, fam.val, fam.c, B=B, precision="fp64",
                eps=0.0, check_every=7) as F:
        F.set_rhs(np.stack([i["b"] for i in insts]))
        F.iterate(200)
        sol = F.solution()
        res = F.residuals()
    for l in (0, 1, nb // 2, nb - 1):
        o = oracle.Oracle.from_instance(insts[l])
        o.iterate(200)
        s = o.state()
        errs = {k: rel(sol[k][l], s[k]) for k in KEYS}
        assert max(errs.values()) <= 1e-9, (l, errs)
        r = o.residuals()
        assert res[l]["iter"] == 200 or res[l]["status"] == "running"


def test_fp64_family_convergence_matches_oracle(small_family):
    fam = small_family
    insts = family_members(fam, [fam.theta(2000 + i, p=8) for i in range(3)])
    with Family(fam.m, fam.n, fam.row_ptr, fam.col_idx, fam.val, fam.c, B=64, precision="fp64",
                eps=1e-4) as F:
        F.set_rhs(np.stack([i["b"] for i in insts]))
        assert F.iterate(300_000) == 0
        res = F.residuals()
    for l, inst in enumerate(insts):
        ro = oracle.Oracle.from_instance(inst).solve(1e-4, check_every=10, max_iter=300_000)
        say(f"member {l}: family {res[l]['iter']} oracle {ro['iter']}")
        assert res[l]["status"] == "converged" and res[l]["iter"] == ro["iter"]
        assert abs(res[l]["pobj"] - ro["pobj"]) <= 1e-9 * abs(ro["pobj"])


def test_warm_start_at_solution_is_converged(small_family):
    """Starting from a solution (x*, lambda*) the predicted-start mapping
    (z = max(x, 0), delta = max(c + A'lambda, 0)) is converged at once."""
    import torch
    assert torch.cuda.is_available()
    fam = small_family
    insts = family_members(fam, [fam.theta(3000 + i, p=8) for i in range(4)])
    b = np.stack([i["b"] for i in insts])
    with Family(fam.m, fam.n, fam.row_ptr, fam.col_idx, fam.val, fam.c, B=64, precision="mixed",
                eps=1e-5) as F:
        F.set_rhs(b)
        assert F.iterate(400_000) == 0
        cold = [r["iter"] for r in F.residuals()]
        sol = F.solution()
        xl = np.concatenate([sol["z"], sol["lambda"]], axis=1).astype(np.float32)
        dev = torch.from_numpy(xl).cuda()
        F.set_rhs(b)
        F.set_start_predicted(dev.data_ptr(), xl.shape[1], "both")
        torch.cuda.synchronize()
        s0 = F.solution()
        np.testing.assert_allclose(s0["z"], np.maximum(xl[:, :fam.n], 0), rtol=1e-6, atol=1e-6)
        A = np.zeros((fam.m, fam.n))
        A[np.repeat(np.arange(fam.m), np.diff(fam.row_ptr)), fam.col_idx] = fam.val
        dl = np.maximum(fam.c[None, :] + xl[:, fam.n:].astype(np.float64) @ A, 0)
        np.testing.assert_allclose(s0["delta"], dl, rtol=1e-9, atol=1e-9)
        F.iterate(400_000)
        warm = [r["iter"] for r in F.residuals()]
    say(f"cold {cold} warm {warm}")
    assert all(w <= 0.1 * c + 20 for w, c in zip(warm, cold))


def test_mixed_family_reaches_optimum(small_family):
    fam = small_family
    thetas = [fam.theta(4000 + i, p=8) for i in range(64)]
    insts = family_members(fam, thetas)
    with Family(fam.m, fam.n, fam.row_ptr, fam.col_idx, fam.val, fam.c, B=64, precision="mixed",
                eps=1e-4) as F:
        F.set_rhs(np.stack([i["b"] for i in insts]))
        assert F.iterate(400_000) == 0
        res = F.residuals()
    for l in range(0, 64, 9):
        ro = oracle.Oracle.from_instance(insts[l]).solve(1e-5, check_every=50, max_iter=400_000)
        assert res[l]["kkt"] <= 1e-4
        assert abs(res[l]["pobj"] - ro["pobj"]) <= 2e-3 * (1 + abs(ro["pobj"]))
