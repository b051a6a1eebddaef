"""Primal half first: a check whose primal part fails the stopping test
skips its column half (full_checks = 0, the default), since it cannot stop
the run.  Against every check evaluated whole (full_checks = 1): the same
stopping iteration and status, bit for bit the same iterates and final
residuals, for the three stopping tests, both precisions, with and without
XCD slabs; residual queries stay whole."""
import sys

import numpy as np
import pytest

from paper_2203_05027_amd import instances as I
from paper_2203_05027_amd.solver import Solver

pytestmark = pytest.mark.gpu

RES = ("r_prim", "r_dual", "r_gap", "kkt", "pobj", "dobj", "res_ax_b", "prim_inf", "dual_inf", "pobj_x", "gap_x",
       "iter", "status")


def say(msg):
    sys.__stderr__.write(f"[gpu-test] {msg}\n")
    sys.__stderr__.flush()


_INST = {}


def inst():
    if not _INST:
        _INST["lp"] = I.lp_instance(1500, 3000, 5, seed=51)
    return _INST["lp"]


CRIT = {"kkt": dict(criterion="kkt", eps=1e-4),
        "inf": dict(criterion="inf", eps=1e-4, eps_abs=1e-6),
        "pogs": dict(criterion="pogs", eps_abs=2e-3, eps_gap=2e-2)}


def _run(full, precision, slabs, crit):
    kw = dict(CRIT[crit], precision=precision, check_every=10, resident="never", max_iter=200_000)
    if slabs > 1:
        kw.update(slabs_row=slabs, slabs_col=slabs)
    with Solver.from_instance(inst(), full_checks=full, **kw) as s:
        while not s.iterate(5000):
            pass
        return s.solution(), s.residuals(), s.launch_shape()


@pytest.mark.parametrize("crit", ["kkt", "inf", "pogs"])
@pytest.mark.parametrize("slabs", [1, 2])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gated_checks_stop_where_whole_checks_stop(precision, slabs, crit):
    g_sol, g_res, shape = _run(False, precision, slabs, crit)
    f_sol, f_res, _ = _run(True, precision, slabs, crit)
    say(f"{precision} slabs {slabs} {crit}: shape {shape}, stop at {g_res['iter']} ({g_res['status']}), "
        f"kkt {g_res['kkt']:.3e}")
    assert g_res["status"] == "converged"
    for k in RES:
        assert g_res[k] == f_res[k], (k, g_res[k], f_res[k])
    for k in g_sol:
        assert np.array_equal(g_sol[k], f_sol[k]), k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_residual_queries_stay_whole(precision):
    """Between checks and right after a check whose column half was skipped,
    a residual query evaluates every residual: the same values as with every
    check whole."""
    out = []
    for full in (False, True):
        with Solver.from_instance(inst(), eps=1e-4, check_every=10, resident="never", precision=precision,
                                  full_checks=full) as s:
            vals = []
            for k in (30, 5, 15):  # ends on a check, between checks, on a check
                s.iterate(k)
                vals.append(s.residuals())
            out.append(vals)
    for a, b in zip(*out):
        assert a["r_prim"] > 1e-4  # these checks' primal halves fail: gated ones skip the column half
        for k in RES:
            assert a[k] == b[k], (k, a[k], b[k])


def test_batched_gated_checks_match_whole_checks():
    """The batched solver with primal-first checks against every check
    whole: every instance stops at the same iteration with the same status,
    bit for bit the same iterates and the same residuals of its stopping
    check."""
    from paper_2203_05027_amd.solver import Batch
    insts = [I.lp_instance(m, 2 * m, 6, seed=60 + q) for q, m in enumerate((60, 90, 150, 240, 400, 700))]
    out = []
    for full in (False, True):
        with Batch(insts, precision="mixed", eps=1e-4, max_iter=200_000, full_checks=full) as b:
            while b.iterate(5000):
                pass
            out.append([(b.solution(i), b.residuals(i)) for i in range(len(insts))])
    for i, ((s1, r1), (s2, r2)) in enumerate(zip(*out)):
        say(f"batched instance {i}: stop at {r1['iter']} ({r1['status']})")
        assert r1["status"] == "converged"
        for k in ("iter", "status", "kkt", "r_prim", "r_dual", "r_gap", "pobj", "dobj", "res_ax_b"):
            assert r1[k] == r2[k], (i, k, r1[k], r2[k])
        for k in s1:
            assert np.array_equal(s1[k], s2[k]), (i, k)


def test_standard_baseline_gated_checks_match_whole_checks():
    """The standard ADMM + CG baseline gates its checks the same way: the
    same stopping iteration, iterates and final residuals."""
    from paper_2203_05027_amd.solver import Standard
    src = inst()
    out = []
    for full in (False, True):
        with Standard(src["m"], src["n"], src["row_ptr"], src["col_idx"], src["val"], src["b"], src["c"],
                      cg_iters=3, eps=1e-4, max_iter=100_000, full_checks=full) as s:
            while not s.iterate(5000):
                pass
            out.append((s.solution(), s.residuals()))
    (s1, r1), (s2, r2) = out
    say(f"standard: stop at {r1['iter']} ({r1['status']})")
    assert r1["status"] == "converged"
    for k in ("iter", "status", "kkt", "r_prim", "r_dual", "r_gap", "pobj", "dobj"):
        assert r1[k] == r2[k], (k, r1[k], r2[k])
    for k in s1:
        assert np.array_equal(s1[k], s2[k]), k


@pytest.mark.parametrize("seed", range(12))
def test_random_problems_gated_like_whole(seed):
    """Drawn LPs and SOCPs (ragged shapes, check intervals 1-12, tolerances
    1e-2 to 1e-5, the three stopping tests, both precisions): primal-first
    checks stop where whole checks stop, with the same iterates."""
    rng = np.random.default_rng(900 + seed)
    if rng.random() < 0.5:
        src = I.lp_instance(int(rng.integers(20, 400)), int(rng.integers(450, 900)), 4, seed=int(rng.integers(1e6)))
    else:
        src = I.socp_instance(int(rng.integers(20, 60)), 6, seed=int(rng.integers(1e6)))
    crit = ["kkt", "inf", "pogs"][seed % 3]
    eps = float(10.0 ** -rng.uniform(2, 5))
    kw = dict(precision=["fp64", "mixed"][seed % 2], check_every=int(rng.integers(1, 13)), resident="never",
              max_iter=30_000, criterion=crit, eps=eps)
    if crit == "inf":
        kw["eps_abs"] = eps * 1e-2
    if crit == "pogs":
        kw.update(eps_abs=eps * 10, eps_gap=eps * 100)
    out = []
    for full in (False, True):
        with Solver.from_instance(src, full_checks=full, **kw) as s:
            while not s.iterate(4000):
                pass
            out.append((s.solution(), s.residuals()))
    (g, rg), (f, rf) = out
    say(f"seed {seed}: m={src['m']} n={src['n']} {kw['precision']} {crit} eps {eps:.1e} ce {kw['check_every']}: "
        f"stop {rg['iter']} ({rg['status']})")
    for k in RES:
        assert rg[k] == rf[k], (k, rg[k], rf[k])
    for k in g:
        assert np.array_equal(g[k], f[k]), k


@pytest.mark.parametrize("crit", ["kkt", "inf", "pogs"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_resident_gated_checks_match_whole_checks(precision, crit):
    """The resident path (the whole problem in one CU's LDS) gates its
    checks inside the launch: the same stopping iteration, iterates and
    final residuals as every check whole; so does the no-allocation solve."""
    from paper_2203_05027_amd.solver import solve
    src = I.lp_instance(300, 700, 5, seed=53)
    kw = dict(CRIT[crit], precision=precision, check_every=10, max_iter=200_000)
    out = []
    for full in (False, True):
        with Solver.from_instance(src, resident="required", full_checks=full, **kw) as s:
            while not s.iterate(5000):
                pass
            out.append((s.solution(), s.residuals()))
    (g, rg), (f, rf) = out
    say(f"resident {precision} {crit}: stop at {rg['iter']} ({rg['status']})")
    assert rg["status"] == "converged"
    for k in RES:
        assert rg[k] == rf[k], (k, rg[k], rf[k])
    for k in g:
        assert np.array_equal(g[k], f[k]), k
    rc, sol, res = solve(src, 200_000, noalloc=True, **kw)
    assert res["iter"] == rg["iter"] and res["kkt"] == rg["kkt"]
    for k in g:
        assert np.array_equal(sol[k], g[k]), k
