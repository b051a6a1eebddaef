"""Parity at full size, in the launch configuration the benchmark times
(automatic lanes, unroll and XCD slabs, graph replay): the 1e6 x 2e6 LP and
the 1e5-cone SOCP after 200 iterations from the zero start, every entry of
x, z, delta and lambda against the FP64 oracle at 1e-9 of the vector's
largest entry; the mixed form's error against the same oracle, stated per
result; and the mixed form's iteration count to a 1e-4 KKT residual against
the FP64 solver's on the LP; and the default primal-first checks against
every check whole on the LP, to 1e-4."""
import sys

import numpy as np
import pytest

import oracle
from paper_2203_05027_amd import instances as I
from paper_2203_05027_amd.solver import Solver

pytestmark = pytest.mark.gpu

KEYS = ("x", "z", "delta", "lambda")
RES = ("r_prim", "r_dual", "r_gap", "kkt", "pobj", "dobj", "res_ax_b")
ITERS = 200


def say(msg):
    sys.__stderr__.write(f"[gpu-test] {msg}\n")
    sys.__stderr__.flush()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


_cache = {}


def _oracle_after(name):
    """Instance and the oracle's state and residuals after 200 iterations
    (computed once per module)."""
    if name not in _cache:
        inst = I.config_instance(name)
        say(f"{name}: m={inst['m']} n={inst['n']} nnz={inst['nnz']}; oracle {ITERS} iterations")
        orc = oracle.Oracle.from_instance(inst)
        orc.iterate(ITERS)
        _cache[name] = (inst, orc.state(), orc.residuals())
        orc.close()
        say(f"{name}: oracle done")
    return _cache[name]


@pytest.mark.parametrize("name", ["lp_large", "socp_large"])
def test_fp64_200_iterations(name):
    inst, o, ro = _oracle_after(name)
    with Solver.from_instance(inst, eps=0.0, check_every=10) as s:
        say(f"{name}: launch shape {s.launch_shape()}")
        s.iterate(ITERS)
        g = s.solution()
        r = s.residuals()
    errs = {k: rel(g[k], o[k]) for k in KEYS}
    say(f"{name} fp64 after {ITERS}: {errs}")
    for k in KEYS:
        assert errs[k] <= 1e-9, (k, errs[k])
    for k in RES:
        assert abs(r[k] - ro[k]) <= 1e-9 * max(abs(ro[k]), 1e-12), (k, r[k], ro[k])
    assert r["iter"] == ITERS


# The mixed form rounds A, x, z, u, b and c to FP32 for the sweep (relative
# 2^-24 per value), keeps lambda and delta in FP64 and evaluates the residuals
# in FP64.  The bounds below are what 200 iterations of that rounding give,
# with margin; the measured values are printed and recorded with the design.
MIXED_BOUND = {"x": 1e-5, "z": 1e-5, "delta": 1e-5, "lambda": 1e-5}


@pytest.mark.parametrize("name", ["lp_large", "socp_large"])
def test_mixed_200_iterations_error_per_result(name):
    """Per result: the vectors relative to their largest entry; the relative
    residuals r_prim, r_dual, r_gap and kkt (already scaled to O(1)) in
    absolute terms against 1 % of the 1e-4 stopping tolerance, so the
    rounding cannot move the stop decision by more than that band; the
    objectives against the vectors' error carried through the dot products;
    ||Ax - b|| against 1e-6 (1 + ||b||), the scale the primal residual is
    normalised by."""
    inst, o, ro = _oracle_after(name)
    with Solver.from_instance(inst, eps=0.0, check_every=10, precision="mixed") as s:
        s.iterate(ITERS)
        g = s.solution()
        r = s.residuals()
    errs = {k: rel(g[k], o[k]) for k in KEYS}
    aerr = {k: abs(r[k] - ro[k]) for k in RES}
    say(f"{name} mixed vs fp64 oracle after {ITERS}: vectors {errs}")
    say(f"{name} oracle residuals after {ITERS}: {ro}")
    say(f"{name} mixed residual errors (absolute) after {ITERS}: {aerr}")
    for k in KEYS:
        assert errs[k] <= MIXED_BOUND[k], (k, errs[k])
    for k in ("r_prim", "r_dual", "r_gap", "kkt"):
        assert aerr[k] <= 1e-6, (k, aerr[k])
    # objectives: c'z and b'lambda move by at most ||c||_1 ||dz||_inf and
    # ||b||_1 ||dlambda||_inf, so their error is the vectors' error carried
    # through, with nothing added by the FP64 reductions
    dz = float(np.abs(g["z"] - o["z"]).max())
    dl = float(np.abs(g["lambda"] - o["lambda"]).max())
    assert aerr["pobj"] <= np.abs(inst["c"]).sum() * dz + 1e-12 * abs(ro["pobj"]), aerr["pobj"]
    assert aerr["dobj"] <= np.abs(inst["b"]).sum() * dl + 1e-12 * abs(ro["dobj"]), aerr["dobj"]
    assert aerr["res_ax_b"] <= 1e-6 * (1.0 + float(np.linalg.norm(inst["b"]))), aerr["res_ax_b"]


def test_mixed_reaches_1e4_with_the_fp64_iteration_count():
    """To a 1e-4 KKT residual on the 1e6 x 2e6 LP: the mixed form stops at
    the same check (or within one check) as FP64, with the objective within
    the KKT bound of the known optimum."""
    inst = I.config_instance("lp_large")
    out = {}
    for prec in ("fp64", "mixed"):
        with Solver.from_instance(inst, eps=1e-4, check_every=10, precision=prec) as s:
            assert s.iterate(40_000)
            out[prec] = s.residuals()
        say(f"lp_large {prec} to 1e-4: iter {out[prec]['iter']} kkt {out[prec]['kkt']:.3e} "
            f"pobj {out[prec]['pobj']:.6f} (p* {inst['p_star']:.6f})")
    for prec in out:
        assert out[prec]["status"] == "converged"
        assert abs(out[prec]["pobj"] - inst["p_star"]) <= 2e-3 * abs(inst["p_star"])
    assert abs(out["mixed"]["iter"] - out["fp64"]["iter"]) <= 10


def test_gated_checks_at_full_size():
    """The 1e6 x 2e6 LP to a 1e-4 KKT residual in FP64, checks primal half
    first (the default) against every check whole: the same stopping
    iteration, final residuals and iterates, bit for bit."""
    inst = I.config_instance("lp_large")
    out = []
    for full in (False, True):
        with Solver.from_instance(inst, eps=1e-4, check_every=10, full_checks=full) as s:
            assert s.iterate(40_000)
            out.append((s.residuals(), s.solution()))
    (rg, g), (rf, f) = out
    say(f"lp_large gated vs whole checks: stop at {rg['iter']} / {rf['iter']}, kkt {rg['kkt']:.3e}")
    for k in RES + ("iter", "status", "pobj_x", "gap_x"):
        assert rg[k] == rf[k], (k, rg[k], rf[k])
    for k in KEYS:
        assert np.array_equal(g[k], f[k]), k
