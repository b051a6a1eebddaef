"""The GPU's residual check (the stopping test of Section V-B) against values
worked out by hand on Example 1's matrix, in both precisions; and a residual
query between checks leaves the run's stopping iteration unchanged."""
import json
import os
import sys
from math import sqrt

import numpy as np
import pytest

from paper_2203_05027_amd import instances as I
from paper_2203_05027_amd.solver import Solver

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(msg):
    sys.__stderr__.write(f"[gpu-test] {msg}\n")
    sys.__stderr__.flush()


def _example1(b, c, **kw):
    A = np.array(json.load(open(os.path.join(GOLDEN, "example1.json")))["A"], float)
    rr, cc = np.nonzero(A)
    row_ptr = np.zeros(4, np.int64)
    np.cumsum(np.bincount(rr, minlength=3), out=row_ptr[1:])
    return Solver(3, 5, row_ptr, cc.astype(np.int32), A[rr, cc], b, c, 5, (), eps=0.0, **kw)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("slabs", [1, 2])
def test_example1_hand_residuals(precision, slabs):
    """Same data and state as the oracle pin: b = (2,1,2), c = (1,2,2,0,4),
    x = (1,1,0,0,0), z = e_1, lambda = (-1,-1,0), delta = (0,1,0,2,0):
    r_prim = sqrt(2)/4, r_dual = sqrt(130)/6, r_gap = 2/5, ||Ax - b|| =
    sqrt(11), ||Az - b||_inf = 1, ||A'lambda + c - delta||_inf = 8 (all
    entries are small integers, exact in FP32 as well)."""
    with _example1([2.0, 1.0, 2.0], [1.0, 2.0, 2.0, 0.0, 4.0], precision=precision,
                   slabs_row=slabs, slabs_col=slabs) as s:
        s.set_start([1, 1, 0, 0, 0], [1, 0, 0, 0, 0], [0, 1, 0, 2, 0], [-1, -1, 0])
        r = s.residuals()
    want = {"r_prim": sqrt(2) / 4, "r_dual": sqrt(130) / 6, "r_gap": 2 / 5, "kkt": sqrt(130) / 6,
            "pobj": 1.0, "dobj": 3.0, "res_ax_b": sqrt(11), "prim_inf": 1.0, "dual_inf": 8.0,
            "scale_p": 2.0, "scale_d": 9.0, "pobj_x": 3.0, "gap_x": 0.0}
    for k, v in want.items():
        assert r[k] == pytest.approx(v, rel=1e-14, abs=1e-15), (k, r[k], v)


def test_gap_dominated_kkt():
    with _example1([1.0, 0.0, 2.0], [1.0, 2.0, 2.0, 0.0, 4.0]) as s:
        s.set_start([1, 0, 0, 0, 0], [1, 0, 0, 0, 0], [2, 2, 6, 6, 12], [1, 0, 0])
        r = s.residuals()
    assert r["r_prim"] == 0.0 and r["r_dual"] == 0.0
    assert r["kkt"] == pytest.approx(2 / 3, rel=1e-15)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_polling_residuals_keeps_the_stopping_iteration(precision):
    """A run that reads its residuals every 7 iterations (between the checks
    every 10) stops at the same check, with the same iterate, as one that
    never reads them."""
    inst = I.config_instance("lp_small")
    with Solver.from_instance(inst, eps=1e-4, check_every=10, precision=precision) as a:
        a.iterate(60_000)
        ra = a.residuals()
        sa = a.solution()
    polls = 0
    with Solver.from_instance(inst, eps=1e-4, check_every=10, precision=precision) as b:
        while not b.iterate(7):
            b.residuals()
            polls += 1
            assert polls < 10_000
        rb = b.residuals()
        sb = b.solution()
    say(f"{precision}: stop at {ra['iter']} without polling, {rb['iter']} with {polls} polls")
    assert ra["status"] == rb["status"] == "converged"
    assert ra["iter"] == rb["iter"] and ra["iter"] % 10 == 0
    for k in ("x", "z", "delta", "lambda"):
        assert np.array_equal(sa[k], sb[k]), k


def test_polling_does_not_override_max_iter():
    inst = I.lp_instance(200, 400, 4, seed=6)
    with Solver.from_instance(inst, eps=1e-12, max_iter=25, check_every=10) as s:
        s.iterate(100)
        r1 = s.residuals()
        r2 = s.residuals()
    assert r1["status"] == r2["status"] == "max_iter" and r1["iter"] == 25
