"""solver_set_rhs: one handle, a new right-hand side.  After set_rhs and a
new start the run is bitwise the run of a handle created with that b; the
handle refuses to iterate until it has a new start; residual queries
evaluate against the new b."""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2203_05027_amd import instances as I
from paper_2203_05027_amd.solver import UV_EINVAL, Solver, UvError

pytestmark = pytest.mark.gpu


def say(msg):
    sys.__stderr__.write(f"[gpu-test] {msg}\n")
    sys.__stderr__.flush()


def _second_rhs(inst, seed):
    A = sp.csr_matrix((inst["val"], inst["col_idx"], inst["row_ptr"]), shape=(inst["m"], inst["n"]))
    x = np.maximum(np.random.default_rng(seed).standard_normal(inst["n"]), 0.0)
    return A, np.ascontiguousarray(A @ x)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("resident", ["auto", "never"])
def test_set_rhs_then_start_equals_a_fresh_handle(precision, resident):
    inst = I.lp_instance(300, 700, 5, seed=41)
    A, b2 = _second_rhs(inst, 42)
    kw = dict(precision=precision, resident=resident, eps=0.0, check_every=10)
    other = dict(inst, b=b2)
    with Solver.from_instance(inst, **kw) as s, Solver.from_instance(other, **kw) as fresh:
        say(f"set_rhs {precision} {resident}: shape {s.launch_shape()}")
        s.iterate(40)
        s.set_rhs(b2)
        with pytest.raises(UvError) as ei:
            s.iterate(10)
        assert ei.value.code == UV_EINVAL
        # a residual query now evaluates the old run's iterate against b2
        x = s.solution()["x"]
        r = s.residuals()
        want = float(np.linalg.norm(A @ x - b2))
        assert r["res_ax_b"] == pytest.approx(want, rel=1e-12), (r["res_ax_b"], want)
        s.set_start()
        s.iterate(90)
        fresh.iterate(90)
        got, ref = s.solution(), fresh.solution()
        rg, rf = s.residuals(), fresh.residuals()
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k
    for k in ("iter", "kkt", "r_prim", "r_dual", "r_gap", "pobj", "dobj", "res_ax_b", "status"):
        assert rg[k] == rf[k], k


def test_set_rhs_rejects_non_finite_entries():
    inst = I.lp_instance(50, 120, 3, seed=43)
    b = inst["b"].copy()
    b[7] = np.nan
    with Solver.from_instance(inst) as s:
        with pytest.raises(UvError) as ei:
            s.set_rhs(b)
        assert ei.value.code == UV_EINVAL
        assert s.iterate(20) is False   # the old b is still in place and the handle runs
