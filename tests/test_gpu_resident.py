"""The resident path (a small orthant problem held whole in one workgroup's
LDS, iterations and checks in one launch) against the oracle and against the
sweep kernels on the same problems."""
import sys

import numpy as np
import pytest

import oracle
from paper_2203_05027_amd import instances as I
from paper_2203_05027_amd.solver import Solver

pytestmark = pytest.mark.gpu

KEYS = ("x", "z", "delta", "lambda")
RES = ("r_prim", "r_dual", "r_gap", "kkt", "pobj", "dobj", "res_ax_b", "prim_inf", "dual_inf", "scale_p",
       "scale_d", "pobj_x")


def say(msg):
    sys.__stderr__.write(f"[gpu-test] {msg}\n")
    sys.__stderr__.flush()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)) if b.size else 0.0


def _with_rows(base, A):
    rr, cc = np.nonzero(A)
    m = A.shape[0]
    row_ptr = np.zeros(m + 1, np.int64)
    np.cumsum(np.bincount(rr, minlength=m), out=row_ptr[1:])
    return dict(base, row_ptr=row_ptr, col_idx=cc.astype(np.int32), val=A[rr, cc], nnz=int(rr.size),
                b=A @ base["x0"])


def _dense(inst):
    A = np.zeros((inst["m"], inst["n"]))
    rows = np.repeat(np.arange(inst["m"]), np.diff(inst["row_ptr"]))
    A[rows, inst["col_idx"]] = inst["val"]
    return A


def _cases():
    lp = I.config_instance("lp_small")
    ragged = I.lp_instance(333, 777, 4, seed=17)
    base = I.lp_instance(400, 900, 3, seed=25)
    A = _dense(base)
    rng = np.random.default_rng(4)
    A[5, :] = rng.standard_normal(900)          # a dense row (900 entries)
    A[:, 7] = rng.standard_normal(400)          # a dense column
    A[100:140, :] = 0.0                         # empty rows
    A[:, 300:320] = 0.0                         # empty columns
    edge = _with_rows(base, A)
    tiny = I.lp_instance(3, 7, 2, seed=3)
    return {"lp_small": lp, "ragged": ragged, "dense_and_empty": edge, "tiny": tiny}


CASES = _cases()


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("check_every", [10, 7])
def test_resident_matches_oracle(name, check_every):
    inst = CASES[name]
    say(f"resident {name}: m={inst['m']} n={inst['n']} nnz={inst['nnz']} check_every={check_every}")
    orc = oracle.Oracle.from_instance(inst, mu=0.8)
    orc.iterate(200)
    o, ro = orc.state(), orc.residuals()
    with Solver.from_instance(inst, mu=0.8, eps=0.0, check_every=check_every, resident="required") as s:
        assert s.launch_shape()["resident"]
        s.iterate(200)
        g, r = s.solution(), s.residuals()
    errs = {k: rel(g[k], o[k]) for k in KEYS}
    say(f"resident {name} rel errors {errs}")
    for k in KEYS:
        assert errs[k] <= 1e-9, (k, errs[k])
    assert r["iter"] == 200
    for k in RES:
        assert abs(r[k] - ro[k]) <= 1e-9 * max(abs(ro[k]), 1e-12), (k, r[k], ro[k])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_resident_and_sweep_kernels_stop_at_the_same_check(precision):
    inst = CASES["lp_small"]
    out = {}
    for path in ("required", "never"):
        with Solver.from_instance(inst, eps=1e-4, precision=precision, resident=path) as s:
            assert s.launch_shape()["resident"] == (path == "required")
            assert s.iterate(60_000)
            out[path] = (s.residuals(), s.solution())
    ra, rb = out["required"][0], out["never"][0]
    say(f"{precision}: resident stops at {ra['iter']}, sweep kernels at {rb['iter']}")
    assert ra["status"] == rb["status"] == "converged"
    assert ra["iter"] == rb["iter"]
    tol = 1e-9 if precision == "fp64" else 1e-4
    for k in KEYS:
        assert rel(out["required"][1][k], out["never"][1][k]) <= tol, k


def test_resident_pieces_equal_one_call():
    """Iterating in pieces of 7 (residual queries between the pieces)
    gives bitwise the iterates of one call."""
    inst = CASES["ragged"]
    with Solver.from_instance(inst, eps=0.0, check_every=10) as a:
        assert a.launch_shape()["resident"]
        a.iterate(203)
        sa, ra = a.solution(), a.residuals()
    with Solver.from_instance(inst, eps=0.0, check_every=10) as b:
        for _ in range(29):
            b.iterate(7)
            b.residuals()
        sb, rb = b.solution(), b.residuals()
    for k in KEYS:
        assert np.array_equal(sa[k], sb[k]), k
    assert ra["iter"] == rb["iter"] == 203


def test_resident_resume_matches_oracle():
    inst = CASES["ragged"]
    rng = np.random.default_rng(5)
    st = (rng.standard_normal(inst["n"]), rng.standard_normal(inst["n"]), rng.standard_normal(inst["n"]),
          rng.standard_normal(inst["m"]))
    orc = oracle.Oracle.from_instance(inst, mu=0.9)
    orc.resume(*st)
    orc.iterate(150)
    with Solver.from_instance(inst, mu=0.9, eps=0.0, resident="required") as s:
        s.resume(*st)
        s.iterate(150)
        g = s.solution()
    o = orc.state()
    for k in KEYS:
        assert rel(g[k], o[k]) <= 1e-9, k


def test_resident_max_iter_and_numeric_stop():
    inst = CASES["ragged"]
    with Solver.from_instance(inst, eps=1e-12, max_iter=25, resident="required") as s:
        assert s.iterate(1000)
        r = s.residuals()
    assert r["status"] == "max_iter" and r["iter"] == 25
    c = inst["c"].copy()
    c[3] = np.nan
    with Solver.from_instance(dict(inst, c=c), eps=1e-4, check_every=10, resident="required") as s:
        s.iterate(500)
        r = s.residuals()
    assert r["status"] == "numeric" and r["iter"] == 10


def test_resident_rejects_what_does_not_fit():
    big = I.lp_instance(5000, 10_000, 6, seed=1)       # beyond one CU's LDS
    with pytest.raises(Exception):
        Solver.from_instance(big, resident="required")
    soc = I.socp_instance(20, 4, seed=2)               # second-order cones
    with pytest.raises(Exception):
        Solver.from_instance(soc, resident="required")
    with Solver.from_instance(big) as s:
        assert not s.launch_shape()["resident"]


def test_largest_resident_problem():
    """A problem just inside the LDS budget (FP64: 32 bytes per row and
    column plus 20 per entry) still runs resident and matches the oracle."""
    inst = I.lp_instance(585, 1170, 5, seed=41)          # 161,520 of the 161,792 bytes
    orc = oracle.Oracle.from_instance(inst)
    orc.iterate(100)
    with Solver.from_instance(inst, eps=0.0, resident="required") as s:
        s.iterate(100)
        g = s.solution()
    o = orc.state()
    for k in KEYS:
        assert rel(g[k], o[k]) <= 1e-9, k


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_one_call_solve_equals_the_handle_calls(precision):
    """solver_solve gives what create, iterate, solution and residuals give
    (bitwise), on the resident path and on the sweep kernels."""
    from paper_2203_05027_amd.solver import solve
    for inst, kw in ((CASES["lp_small"], {}), (I.socp_instance(30, 4, seed=3), {})):
        rc, sol, res = solve(inst, 1234, precision=precision, eps=1e-4, **kw)
        assert rc == 0
        with Solver.from_instance(inst, precision=precision, eps=1e-4, **kw) as s:
            s.iterate(1234)
            g, r = s.solution(), s.residuals()
        for k in KEYS:
            assert np.array_equal(sol[k], g[k]), k
        assert res == r
