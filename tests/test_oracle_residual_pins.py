"""Pins of the oracle's residuals (the stopping test of Section V-B) on states
that are NOT optimal, where every residual is non-zero and its value is fixed
by hand or in closed form:

* Example 1's matrix (Section IV) with small integer data and state, every
  residual worked out by hand below (exact surds and fractions);
* the generator's known optimum (x0, lambda = -y0, delta = s0) moved along one
  coordinate: exactly one residual becomes non-zero, with a closed-form value
  (a column norm, a row norm, the moved amount);
* the zero state, where the primal and dual residuals reduce to
  ||b|| / (1 + ||b||) and ||c|| / (1 + ||c||) and the gap to 0;
* dense products of random states (the definitions written with dense A).

The readings taken of the printed test: the dual residual subtracts delta (x
is cone-constrained), the gap takes an absolute value, and the residuals are
evaluated at z (in K) with lambda and delta:
  r_prim = ||A z - b|| / (1 + ||b||),  r_dual = ||A'lambda + c - delta|| / (1 + ||c||)
  r_gap  = |c'z + b'lambda| / (1 + |c'z| + |b'lambda|),  kkt = max of the three.
"""
import json
import os
from math import sqrt

import numpy as np
import pytest

from paper_2203_05027_amd import instances as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _example1_oracle(oracle_mod, b, c):
    A = np.array(json.load(open(os.path.join(GOLDEN, "example1.json")))["A"], float)
    rr, cc = np.nonzero(A)
    row_ptr = np.zeros(4, np.int64)
    np.cumsum(np.bincount(rr, minlength=3), out=row_ptr[1:])
    return oracle_mod.Oracle(3, 5, row_ptr, cc.astype(np.int32), A[rr, cc], b, c, 5, ())


def test_example1_hand_residuals(oracle_mod):
    """A = [[1,0,4,6,8],[0,0,5,0,0],[2,3,0,7,0]] (Example 1), b = (2,1,2)
    (||b|| = 3), c = (1,2,2,0,4) (||c|| = 5), and the state
    x = (1,1,0,0,0), z = (1,0,0,0,0), lambda = (-1,-1,0), delta = (0,1,0,2,0).
    By hand:
      A z = column 1 = (1,0,2);  A z - b = (-1,-1,0)          -> sqrt(2)
      A'lambda = -(row 1) - (row 2) = (-1,0,-9,-6,-8)
      A'lambda + c - delta = (0,1,-7,-8,-4)                   -> sqrt(130)
      c'z = 1,  b'lambda = -2 - 1 + 0 = -3                     -> gap |1 - 3| / (1 + 1 + 3)
      A x = columns 1 + 2 = (1,0,5);  A x - b = (-1,-1,3)     -> sqrt(11)
      x - z = (0,1,0,0,0)                                     -> 1
      ||Az||_inf = 2, ||b||_inf = 2, ||A'lambda||_inf = 9, ||c||_inf = 4
      c'x = 1 + 2 = 3 (the objective at x of the POGS-form gap)."""
    orc = _example1_oracle(oracle_mod, [2.0, 1.0, 2.0], [1.0, 2.0, 2.0, 0.0, 4.0])
    orc.set_state(x=[1, 1, 0, 0, 0], z=[1, 0, 0, 0, 0], delta=[0, 1, 0, 2, 0], lam=[-1, -1, 0])
    r = orc.residuals()
    want = {
        "r_prim": sqrt(2) / 4, "r_dual": sqrt(130) / 6, "r_gap": 2 / 5, "kkt": sqrt(130) / 6,
        "pobj": 1.0, "dobj": 3.0, "res_ax_b": sqrt(11), "res_x_z": 1.0,
        "prim_inf": 1.0, "dual_inf": 8.0, "scale_p": 2.0, "scale_d": 9.0, "pobj_x": 3.0,
    }
    for k, v in want.items():
        assert r[k] == pytest.approx(v, rel=1e-14, abs=1e-15), (k, r[k], v)


def test_example1_gap_dominates(oracle_mod):
    """A state with A z = b and A'lambda + c - delta = 0 exactly but a
    non-zero gap, so kkt is the gap: z = e_1, b = A e_1 = (1,0,2),
    lambda = (1,0,0) (b'lambda = 1), c = (1,2,2,0,4) (c'z = 1),
    delta = A'lambda + c = row 1 + c = (2,2,6,6,12):
    r_gap = |1 + 1| / (1 + 1 + 1) = 2/3."""
    orc = _example1_oracle(oracle_mod, [1.0, 0.0, 2.0], [1.0, 2.0, 2.0, 0.0, 4.0])
    orc.set_state(x=[1, 0, 0, 0, 0], z=[1, 0, 0, 0, 0], delta=[2, 2, 6, 6, 12], lam=[1, 0, 0])
    r = orc.residuals()
    assert r["r_prim"] == 0.0 and r["r_dual"] == 0.0
    assert r["r_gap"] == pytest.approx(2 / 3, rel=1e-15)
    assert r["kkt"] == pytest.approx(2 / 3, rel=1e-15)


@pytest.mark.parametrize("seed", [3, 8])
def test_zero_state_closed_forms(oracle_mod, seed):
    """At x = z = delta = 0, lambda = 0: r_prim = ||b|| / (1 + ||b||),
    r_dual = ||c|| / (1 + ||c||), r_gap = 0, res_ax_b = ||b||."""
    inst = I.lp_instance(40, 90, 4, seed=seed)
    orc = oracle_mod.Oracle.from_instance(inst)
    r = orc.residuals()
    nb, nc = np.linalg.norm(inst["b"]), np.linalg.norm(inst["c"])
    assert r["r_prim"] == pytest.approx(nb / (1 + nb), rel=1e-13)
    assert r["r_dual"] == pytest.approx(nc / (1 + nc), rel=1e-13)
    assert r["r_gap"] == 0.0
    assert r["kkt"] == pytest.approx(max(nb / (1 + nb), nc / (1 + nc)), rel=1e-13)
    assert r["res_ax_b"] == pytest.approx(nb, rel=1e-13)
    assert r["res_x_z"] == 0.0


def _column(inst, j):
    rows = np.repeat(np.arange(inst["m"]), np.diff(inst["row_ptr"]))
    sel = inst["col_idx"] == j
    col = np.zeros(inst["m"])
    col[rows[sel]] = inst["val"][sel]
    return col


@pytest.mark.parametrize("t", [0.5, -2.0])
def test_moves_from_the_optimum(oracle_mod, t):
    """The generator's optimum (x0, lambda = -y0, delta = s0) has A x0 = b,
    A'(-y0) + c - s0 = 0 and c'x0 = b'y0.  Moving one coordinate by t:
    * z = x0 + t e_j: A z - b = t A e_j, only r_prim and r_gap move:
      r_prim = |t| ||A e_j|| / (1 + ||b||), r_gap = |t c_j| / (1 + |c'z| + |b'lambda|);
    * delta = s0 + t e_j: only r_dual moves, to |t| / (1 + ||c||);
    * lambda = -y0 + t e_i: A'lambda + c - delta = t A' e_i, gap t b_i:
      r_dual = |t| ||row i|| / (1 + ||c||), r_gap = |t b_i| / (1 + |c'z| + |b'lambda|);
    * x = x0 + t e_j (z kept): res_ax_b = |t| ||A e_j||, res_x_z = |t|."""
    inst = I.lp_instance(30, 70, 4, seed=11)
    x0, y0, s0, b, c = inst["x0"], inst["y0"], inst["s0"], inst["b"], inst["c"]
    nb, nc = np.linalg.norm(b), np.linalg.norm(c)
    orc = oracle_mod.Oracle.from_instance(inst)
    j, i = 5, 7
    aj = _column(inst, j)
    row_i = np.zeros(inst["n"])
    k0, k1 = inst["row_ptr"][i], inst["row_ptr"][i + 1]
    row_i[inst["col_idx"][k0:k1]] = inst["val"][k0:k1]
    tol = dict(rel=1e-11, abs=1e-13)

    z = x0.copy(); z[j] += t
    orc.set_state(x=x0, z=z, delta=s0, lam=-y0)
    r = orc.residuals()
    cz, bl = c @ z, -(b @ y0)
    assert r["r_prim"] == pytest.approx(abs(t) * np.linalg.norm(aj) / (1 + nb), **tol)
    assert r["r_dual"] == pytest.approx(0.0, abs=1e-13)
    assert r["r_gap"] == pytest.approx(abs(t * c[j]) / (1 + abs(cz) + abs(bl)), **tol)

    d = s0.copy(); d[j] += t
    orc.set_state(x=x0, z=x0, delta=d, lam=-y0)
    r = orc.residuals()
    assert r["r_prim"] == pytest.approx(0.0, abs=1e-13)
    assert r["r_dual"] == pytest.approx(abs(t) / (1 + nc), **tol)
    assert r["r_gap"] == pytest.approx(0.0, abs=1e-13)

    lam = -y0.copy(); lam[i] += t
    orc.set_state(x=x0, z=x0, delta=s0, lam=lam)
    r = orc.residuals()
    cz, bl = c @ x0, b @ lam
    assert r["r_dual"] == pytest.approx(abs(t) * np.linalg.norm(row_i) / (1 + nc), **tol)
    assert r["r_gap"] == pytest.approx(abs(t * b[i]) / (1 + abs(cz) + abs(bl)), **tol)
    assert r["dobj"] == pytest.approx(-bl, **tol)
    assert r["kkt"] == pytest.approx(max(r["r_prim"], r["r_dual"], r["r_gap"]), rel=0, abs=0)

    x = x0.copy(); x[j] += t
    orc.set_state(x=x, z=x0, delta=s0, lam=-y0)
    r = orc.residuals()
    assert r["res_ax_b"] == pytest.approx(abs(t) * np.linalg.norm(aj), **tol)
    assert r["res_x_z"] == pytest.approx(abs(t), **tol)
    assert r["kkt"] == pytest.approx(0.0, abs=1e-13)


@pytest.mark.parametrize("kind", ["lp", "socp"])
def test_random_states_against_dense_products(oracle_mod, kind):
    """Every residual on random (non-optimal) states against the definitions
    written with a dense A."""
    inst = I.lp_instance(25, 60, 3, seed=2) if kind == "lp" else I.socp_instance(9, 3, seed=6)
    m, n = inst["m"], inst["n"]
    A = np.zeros((m, n))
    rows = np.repeat(np.arange(m), np.diff(inst["row_ptr"]))
    A[rows, inst["col_idx"]] = inst["val"]
    b, c = inst["b"], inst["c"]
    orc = oracle_mod.Oracle.from_instance(inst)
    rng = np.random.default_rng(4)
    for _ in range(5):
        x, z, d = (rng.standard_normal(n) * 2 for _ in range(3))
        lam = rng.standard_normal(m) * 3
        orc.set_state(x=x, z=z, delta=d, lam=lam)
        r = orc.residuals()
        rp = np.linalg.norm(A @ z - b) / (1 + np.linalg.norm(b))
        rd = np.linalg.norm(A.T @ lam + c - d) / (1 + np.linalg.norm(c))
        rg = abs(c @ z + b @ lam) / (1 + abs(c @ z) + abs(b @ lam))
        want = dict(r_prim=rp, r_dual=rd, r_gap=rg, kkt=max(rp, rd, rg), pobj=c @ z, dobj=-(b @ lam),
                    res_ax_b=np.linalg.norm(A @ x - b), res_x_z=np.linalg.norm(x - z), pobj_x=c @ x)
        for k, v in want.items():
            assert r[k] == pytest.approx(v, rel=1e-12), k
