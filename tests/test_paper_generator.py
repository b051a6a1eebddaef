"""The experiments' own generator (Section V, "Problem instances"): feasible
by construction, and -- unlike what the section states -- not bounded in
general, because c ~ N(0, I) is drawn without regard to A.  These CPU tests
show both on small instances of every density the section lists, with
scipy's LP solver (HiGHS) as the independent judge:

* feasibility: proj_K(xdot) satisfies A x = b and x in K exactly;
* LP: the solver reports the problem unbounded;
* SOCP with K = (K_4)^(n/4): a recession direction d with A d = 0, d in K
  and c'd < 0 exists (found by an LP over the polyhedral part
  |u_i| <= t / sqrt(3) of each cone, which lies inside it), so
  x + s d stays feasible while c'(x + s d) -> -inf.

This is why the single-instance workloads use the complementary
constructions (bounded with a known optimum) and the generator itself is
used for the sweep rate only."""
import numpy as np
import pytest
from scipy.optimize import linprog
from scipy.sparse import csr_matrix

from paper_2203_05027_amd import instances as I


def _dense(inst):
    return csr_matrix((inst["val"], inst["col_idx"], inst["row_ptr"]), shape=(inst["m"], inst["n"]))


@pytest.mark.parametrize("density", [0.001, 0.005, 0.01])
@pytest.mark.parametrize("cone", ["lp", "socp"])
def test_generator_is_feasible_by_construction(density, cone):
    inst = I.paper_instance(400, 2000, density, cone, seed=11)
    A = _dense(inst)
    x = inst["x_feasible"]
    assert np.allclose(A @ x, inst["b"], rtol=0, atol=1e-12)
    if cone == "lp":
        assert (x >= 0).all()
    else:
        w = x.reshape(-1, 4)
        assert (np.linalg.norm(w[:, 1:], axis=1) <= w[:, 0] * (1 + 1e-12) + 1e-15).all()
    nnz = inst["nnz"]
    assert nnz == round(density * 400 * 2000)


@pytest.mark.parametrize("density", [0.001, 0.005, 0.01])
def test_lp_generator_is_unbounded(density):
    inst = I.paper_instance(200, 1000, density, "lp", seed=12)
    A = _dense(inst)
    res = linprog(inst["c"], A_eq=A, b_eq=inst["b"], bounds=(0, None), method="highs")
    assert res.status == 3, res.message   # 3: the problem is unbounded


@pytest.mark.parametrize("density", [0.001, 0.005, 0.01])
def test_socp_generator_has_a_descent_ray(density):
    inst = I.paper_instance(200, 1000, density, "socp", seed=13)
    A = _dense(inst)
    n = inst["n"]
    q = n // 4
    # d = (t_1, u_1, ..., t_q, u_q): A d = 0, 0 <= t <= 1, -t/sqrt(3) <= u_i <= t/sqrt(3)
    rows, rhs = [], []
    s3 = 1 / np.sqrt(3.0)
    for k in range(q):
        for i in range(1, 4):
            for sign in (1.0, -1.0):
                r = np.zeros(n)
                r[4 * k + i] = sign
                r[4 * k] = -s3
                rows.append(r)
                rhs.append(0.0)
    bounds = [(0, 1) if j % 4 == 0 else (None, None) for j in range(n)]
    res = linprog(inst["c"], A_ub=np.array(rows), b_ub=np.array(rhs), A_eq=A, b_eq=np.zeros(inst["m"]),
                  bounds=bounds, method="highs")
    assert res.status == 0, res.message
    d = res.x
    assert inst["c"] @ d < -1e-6
    assert np.abs(A @ d).max() <= 1e-9
    w = d.reshape(-1, 4)
    assert (np.linalg.norm(w[:, 1:], axis=1) <= w[:, 0] + 1e-9).all()
