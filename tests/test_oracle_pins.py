"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself:
* the UV decomposition printed in Example 1 (Section IV) -> tests/golden;
* the projection onto Lorentz cones (eq. proj) against its textbook special
  case (size-1 cone = max(w, 0)), hand-computed values and Moreau's
  characterisation, which determines a projection onto a closed convex cone
  uniquely;
* the closed-form x- and y-steps of Block 1 / Block 2 against a numerical
  minimisation of the augmented Lagrangian (eq. lll) built from dense U, V;
* invariants every ADMM iterate must satisfy, the fixed point at a known
  optimum, brute-force vertex enumeration on tiny LPs and closed-form optima
  of tiny SOCPs.
"""
import itertools
import json
import os

import numpy as np
import pytest
import torch

from paper_2203_05027_amd import instances as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dense(inst):
    A = np.zeros((inst["m"], inst["n"]))
    rp = inst["row_ptr"]
    for i in range(inst["m"]):
        for k in range(rp[i], rp[i + 1]):
            A[i, inst["col_idx"][k]] = inst["val"][k]
    return A


def _csr_from_dense(A):
    m, n = A.shape
    row_ptr = [0]
    cols, vals = [], []
    for i in range(m):
        for j in range(n):
            if A[i, j] != 0:
                cols.append(j)
                vals.append(A[i, j])
        row_ptr.append(len(cols))
    return (np.array(row_ptr, np.int64), np.array(cols, np.int32), np.array(vals, float))


def _in_cone(v, n_orth, sizes, tol):
    if n_orth and v[:n_orth].min() < -tol:
        return False
    off = n_orth
    for s in sizes:
        blk = v[off:off + s]
        if blk[0] + tol < np.linalg.norm(blk[1:]):
            return False
        off += s
    return True


# --------------------------------------------------------------------------
# Example 1 (Section IV)
# --------------------------------------------------------------------------
def test_example1_uv_matches_printed(oracle_mod):
    g = json.load(open(os.path.join(GOLDEN, "example1.json")))
    A, U_p, V_p = (np.array(g[k], float) for k in ("A", "U", "V"))
    # nonzeros in the order the example numbers them: column by column
    nz = [(i, j, A[i, j]) for j in range(A.shape[1]) for i in range(A.shape[0]) if A[i, j] != 0]
    rows, cols, vals = zip(*nz)
    U, V = oracle_mod.uv_dense(3, 5, rows, cols, vals)
    np.testing.assert_array_equal(U, U_p)
    np.testing.assert_array_equal(V, V_p)
    np.testing.assert_array_equal(U @ V.T, A)
    for M in (U @ U.T, V @ V.T):
        np.testing.assert_array_equal(M, np.diag(np.diag(M)))


def test_example1_factors_from_printed_uv(oracle_mod):
    """The set-up of Algorithm 1 on Example 1: F_U, F_V are the inverses of
    I + UU' and I + VV' formed from the printed U and V."""
    g = json.load(open(os.path.join(GOLDEN, "example1.json")))
    A, U_p, V_p = (np.array(g[k], float) for k in ("A", "U", "V"))
    rp, ci, va = _csr_from_dense(A)
    o = oracle_mod.Oracle(3, 5, rp, ci, va, np.zeros(3), np.zeros(5), 5, mu=1.0)
    FU, FV = o.diagonals()
    np.testing.assert_allclose(np.diag(FU), np.linalg.inv(np.eye(3) + U_p @ U_p.T), rtol=1e-15)
    np.testing.assert_allclose(np.diag(FV), np.linalg.inv(np.eye(5) + V_p @ V_p.T), rtol=1e-15)
    # the values written out: diag(UU') = (117, 25, 62), diag(VV') = (2,1,2,2,1)
    np.testing.assert_allclose(FU, [1 / 118, 1 / 26, 1 / 63], rtol=1e-15)
    np.testing.assert_allclose(FV, [1 / 3, 1 / 2, 1 / 3, 1 / 3, 1 / 2], rtol=1e-15)


def test_matrix_inversion_lemma_example1():
    """(I + U'U)^{-1} = I - U'(I + UU')^{-1}U on Example 1 (Block 2)."""
    g = json.load(open(os.path.join(GOLDEN, "example1.json")))
    U = np.array(g["U"], float)
    lhs = np.linalg.inv(np.eye(8) + U.T @ U)
    rhs = np.eye(8) - U.T @ np.linalg.inv(np.eye(3) + U @ U.T) @ U
    np.testing.assert_allclose(lhs, rhs, atol=1e-14)


# --------------------------------------------------------------------------
# Projection (eq. proj)
# --------------------------------------------------------------------------
def test_projection_size1_is_relu(oracle_mod):
    w = np.random.default_rng(1).standard_normal(1000)
    w[:5] = [0.0, -0.0, 1e-300, -1e-300, 3.0]
    np.testing.assert_array_equal(oracle_mod.project(w, 1000), np.maximum(w, 0.0))
    # a size-1 Lorentz cone listed as a second-order block behaves the same
    np.testing.assert_array_equal(oracle_mod.project(w[:7], 0, [1] * 7), np.maximum(w[:7], 0.0))


def test_projection_hand_values(oracle_mod):
    # alpha = 2 > |w1| = 1: (w/2) + (alpha/2, w1 w2/(2 alpha), w1 w3/(2 alpha))
    np.testing.assert_allclose(oracle_mod.project([1.0, 2.0, 0.0], 0, [3]), [1.5, 1.5, 0.0])
    np.testing.assert_allclose(oracle_mod.project([-1.0, 2.0, 0.0], 0, [3]), [0.5, 0.5, 0.0])
    np.testing.assert_array_equal(oracle_mod.project([-3.0, 1.0, 1.0], 0, [3]), [0, 0, 0])
    np.testing.assert_array_equal(oracle_mod.project([3.0, 1.0, 1.0], 0, [3]), [3, 1, 1])
    # 3-4-5: (0, 3, 4) -> alpha = 5, result (2.5, 1.5, 2.0), on the boundary
    np.testing.assert_allclose(oracle_mod.project([0.0, 3.0, 4.0], 0, [3]), [2.5, 1.5, 2.0])
    # ties: alpha = -w1 and alpha = w1 (continuous there) and alpha = w1 = 0
    np.testing.assert_array_equal(oracle_mod.project([-5.0, 3.0, 4.0], 0, [3]), [0, 0, 0])
    np.testing.assert_array_equal(oracle_mod.project([5.0, 3.0, 4.0], 0, [3]), [5, 3, 4])
    np.testing.assert_array_equal(oracle_mod.project([0.0, 0.0, 0.0], 0, [3]), [0, 0, 0])


@pytest.mark.parametrize("seed", range(4))
def test_projection_moreau_characterisation(oracle_mod, seed):
    """P(w) in K, P(-w) in K, w = P(w) - P(-w), P(w)'P(-w) = 0 per cone
    (Moreau; K is self-dual), which pins P uniquely; plus idempotence and the
    variational inequality against random points of K."""
    rng = np.random.default_rng(seed)
    n_orth = 37
    sizes = rng.integers(2, 51, size=40).astype(np.int32)
    n = n_orth + int(sizes.sum())
    w = rng.standard_normal(n) * rng.choice([0.1, 1.0, 10.0], size=n)
    p, q = oracle_mod.project(w, n_orth, sizes), oracle_mod.project(-w, n_orth, sizes)
    assert _in_cone(p, n_orth, sizes, 1e-12) and _in_cone(q, n_orth, sizes, 1e-12)
    np.testing.assert_allclose(p - q, w, atol=1e-12)
    off = 0
    for s in [1] * n_orth + list(sizes):
        assert abs(p[off:off + s] @ q[off:off + s]) <= 1e-12 * (1 + np.abs(w[off:off + s]).sum() ** 2)
        off += s
    np.testing.assert_allclose(oracle_mod.project(p, n_orth, sizes), p, atol=1e-13)
    for _ in range(20):
        v = oracle_mod.project(rng.standard_normal(n) * 3, n_orth, sizes)
        assert (w - p) @ (v - p) <= 1e-10
        assert np.linalg.norm(w - p) <= np.linalg.norm(w - v) + 1e-12


# --------------------------------------------------------------------------
# Closed-form steps vs minimising the augmented Lagrangian (eq. lll)
# --------------------------------------------------------------------------
def _lagrangian(U, V, b, c, mu):
    Ut, Vt, bt, ct = (torch.tensor(a, dtype=torch.float64) for a in (U, V, b, c))

    def L(x, y, z, lam, gam, dlt):
        r1 = Ut @ y - bt
        r2 = y - Vt.T @ x
        r3 = z - x
        return (ct @ x + lam @ r1 + mu / 2 * (r1 @ r1) + gam @ r2 + mu / 2 * (r2 @ r2)
                + dlt @ r3 + mu / 2 * (r3 @ r3))
    return L


def _argmin_quadratic(f, dim):
    """Exact minimiser of a strictly convex quadratic f: R^dim -> R."""
    z0 = torch.zeros(dim, dtype=torch.float64)
    g = torch.autograd.functional.jacobian(f, z0)
    H = torch.autograd.functional.hessian(f, z0)
    return torch.linalg.solve(H, -g).numpy()


@pytest.mark.parametrize("case", ["example1", "random"])
def test_closed_form_steps_minimise_lagrangian(oracle_mod, case):
    rng = np.random.default_rng(11)
    if case == "example1":
        g = json.load(open(os.path.join(GOLDEN, "example1.json")))
        A = np.array(g["A"], float)
        n_orth, sizes = 2, [3]
    else:
        inst = I.lp_instance(6, 10, 2, seed=5)
        A = _dense(inst)
        n_orth, sizes = 4, [2, 4]
    m, n = A.shape
    rp, ci, va = _csr_from_dense(A)
    # U, V straight from their definitions with nonzeros in CSR order
    nzr = np.repeat(np.arange(m), np.diff(rp))
    o = len(va)
    U = np.zeros((m, o)); U[nzr, np.arange(o)] = va
    V = np.zeros((n, o)); V[ci, np.arange(o)] = 1.0
    b, c = rng.standard_normal(m), rng.standard_normal(n)
    mu = 0.7
    st = {k: rng.standard_normal(d) for k, d in
          (("x", n), ("z", n), ("delta", n), ("y", o), ("gamma", o), ("lam", m))}
    orc = oracle_mod.Oracle(m, n, rp, ci, va, b, c, n_orth, sizes, mu=mu)
    orc.set_state(st["x"], st["z"], st["delta"], st["y"], st["gamma"], st["lam"])
    orc.iterate(1)
    out = orc.state()

    L = _lagrangian(U, V, b, c, mu)
    T = {k: torch.tensor(v) for k, v in st.items()}
    x1 = _argmin_quadratic(lambda x: L(x, T["y"], T["z"], T["lam"], T["gamma"], T["delta"]), n)
    np.testing.assert_allclose(out["x"], x1, rtol=1e-10, atol=1e-12)
    x1t = torch.tensor(x1)
    y1 = _argmin_quadratic(lambda y: L(x1t, y, T["z"], T["lam"], T["gamma"], T["delta"]), o)
    np.testing.assert_allclose(out["y"], y1, rtol=1e-10, atol=1e-12)
    # z-step: argmin over z in K of L = projection of w = x1 - delta/mu;
    # checked through Moreau's characterisation (z in K, z - w in K, orthogonal)
    w = x1 - st["delta"] / mu
    z1 = out["z"]
    assert _in_cone(z1, n_orth, sizes, 1e-12) and _in_cone(z1 - w, n_orth, sizes, 1e-12)
    assert abs(z1 @ (z1 - w)) < 1e-11
    # dual ascent with step mu on each constraint residual
    np.testing.assert_allclose(out["lambda"], st["lam"] + mu * (U @ y1 - b), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(out["gamma"], st["gamma"] + mu * (y1 - V.T @ x1), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(out["delta"], st["delta"] + mu * (z1 - x1), rtol=1e-10, atol=1e-12)


# --------------------------------------------------------------------------
# Invariants of the iterates
# --------------------------------------------------------------------------
@pytest.mark.parametrize("kind", ["lp", "socp"])
def test_iterate_invariants(oracle_mod, kind):
    """After every iteration: gamma = -U'lambda (optimality of the y-step plus
    the two dual updates), z in K, delta in K* = K, z'delta = 0 (Moreau on the
    z-step), and, once gamma = -U'lambda holds on entry, U y - b = F_U (A x - b)."""
    if kind == "lp":
        inst = I.lp_instance(50, 100, 5, seed=3)
    else:
        inst = I.socp_instance(12, 4, seed=3)
    A = _dense(inst)
    orc = oracle_mod.Oracle.from_instance(inst, mu=0.8)
    FU, _ = orc.diagonals()
    rp = inst["row_ptr"]
    nzr = np.repeat(np.arange(inst["m"]), np.diff(rp))
    a = inst["val"]
    rng = np.random.default_rng(0)
    orc.set_state(*(rng.standard_normal(d) for d in
                    (inst["n"], inst["n"], inst["n"], inst["nnz"], inst["nnz"], inst["m"])))
    for it in range(6):
        orc.iterate(1)
        s = orc.state()
        scale = 1 + np.abs(s["lambda"]).max()
        np.testing.assert_allclose(s["gamma"], -a * s["lambda"][nzr], atol=1e-12 * scale)
        assert _in_cone(s["z"], inst["n_orth"], inst["soc_sizes"], 1e-12)
        assert _in_cone(s["delta"], inst["n_orth"], inst["soc_sizes"], 1e-12)
        assert abs(s["z"] @ s["delta"]) <= 1e-10 * (1 + np.abs(s["z"]).sum() * np.abs(s["delta"]).max())
        if it >= 1:  # needs gamma = -U'lambda on entry, true from the 2nd iteration
            Uy = np.bincount(nzr, weights=a * s["y"], minlength=inst["m"])
            np.testing.assert_allclose(Uy - inst["b"], FU * (A @ s["x"] - inst["b"]),
                                       atol=1e-11 * scale)


def test_resume_continues_the_literal_run(oracle_mod):
    """The full Algorithm 1 state at the end of an iteration is fixed by
    (x, z, delta, lambda): resuming from those four continues the run that
    kept y and gamma."""
    inst = I.socp_instance(15, 4, seed=4)
    a = oracle_mod.Oracle.from_instance(inst, mu=0.6)
    a.iterate(30)
    s = a.state()
    b = oracle_mod.Oracle.from_instance(inst, mu=0.6)
    b.resume(s["x"], s["z"], s["delta"], s["lambda"])
    sb = b.state()
    np.testing.assert_allclose(sb["y"], s["y"], atol=1e-12 * (1 + np.abs(s["y"]).max()))
    np.testing.assert_allclose(sb["gamma"], s["gamma"], atol=1e-12 * (1 + np.abs(s["gamma"]).max()))
    a.iterate(40)
    b.iterate(40)
    for k in ("x", "z", "delta", "lambda"):
        np.testing.assert_allclose(b.state()[k], a.state()[k], atol=1e-11)


@pytest.mark.parametrize("mu", [0.37, 1.0, 4.0])
def test_fixed_point_at_known_optimum(oracle_mod, mu):
    """At a primal-dual optimum (x0, lambda = -y0, delta = s0) every vector
    is left unchanged by an iteration, for any mu."""
    inst = I.lp_instance(60, 120, 4, seed=7)
    orc = oracle_mod.Oracle.from_instance(inst, mu=mu)
    orc.set_start(inst["x0"], inst["x0"], inst["s0"], -inst["y0"])
    s0 = orc.state()
    orc.iterate(5)
    s1 = orc.state()
    for k in ("x", "z", "delta", "lambda", "y", "gamma"):
        np.testing.assert_allclose(s1[k], s0[k], atol=1e-12 * (1 + np.abs(s0[k]).max()))
    r = orc.residuals()
    assert r["kkt"] < 1e-13
    # infinity-norm measures at the optimum: both residuals vanish, and the
    # scales are the larger of the data and product norms
    assert r["prim_inf"] < 1e-12 and r["dual_inf"] < 1e-12
    A = _dense(inst)
    assert r["scale_p"] == pytest.approx(np.abs(inst["b"]).max(), rel=1e-12)
    atl = A.T @ (-inst["y0"])
    assert r["scale_d"] == pytest.approx(max(np.abs(atl).max(), np.abs(inst["c"]).max()), rel=1e-12)


# --------------------------------------------------------------------------
# Optima
# --------------------------------------------------------------------------
def _brute_force_lp(A, b, c):
    """Minimum of c'x over the vertices of {Ax = b, x >= 0} (A full row rank)."""
    m, n = A.shape
    best = np.inf
    for B in itertools.combinations(range(n), m):
        AB = A[:, B]
        if abs(np.linalg.det(AB)) < 1e-12:
            continue
        xB = np.linalg.solve(AB, b)
        if xB.min() < -1e-12:
            continue
        best = min(best, float(c[list(B)] @ xB))
    return best


@pytest.mark.parametrize("seed", [21, 22, 23, 24, 25])
def test_tiny_lp_against_vertex_enumeration(oracle_mod, seed):
    inst = I.lp_instance(3, 7, 2, seed=seed)
    A = _dense(inst)
    assert np.linalg.matrix_rank(A) == 3
    p_star = _brute_force_lp(A, inst["b"], inst["c"])
    assert abs(p_star - inst["p_star"]) <= 1e-9 * (1 + abs(p_star))
    orc = oracle_mod.Oracle.from_instance(inst, mu=1.0)
    r = orc.solve(1e-9, check_every=10, max_iter=400_000)
    assert r["kkt"] <= 1e-9
    assert abs(r["pobj"] - p_star) <= 1e-6 * (1 + abs(p_star))
    assert abs(r["dobj"] - p_star) <= 1e-6 * (1 + abs(p_star))


def test_tiny_lp_non_generator(oracle_mod):
    """A hand-written LP: min -x1 - 2x2, x1 + x2 + s1 = 4, x1 + 3x2 + s2 = 6,
    x >= 0.  Vertex enumeration and the textbook answer (x1, x2) = (3, 1):
    value -5."""
    A = np.array([[1.0, 1.0, 1.0, 0.0], [1.0, 3.0, 0.0, 1.0]])
    b = np.array([4.0, 6.0])
    c = np.array([-1.0, -2.0, 0.0, 0.0])
    assert _brute_force_lp(A, b, c) == pytest.approx(-5.0, abs=1e-12)
    orc = oracle_mod.Oracle(2, 4, *_csr_from_dense(A), b, c, 4, mu=1.0)
    r = orc.solve(1e-10, max_iter=200_000)
    np.testing.assert_allclose(orc.state()["z"], [3, 1, 0, 0], atol=1e-7)
    assert r["pobj"] == pytest.approx(-5.0, abs=1e-7)


@pytest.mark.parametrize("u,expect", [((1.0, 2.0), np.sqrt(5.0)), ((3.0, 4.0), 5.0),
                                      ((0.0, 0.0), 0.0)])
def test_tiny_socp_closed_form(oracle_mod, u, expect):
    """min t s.t. (t, u1, u2) in K_3 with u fixed: the optimum is ||u||."""
    A = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    orc = oracle_mod.Oracle(2, 3, *_csr_from_dense(A), np.array(u), np.array([1.0, 0, 0]),
                            0, [3], mu=1.0)
    r = orc.solve(1e-10, max_iter=200_000)
    assert r["pobj"] == pytest.approx(expect, abs=1e-7)


def test_socp_two_cones_mixed_orthant(oracle_mod):
    """min x1 + t s.t. x1 + t = 3 with t >= ||(u1, u2)||, u = (1, 1), x1 >= 0:
    the optimum keeps t at its smallest, sqrt(2), value 3."""
    A = np.array([[1.0, 1.0, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0], [0.0, 0.0, 0.0, 1.0]])
    b = np.array([3.0, 1.0, 1.0])
    c = np.array([1.0, 2.0, 0.0, 0.0])  # min x1 + 2t -> t = sqrt(2), x1 = 3 - sqrt(2)
    orc = oracle_mod.Oracle(3, 4, *_csr_from_dense(A), b, c, 1, [3], mu=1.0)
    r = orc.solve(1e-10, max_iter=400_000)
    z = orc.state()["z"]
    np.testing.assert_allclose(z, [3 - np.sqrt(2), np.sqrt(2), 1, 1], atol=1e-6)
    assert r["pobj"] == pytest.approx(3 + np.sqrt(2), abs=1e-6)


def test_generator_lp_reaches_known_optimum(oracle_mod):
    inst = I.lp_instance(80, 160, 5, seed=10)
    assert inst["p_star"] == pytest.approx(inst["d_star"], rel=1e-13)
    orc = oracle_mod.Oracle.from_instance(inst, mu=1.0)
    r = orc.solve(1e-5, check_every=20, max_iter=400_000)
    assert r["kkt"] <= 1e-5
    # the relative gap bound at kkt <= 1e-5 carries over to the objective
    assert r["pobj"] == pytest.approx(inst["p_star"], rel=1e-4)


def test_socp_generator_bracket(oracle_mod):
    inst = I.socp_instance(20, 4, seed=13)
    orc = oracle_mod.Oracle.from_instance(inst, mu=1.0)
    r = orc.solve(1e-8, check_every=20, max_iter=400_000)
    assert r["kkt"] <= 1e-8
    assert inst["d_lower"] - 1e-6 <= r["pobj"] <= inst["p_upper"] + 1e-6


def test_infinity_norm_measures_on_a_random_state(oracle_mod):
    """prim_inf / dual_inf against dense products of a random state."""
    inst = I.socp_instance(10, 4, seed=19)
    rng = np.random.default_rng(8)
    orc = oracle_mod.Oracle.from_instance(inst)
    x, z, d = (rng.standard_normal(inst["n"]) for _ in range(3))
    lam = rng.standard_normal(inst["m"])
    orc.set_start(x, z, d, lam)
    r = orc.residuals()
    A = _dense(inst)
    assert r["prim_inf"] == pytest.approx(np.abs(A @ z - inst["b"]).max(), rel=1e-12)
    assert r["dual_inf"] == pytest.approx(np.abs(A.T @ lam + inst["c"] - d).max(), rel=1e-12)
    assert r["scale_p"] == pytest.approx(max(np.abs(A @ z).max(), np.abs(inst["b"]).max()), rel=1e-12)


def test_small_lp_reaches_1e4(oracle_mod):
    inst = I.config_instance("lp_small")
    orc = oracle_mod.Oracle.from_instance(inst, mu=1.0)
    r = orc.solve(1e-4, check_every=10, max_iter=50_000)
    assert r["kkt"] <= 1e-4
    assert r["pobj"] == pytest.approx(inst["p_star"], rel=1e-3)


def test_threads_do_not_change_results(oracle_mod):
    """Every reduction runs in a fixed serial order, so results are bitwise
    independent of the OpenMP thread count (checked in a subprocess)."""
    import subprocess, sys, textwrap
    code = textwrap.dedent("""
        import sys, numpy as np
        sys.path.insert(0, %r)
        import oracle
        from paper_2203_05027_amd import instances as I
        inst = I.socp_instance(30, 4, seed=1)
        o = oracle.Oracle.from_instance(inst); o.iterate(50)
        s = o.state(); print(np.concatenate([s['x'], s['lambda']]).tobytes().hex()[:4000])
    """ % os.path.dirname(GOLDEN).rsplit("/tests", 1)[0])
    outs = []
    for t in ("1", "3"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, check=True,
                                   capture_output=True, text=True).stdout)
    assert outs[0] == outs[1]


def test_paper_generator_is_feasible(oracle_mod):
    """The experiments' own generator: b = A proj_K(xdot), so proj_K(xdot) is
    feasible (in K and A x = b); density as requested."""
    for cone in ("lp", "socp"):
        inst = I.paper_instance(40, 80, 0.05, cone, seed=3)
        A = _dense(inst)
        x = inst["x_feasible"]
        assert abs(inst["nnz"] / (40 * 80) - 0.05) < 1e-3
        np.testing.assert_allclose(A @ x, inst["b"], atol=1e-12)
        np.testing.assert_allclose(oracle_mod.project(x, inst["n_orth"], inst["soc_sizes"]), x, atol=1e-12)
