"""Pins of the standard-ADMM + CG oracle (Sections II-B and III-B) against
what the mathematics fixes:
* one iteration against a dense solve of the block system eq. lin (the CG
  runs to exactness on a tiny problem) and the closed-form prox of the
  orthant indicator;
* the fixed point at a known primal-dual optimum, for several mu;
* exact invariants of every iterate (x1 in K, delta in K*, complementarity)
  whatever the CG accuracy, and the dual-residual identity of an exact solve;
* brute-force vertex enumeration on tiny LPs and a hand-solved LP;
* with Lorentz cones: one iteration against the (separately pinned)
  projection and the dense block solve, cone invariants, closed-form tiny
  SOCPs.
"""
import itertools

import numpy as np
import pytest

from paper_2203_05027_amd import instances as I


@pytest.fixture(scope="module")
def std():
    from oracle import standard
    return standard


@pytest.fixture(scope="module")
def oracle_mod():
    import oracle
    return oracle


def _dense(inst):
    A = np.zeros((inst["m"], inst["n"]))
    rp = inst["row_ptr"]
    for i in range(inst["m"]):
        for k in range(rp[i], rp[i + 1]):
            A[i, inst["col_idx"][k]] = inst["val"][k]
    return A


def _brute_force_lp(A, b, c):
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


@pytest.mark.parametrize("seed,mu", [(31, 1.0), (32, 0.4), (33, 3.0)])
def test_one_iteration_against_dense_block_solve(std, seed, mu):
    inst = I.lp_instance(4, 9, 2, seed=seed)
    A = _dense(inst)
    m, n = A.shape
    rng = np.random.default_rng(seed)
    x2, lam = rng.standard_normal(n), rng.standard_normal(n)
    s = std.StandardADMM.from_instance(inst, mu=mu, cg_iters=50, cg_tol=0.0)
    s.set_state(x2=x2, lam=lam)
    s.iterate(1)
    st = s.state()
    x1 = np.maximum(x2 - lam / mu, 0.0)                       # prox of the cone indicator
    np.testing.assert_allclose(st["x1"], x1, atol=1e-14)
    K = np.block([[np.eye(n), A.T], [A, np.zeros((m, m))]])   # eq. lin
    sol = np.linalg.solve(K, np.concatenate([x1 + lam / mu - inst["c"] / mu, inst["b"]]))
    w, nu = sol[:n], sol[n:]
    np.testing.assert_allclose(st["x2"], w, atol=1e-10)
    np.testing.assert_allclose(st["nu"], nu, atol=1e-10)
    np.testing.assert_allclose(A @ st["x2"], inst["b"], atol=1e-10)
    np.testing.assert_allclose(st["lam"], lam + mu * (x1 - w), atol=1e-10)
    np.testing.assert_allclose(st["delta"], lam + mu * (x1 - x2), atol=1e-13)


@pytest.mark.parametrize("mu", [0.37, 1.0, 4.0])
def test_fixed_point_at_known_optimum(std, mu):
    """x2 = x0, lam = s0 (the cone multiplier), nu = -y0/mu is a fixed point."""
    inst = I.lp_instance(60, 120, 4, seed=7)
    s = std.StandardADMM.from_instance(inst, mu=mu, cg_iters=3, cg_tol=0.0)
    s.set_state(x2=inst["x0"], lam=inst["s0"], nu=-inst["y0"] / mu)
    s.iterate(5)
    st = s.state()
    for k, ref in (("x1", inst["x0"]), ("x2", inst["x0"]), ("lam", inst["s0"]),
                   ("delta", inst["s0"]), ("nu", -inst["y0"] / mu)):
        np.testing.assert_allclose(st[k], ref, atol=1e-11 * (1 + np.abs(ref).max()))
    r = s.residuals()
    assert r["kkt"] < 1e-12
    assert r["pobj"] == pytest.approx(inst["p_star"], rel=1e-12)
    assert r["dobj"] == pytest.approx(inst["p_star"], rel=1e-12)


@pytest.mark.parametrize("cg_iters", [0, 1, 4])
def test_exact_invariants_with_inexact_cg(std, cg_iters):
    inst = I.lp_instance(40, 80, 3, seed=11)
    s = std.StandardADMM.from_instance(inst, mu=1.3, cg_iters=cg_iters, cg_tol=0.0)
    for _ in range(5):
        s.iterate(7)
        st = s.state()
        tol = 1e-13 * (1 + np.abs(st["lam"]).max())          # delta is formed as lam + mu (x1 - x2)
        assert st["x1"].min() >= 0.0
        assert st["delta"].min() >= -tol
        assert np.abs(st["x1"] * st["delta"]).max() <= tol * (1 + st["x1"].max())
    assert s.cg_steps == 35 * cg_iters


def test_dual_residual_identity_of_an_exact_solve(std):
    """With eq. lin solved exactly, A'(mu nu) + c - delta = mu (x2_prev - x2)."""
    inst = I.lp_instance(5, 10, 2, seed=12)
    A = _dense(inst)
    mu = 0.8
    s = std.StandardADMM.from_instance(inst, mu=mu, cg_iters=60, cg_tol=0.0)
    s.iterate(3)
    prev = s.state()["x2"].copy()
    s.iterate(1)
    st = s.state()
    lhs = A.T @ (mu * st["nu"]) + inst["c"] - st["delta"]
    np.testing.assert_allclose(lhs, mu * (prev - st["x2"]), atol=1e-10)
    r = s.residuals()
    assert r["r_dual"] == pytest.approx(np.linalg.norm(lhs) / (1 + np.linalg.norm(inst["c"])), rel=1e-8, abs=1e-14)


def test_tolerance_stops_cg_early(std):
    inst = I.lp_instance(40, 80, 3, seed=13)
    a = std.StandardADMM.from_instance(inst, cg_iters=50, cg_tol=1e-3)
    a.iterate(20)
    b = std.StandardADMM.from_instance(inst, cg_iters=50, cg_tol=0.0)
    b.iterate(20)
    assert a.cg_steps < b.cg_steps == 1000


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_tiny_lp_against_vertex_enumeration(std, seed):
    inst = I.lp_instance(3, 7, 2, seed=seed)
    A = _dense(inst)
    p_star = _brute_force_lp(A, inst["b"], inst["c"])
    s = std.StandardADMM.from_instance(inst, mu=1.0, cg_iters=20, cg_tol=0.0)
    r = s.solve(1e-9, max_iter=200_000)
    assert r["kkt"] <= 1e-9
    assert abs(r["pobj"] - p_star) <= 1e-6 * (1 + abs(p_star))
    assert abs(r["dobj"] - p_star) <= 1e-6 * (1 + abs(p_star))


def test_hand_lp(std):
    """min -x1 - 2x2 s.t. x1 + x2 + s1 = 4, x1 + 3x2 + s2 = 6, x >= 0:
    (x1, x2) = (3, 1), value -5."""
    row_ptr = np.array([0, 3, 6], np.int64)
    col_idx = np.array([0, 1, 2, 0, 1, 3], np.int32)
    val = np.array([1.0, 1.0, 1.0, 1.0, 3.0, 1.0])
    s = std.StandardADMM(2, 4, row_ptr, col_idx, val, np.array([4.0, 6.0]),
                         np.array([-1.0, -2.0, 0.0, 0.0]), mu=1.0, cg_iters=10)
    r = s.solve(1e-10, max_iter=100_000)
    np.testing.assert_allclose(s.state()["x1"], [3, 1, 0, 0], atol=1e-7)
    assert r["pobj"] == pytest.approx(-5.0, abs=1e-7)


def test_generator_lp_reaches_known_optimum(std):
    inst = I.lp_instance(100, 200, 4, seed=14)
    s = std.StandardADMM.from_instance(inst, mu=1.0, cg_iters=30, cg_tol=1e-10)
    r = s.solve(1e-5, max_iter=50_000)
    assert r["kkt"] <= 1e-5
    assert r["pobj"] == pytest.approx(inst["p_star"], rel=1e-4)
    assert r["dobj"] == pytest.approx(inst["p_star"], rel=1e-4)


# --------------------------------------------------------------------------
# Lorentz cones
# --------------------------------------------------------------------------
def _csr_from_dense(A):
    rows, cols = np.nonzero(A)
    row_ptr = np.zeros(A.shape[0] + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=A.shape[0]), out=row_ptr[1:])
    return row_ptr, cols.astype(np.int32), A[rows, cols]


@pytest.mark.parametrize("seed,mu", [(61, 1.0), (62, 0.5)])
def test_one_iteration_with_cones_against_dense_block_solve(std, oracle_mod, seed, mu):
    """x1 is the projection onto K (the UV oracle's, pinned on its own), x2
    the dense solve of eq. lin."""
    inst = I.conic_instance(6, 3, [3, 4, 1], 2, seed=seed)
    A = _dense(inst)
    m, n = A.shape
    rng = np.random.default_rng(seed)
    x2, lam = rng.standard_normal(n), rng.standard_normal(n)
    s = std.StandardADMM.from_instance(inst, mu=mu, cg_iters=60, cg_tol=0.0)
    s.set_state(x2=x2, lam=lam)
    s.iterate(1)
    st = s.state()
    x1 = oracle_mod.project(x2 - lam / mu, inst["n_orth"], inst["soc_sizes"])
    np.testing.assert_allclose(st["x1"], x1, atol=1e-13)
    K = np.block([[np.eye(n), A.T], [A, np.zeros((m, m))]])
    sol = np.linalg.lstsq(K, np.concatenate([x1 + lam / mu - inst["c"] / mu, inst["b"]]), rcond=None)[0]
    np.testing.assert_allclose(st["x2"], sol[:n], atol=1e-9)
    np.testing.assert_allclose(st["lam"], lam + mu * (x1 - sol[:n]), atol=1e-9)


def _cone_parts(v, n_orth, sizes):
    parts, off = [v[:n_orth]], n_orth
    for k in sizes:
        parts.append(v[off:off + k])
        off += k
    return parts


def test_cone_invariants_with_inexact_cg(std):
    inst = I.conic_instance(60, 20, [3, 7, 12, 5, 1, 30], 3, seed=63)
    s = std.StandardADMM.from_instance(inst, mu=0.9, cg_iters=2, cg_tol=0.0)
    for _ in range(4):
        s.iterate(9)
        st = s.state()
        tol = 1e-12 * (1 + np.abs(st["lam"]).max() + np.abs(st["x1"]).max())
        xp = _cone_parts(st["x1"], inst["n_orth"], inst["soc_sizes"])
        dp = _cone_parts(st["delta"], inst["n_orth"], inst["soc_sizes"])
        assert xp[0].min() >= 0.0 and dp[0].min() >= -tol
        for xb, db in zip(xp[1:], dp[1:]):                  # K and K* (self-dual) per cone
            assert xb[0] >= np.linalg.norm(xb[1:]) - tol
            assert db[0] >= np.linalg.norm(db[1:]) - tol
            assert abs(xb @ db) <= 10 * tol * (1 + np.abs(db).max())


@pytest.mark.parametrize("u,expect", [((1.0, 2.0), np.sqrt(5.0)), ((3.0, 4.0), 5.0)])
def test_tiny_socp_closed_form(std, u, expect):
    """min t s.t. (t, u1, u2) in K_3 with u fixed: the optimum is ||u||."""
    A = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
    s = std.StandardADMM(2, 3, *_csr_from_dense(A), np.array(u), np.array([1.0, 0, 0]), mu=1.0,
                         cg_iters=10, n_orth=0, soc_sizes=[3])
    r = s.solve(1e-10, max_iter=100_000)
    assert r["pobj"] == pytest.approx(expect, abs=1e-7)


def test_socp_two_cones_mixed_orthant(std):
    """min x1 + 2t s.t. x1 + t = 3, u = (1, 1), x1 >= 0, t >= ||u||:
    t = sqrt(2), x1 = 3 - sqrt(2)."""
    A = np.array([[1.0, 1.0, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0], [0.0, 0.0, 0.0, 1.0]])
    s = std.StandardADMM(3, 4, *_csr_from_dense(A), np.array([3.0, 1.0, 1.0]),
                         np.array([1.0, 2.0, 0.0, 0.0]), mu=1.0, cg_iters=10, n_orth=1, soc_sizes=[3])
    r = s.solve(1e-10, max_iter=200_000)
    np.testing.assert_allclose(s.state()["x1"], [3 - np.sqrt(2), np.sqrt(2), 1, 1], atol=1e-6)
    assert r["pobj"] == pytest.approx(3 + np.sqrt(2), abs=1e-6)


def test_projection_characterisation(std):
    """Moreau for a self-dual cone: w = P(w) - P(-w) with P(w), P(-w) in K
    and orthogonal -- which determines the projection -- on random points,
    points near the cone's boundary and on it, and size-1 cones (ReLU)."""
    rng = np.random.default_rng(64)
    sizes = [1, 2, 3, 5, 8, 13]
    pts = [rng.standard_normal(sum(sizes) + 4) for _ in range(20)]
    for eps in (0.0, 1e-9, 1e-6, 1e-4, -1e-6, -1e-4):           # t = ||u|| (1 + eps)
        w = rng.standard_normal(sum(sizes) + 4)
        off = 4
        for k in sizes:
            if k > 1:
                w[off] = np.linalg.norm(w[off + 1:off + k]) * (1 + eps) * rng.choice([-1, 1])
            off += k
        pts.append(w)
    for w in pts:
        p, q = std.project(w, 4, sizes), std.project(-w, 4, sizes)
        np.testing.assert_allclose(p - q, w, atol=1e-12)
        np.testing.assert_allclose(p[:4], np.maximum(w[:4], 0.0), atol=0)
        off = 4
        for k in sizes:
            pb, qb = p[off:off + k], q[off:off + k]
            for v in (pb, qb):
                assert v[0] >= np.linalg.norm(v[1:]) - 1e-12 * (1 + np.abs(w).max())
            assert abs(pb @ qb) <= 1e-12 * (1 + np.abs(w).max()) ** 2
            off += k
