"""GPU parity: the HIP solver (through the C ABI) against the FP64 CPU oracle.

The oracle runs Algorithm 1 literally (o-space y and gamma); the GPU runs the
reduced form.  In exact arithmetic both produce the same iterates; in FP64
they agree to rounding, and the bar is ||v_gpu - v_oracle||_inf <=
1e-9 * ||v_oracle||_inf for v in {x, z, delta, lambda} after 200 iterations
from the same start.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2203_05027_amd import instances as I
from paper_2203_05027_amd.solver import Solver

pytestmark = pytest.mark.gpu

TOL64 = 1e-9
KEYS = ("x", "z", "delta", "lambda")


def say(msg):
    sys.__stderr__.write(f"[gpu-test] {msg}\n")
    sys.__stderr__.flush()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)) if b.size else 0.0


def run_pair(inst, iters, mu=1.0, start=None, **kw):
    say(f"m={inst['m']} n={inst['n']} nnz={inst['nnz']} iters={iters} mu={mu} {kw}")
    orc = oracle.Oracle.from_instance(inst, mu=mu)
    with Solver.from_instance(inst, mu=mu, eps=0.0, **kw) as s:
        if start is not None:
            orc.set_start(*start)
            s.set_start(*start)
        orc.iterate(iters)
        s.iterate(iters)
        g = s.solution()
        gr = s.residuals()
    o = orc.state()
    return g, o, gr, orc.residuals()


def assert_parity(g, o, tol=TOL64):
    errs = {k: rel(g[k], o[k]) for k in KEYS}
    say(f"rel errors {errs}")
    for k in KEYS:
        assert errs[k] <= tol, (k, errs[k])


def test_small_lp_200_iterations():
    g, o, gr, orr = run_pair(I.config_instance("lp_small"), 200)
    assert_parity(g, o)
    for k in ("r_prim", "r_dual", "r_gap", "kkt", "pobj", "dobj", "res_ax_b", "prim_inf", "dual_inf",
              "scale_p", "scale_d", "pobj_x"):
        assert abs(gr[k] - orr[k]) <= 1e-9 * max(abs(orr[k]), 1e-12), k
    gap_x = abs(orr["pobj_x"] - orr["dobj"])
    assert abs(gr["gap_x"] - gap_x) <= 1e-9 * max(gap_x, 1e-12)
    assert gr["iter"] == 200


def test_infinity_norm_criterion_stops_like_oracle():
    """The infinity-norm stopping test (eps_abs 1e-4, eps_rel 1e-3) stops at
    the same check as the same test evaluated on the oracle's iterates."""
    inst = I.config_instance("lp_small")
    orc = oracle.Oracle.from_instance(inst)
    it = 0
    while it < 60_000:
        orc.iterate(10)
        it += 10
        r = orc.residuals()
        if (r["prim_inf"] <= 1e-4 + 1e-3 * r["scale_p"] and r["dual_inf"] <= 1e-4 + 1e-3 * r["scale_d"]):
            break
    with Solver.from_instance(inst, eps=1e-3, eps_abs=1e-4, criterion="inf") as s:
        assert s.iterate(60_000)
        g = s.residuals()
    say(f"inf criterion: gpu {g['iter']} oracle {it}")
    assert g["status"] == "converged" and g["iter"] == it


def _oracle_stop(inst, test, cap=60_000):
    """Iteration at which `test(residuals)` first holds on the oracle's
    iterates, checked every 10 iterations."""
    orc = oracle.Oracle.from_instance(inst)
    it = 0
    while it < cap:
        orc.iterate(10)
        it += 10
        if test(orc.residuals()):
            return it
    return None


@pytest.mark.parametrize("slabs", [1, 4])
def test_pogs_criterion_stops_like_oracle(slabs):
    """The stopping test of the POGS comparison (Section V-A2, eq. stopcri):
    ||Ax - b||_2 and |c'x + b'lambda| below given bounds (there the
    competitor's values; here fixed ones), at the same check as the same test
    on the oracle's iterates."""
    inst = I.config_instance("lp_small")
    tp = 1e-3 * (1.0 + float(np.linalg.norm(inst["b"])))
    tg = 1e-3 * (1.0 + abs(inst["p_star"]))
    it = _oracle_stop(inst, lambda r: r["res_ax_b"] < tp and abs(r["pobj_x"] - r["dobj"]) < tg)
    with Solver.from_instance(inst, eps=0.0, eps_abs=tp, eps_gap=tg, criterion="pogs",
                              slabs_row=slabs, slabs_col=slabs) as s:
        assert s.iterate(60_000)
        g = s.residuals()
    say(f"pogs criterion: gpu {g['iter']} oracle {it}")
    assert g["status"] == "converged" and g["iter"] == it
    assert g["res_ax_b"] < tp and g["gap_x"] < tg


def test_infinity_norm_criterion_with_gap_stops_like_oracle():
    """The OSQP comparison's test (Section V-A1) with its extra gap
    condition |c'x + b'lambda| < eps_gap."""
    inst = I.config_instance("lp_small")
    tg = 3e-4 * (1.0 + abs(inst["p_star"]))

    def test(r):
        return (r["prim_inf"] <= 1e-4 + 1e-3 * r["scale_p"] and r["dual_inf"] <= 1e-4 + 1e-3 * r["scale_d"]
                and abs(r["pobj_x"] - r["dobj"]) < tg)
    it = _oracle_stop(inst, test)
    with Solver.from_instance(inst, eps=1e-3, eps_abs=1e-4, eps_gap=tg, criterion="inf") as s:
        assert s.iterate(60_000)
        g = s.residuals()
    say(f"inf + gap criterion: gpu {g['iter']} oracle {it}")
    assert g["status"] == "converged" and g["iter"] == it


@pytest.mark.parametrize("lanes,unroll", [((1, 1), (1, 8)), ((2, 16), (8, 1)), ((64, 64), (2, 4)),
                                          ((32, 4), (4, 2)), ((4, 2), (8, 8))])
@pytest.mark.parametrize("graph", [True, False])
def test_launch_shapes(lanes, unroll, graph):
    inst = I.lp_instance(333, 777, 4, seed=17)          # ragged: no size divides a tile
    g, o, _, _ = run_pair(inst, 200, mu=0.7, lanes_row=lanes[0], lanes_col=lanes[1],
                          unroll_row=unroll[0], unroll_col=unroll[1], use_graph=graph,
                          check_every=7)
    assert_parity(g, o)


@pytest.mark.parametrize("slabs", [(2, 2), (8, 4), (4, 8), (8, 1), (1, 8)])
@pytest.mark.parametrize("kernel", ["chunked", "chunked4", "lanes"])
def test_xcd_slabs(slabs, kernel):
    """Slab-split passes (forced on a small ragged problem) against the oracle,
    with the fused residual check inside the chunk."""
    inst = I.conic_instance(1003, 411, [3, 7, 50, 1, 260] + [5] * 40, 4, seed=23)
    g, o, gr, orr = run_pair(inst, 200, mu=0.9, slabs_row=slabs[0], slabs_col=slabs[1], check_every=9,
                             lanes_row=4, lanes_col=2, slab_kernel=kernel)
    assert_parity(g, o)
    for k in ("r_prim", "r_dual", "r_gap", "pobj", "dobj", "res_ax_b"):
        assert abs(gr[k] - orr[k]) <= 1e-9 * max(abs(orr[k]), 1e-12), k


@pytest.mark.parametrize("kernel", ["chunked", "chunked4"])
def test_chunked_long_segments(kernel):
    """Segments longer than a wavefront's LDS round (dense rows and columns)
    and empty ones, through the chunked slab kernel."""
    base = I.lp_instance(700, 1500, 3, seed=25)
    A = np.zeros((700, 1500))
    rows = np.repeat(np.arange(700), np.diff(base["row_ptr"]))
    A[rows, base["col_idx"]] = base["val"]
    rng = np.random.default_rng(4)
    A[5, :] = rng.standard_normal(1500)          # a dense row (1500 entries)
    A[:, 7] = rng.standard_normal(700)           # a dense column
    A[100:140, :] = 0.0                          # empty rows
    rr, cc = np.nonzero(A)
    row_ptr = np.zeros(701, np.int64)
    np.cumsum(np.bincount(rr, minlength=700), out=row_ptr[1:])
    inst = dict(base, row_ptr=row_ptr, col_idx=cc.astype(np.int32), val=A[rr, cc], nnz=int(rr.size),
                b=A @ base["x0"])
    g, o, _, _ = run_pair(inst, 200, slabs_row=4, slabs_col=2, check_every=6, slab_kernel=kernel)
    assert_parity(g, o)


def test_xcd_slabs_resume_and_mixed():
    inst = I.lp_instance(3000, 6100, 6, seed=24)
    rng = np.random.default_rng(2)
    st = (rng.standard_normal(inst["n"]), rng.standard_normal(inst["n"]),
          rng.standard_normal(inst["n"]), rng.standard_normal(inst["m"]))
    orc = oracle.Oracle.from_instance(inst)
    orc.resume(*st)
    orc.iterate(100)
    with Solver.from_instance(inst, eps=0.0, slabs_row=8, slabs_col=8) as s:
        assert s.launch_shape()["slabs_row"] == 8
        s.resume(*st)
        s.iterate(100)
        assert_parity(s.solution(), orc.state())
    with Solver.from_instance(inst, eps=1e-4, precision="mixed", slabs_row=4, slabs_col=2) as s:
        assert s.iterate(200_000)
        r = s.residuals()
    assert r["status"] == "converged" and r["kkt"] <= 1e-4
    assert abs(r["pobj"] - inst["p_star"]) <= 2e-3 * abs(inst["p_star"])


@pytest.mark.parametrize("unroll", [1, 2, 8])
def test_socp_unroll_shapes(unroll):
    inst = I.socp_instance(150, 8, seed=21)
    g, o, _, _ = run_pair(inst, 100, unroll_row=unroll, unroll_col=unroll, lanes_col=2)
    assert_parity(g, o)


def test_scaled_large_lp_unit_rows():
    inst = I.lp_instance(20_000, 40_000, 10, seed=1, unit_rows=True)
    g, o, _, _ = run_pair(inst, 200)
    assert_parity(g, o)


def test_socp_200_iterations():
    inst = I.socp_instance(400, 8, seed=2)
    g, o, gr, orr = run_pair(inst, 200)
    assert_parity(g, o)
    assert abs(gr["kkt"] - orr["kkt"]) <= 1e-9 * orr["kkt"]


def test_mixed_cones_big_and_size1():
    """Orthant + SOCs of sizes 1 (a half line), 2, and above 256 columns
    (one cone alone fills a wider tile)."""
    sizes = [1, 2, 3, 700, 1, 50, 1024, 5] + [4] * 60
    inst = I.conic_instance(900, 123, sizes, 3, seed=5)
    g, o, _, _ = run_pair(inst, 200, mu=1.3)
    assert_parity(g, o)


def test_warm_start():
    inst = I.socp_instance(60, 5, seed=8)
    rng = np.random.default_rng(3)
    n, m = inst["n"], inst["m"]
    start = (rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(n),
             rng.standard_normal(m))
    g, o, _, _ = run_pair(inst, 200, mu=0.5, start=start)
    assert_parity(g, o)


def test_empty_rows_and_columns():
    base = I.lp_instance(300, 700, 3, seed=4)
    A = np.zeros((300, 700))
    rows = np.repeat(np.arange(300), np.diff(base["row_ptr"]))
    A[rows, base["col_idx"]] = base["val"]
    A[:10, :] = 0.0
    A[:, :20] = 0.0
    rr, cc = np.nonzero(A)
    row_ptr = np.zeros(301, np.int64)
    np.cumsum(np.bincount(rr, minlength=300), out=row_ptr[1:])
    inst = dict(base, row_ptr=row_ptr, col_idx=cc.astype(np.int32), val=A[rr, cc],
                nnz=int(rr.size), b=A @ base["x0"])
    g, o, _, _ = run_pair(inst, 200)
    assert_parity(g, o)


def test_no_nonzeros():
    m, n = 5, 9
    inst = dict(m=m, n=n, nnz=0, row_ptr=np.zeros(m + 1, np.int64), col_idx=np.zeros(0, np.int32),
                val=np.zeros(0), b=np.zeros(m), c=np.linspace(-1, 1, n), n_orth=4,
                soc_sizes=np.array([5], np.int32))
    g, o, _, _ = run_pair(inst, 50)
    assert_parity(g, o)


def test_converges_at_same_check_as_oracle():
    inst = I.config_instance("lp_small")
    orc = oracle.Oracle.from_instance(inst)
    ro = orc.solve(1e-4, check_every=10, max_iter=50_000)
    say(f"oracle converged at {ro['iter']}")
    with Solver.from_instance(inst, eps=1e-4, check_every=10) as s:
        done = s.iterate(50_000)
        r = s.residuals()
    assert done and r["status"] == "converged"
    assert r["iter"] == ro["iter"]
    assert r["kkt"] <= 1e-4
    assert abs(r["pobj"] - inst["p_star"]) <= 1e-3 * abs(inst["p_star"])


def test_max_iter_and_resume():
    inst = I.lp_instance(200, 400, 4, seed=6)
    with Solver.from_instance(inst, eps=0.0, max_iter=25, check_every=10) as s:
        assert s.iterate(100)
        r = s.residuals()
        assert r["status"] == "max_iter" and r["iter"] == 25
    # checkpoint / resume: solution + resume continues the same trajectory
    with Solver.from_instance(inst, eps=0.0) as a, Solver.from_instance(inst, eps=0.0) as b:
        a.iterate(40)
        sol = a.solution()
        a.iterate(60)
        b.resume(sol["x"], sol["z"], sol["delta"], sol["lambda"])
        b.iterate(60)
        assert_parity(b.solution(), a.solution(), tol=1e-12)


def test_resume_matches_oracle_resume():
    inst = I.socp_instance(80, 6, seed=14)
    rng = np.random.default_rng(5)
    st = (rng.standard_normal(inst["n"]), rng.standard_normal(inst["n"]),
          rng.standard_normal(inst["n"]), rng.standard_normal(inst["m"]))
    orc = oracle.Oracle.from_instance(inst, mu=0.9)
    orc.resume(*st)
    orc.iterate(150)
    with Solver.from_instance(inst, mu=0.9, eps=0.0) as s:
        s.resume(*st)
        s.iterate(150)
        assert_parity(s.solution(), orc.state())


def test_residuals_off_check_iteration():
    inst = I.socp_instance(50, 6, seed=9)
    orc = oracle.Oracle.from_instance(inst)
    orc.iterate(7)
    with Solver.from_instance(inst, eps=0.0, check_every=10) as s:
        s.iterate(7)
        r = s.residuals()
    ro = orc.residuals()
    assert r["iter"] == 7
    for k in ("r_prim", "r_dual", "r_gap", "pobj", "dobj"):
        assert abs(r[k] - ro[k]) <= 1e-9 * max(abs(ro[k]), 1e-12), k


def test_bitwise_reproducible():
    inst = I.socp_instance(300, 8, seed=12)
    outs = []
    for graph in (True, True, False):
        with Solver.from_instance(inst, eps=0.0, use_graph=graph) as s:
            s.iterate(100)
            outs.append(s.solution())
    for o in outs[1:]:
        for k in KEYS:
            assert np.array_equal(o[k], outs[0][k])


@pytest.mark.parametrize("name", ["lp_large", "socp_large", "paper_lp", "paper_socp", "paper_lp_0p1",
                                  "paper_socp_0p1", "paper_lp_1p0", "paper_socp_1p0"])
def test_full_size_sampled_parity(name):
    """The full-size workloads in the launch configuration the benchmark
    times (automatic lanes, unroll and XCD slabs, graph replay): 3 iterations
    from the zero start, every entry against the oracle."""
    inst = I.config_instance(name)
    say(f"{name}: m={inst['m']} n={inst['n']} nnz={inst['nnz']}")
    g, o, gr, orr = run_pair(inst, 3, check_every=3)
    assert_parity(g, o)
    for k in ("r_prim", "r_dual", "r_gap", "pobj", "dobj"):
        assert abs(gr[k] - orr[k]) <= 1e-9 * max(abs(orr[k]), 1e-12), k


def test_full_size_mixed_precision():
    """The 1e6 x 2e6 LP in the mixed form the benchmark times: 3 iterations
    against the FP64 oracle, every entry within FP32 rounding of the sweep."""
    inst = I.config_instance("lp_large")
    g, o, _, _ = run_pair(inst, 3, check_every=3, precision="mixed")
    errs = {k: rel(g[k], o[k]) for k in KEYS}
    say(f"lp_large mixed vs fp64 oracle after 3 iterations: {errs}")
    for k in KEYS:
        assert errs[k] <= 1e-5, (k, errs[k])


def test_mixed_precision_small_lp():
    """FP32 sweep, FP64 duals and residuals: reaches 1e-4 and the objective
    stays within the KKT bound of the oracle's optimum."""
    inst = I.config_instance("lp_small")
    g, o, _, _ = run_pair(inst, 200, precision="mixed")
    errs = {k: rel(g[k], o[k]) for k in KEYS}
    say(f"mixed vs fp64 oracle after 200 iterations: {errs}")
    for k in KEYS:
        assert errs[k] <= 1e-4, (k, errs[k])
    with Solver.from_instance(inst, eps=1e-4, precision="mixed") as s:
        assert s.iterate(60_000)
        r = s.residuals()
    say(f"mixed converged: {r}")
    assert r["status"] == "converged" and r["kkt"] <= 1e-4
    assert abs(r["pobj"] - inst["p_star"]) <= 2e-3 * abs(inst["p_star"])


def test_mixed_precision_socp():
    inst = I.socp_instance(400, 8, seed=2)
    with Solver.from_instance(inst, eps=1e-4, precision="mixed") as s:
        assert s.iterate(20_000)
        r = s.residuals()
    say(f"mixed socp: {r}")
    assert r["status"] == "converged" and r["kkt"] <= 1e-4
    assert inst["d_lower"] - 1e-3 <= r["pobj"] <= inst["p_upper"] + 1e-3


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("slabs", [(2, 2), (4, 2), (8, 8), (2, 1), (1, 4)])
def test_chunk_depths_bitwise(precision, slabs):
    """Four or eight 64-entry steps in flight per wavefront change only the
    schedule of the chunked slab product, never its sums: bitwise the same
    iterates and residuals, on a ragged LP and on a conic problem, and the
    FP64 ones match the oracle."""
    lp = I.lp_instance(1003, 2411, 5, seed=31)
    conic = I.conic_instance(1003, 411, [3, 7, 50, 1, 260] + [5] * 40, 4, seed=23)
    for inst in (lp, conic):
        outs = []
        for kernel in ("chunked", "chunked4", "auto"):
            say(f"{precision} slabs={slabs} kernel={kernel} m={inst['m']} n={inst['n']}")
            with Solver.from_instance(inst, eps=0.0, precision=precision, slabs_row=slabs[0],
                                      slabs_col=slabs[1], check_every=9, slab_kernel=kernel) as s:
                s.iterate(200)
                outs.append((s.solution(), s.residuals()))
        for sol, res in outs[1:]:
            for k in KEYS:
                assert np.array_equal(sol[k], outs[0][0][k]), k
            assert res == outs[0][1]
        if precision == "fp64":
            orc = oracle.Oracle.from_instance(inst)
            orc.iterate(200)
            assert_parity(outs[0][0], orc.state())


@pytest.mark.parametrize("slabs", [(4, 2), (1, 1), (2, 8)])
@pytest.mark.parametrize("conic", [False, True])
def test_mixed_check_residuals_at_the_state(slabs, conic):
    """The mixed form's checks (FP64 values of A through the slab copies, FP64
    sums) equal the oracle's residuals evaluated at the GPU's own iterate."""
    inst = (I.conic_instance(2003, 911, [3, 7, 50, 1, 260] + [5] * 100, 4, seed=33) if conic
            else I.lp_instance(3001, 6100, 6, seed=32))
    with Solver.from_instance(inst, eps=0.0, precision="mixed", slabs_row=slabs[0], slabs_col=slabs[1],
                              check_every=10) as s:
        s.iterate(60)
        g = s.solution()
        gr = s.residuals()
    assert gr["iter"] == 60
    orc = oracle.Oracle.from_instance(inst)
    orc.set_state(x=g["x"], z=g["z"], delta=g["delta"], lam=g["lambda"])
    ro = orc.residuals()
    say(f"mixed check slabs={slabs} conic={conic}: gpu kkt {gr['kkt']:.6e} oracle {ro['kkt']:.6e}")
    for k in ("r_prim", "r_dual", "r_gap", "kkt", "pobj", "dobj", "res_ax_b", "prim_inf", "dual_inf",
              "scale_p", "scale_d"):
        assert abs(gr[k] - ro[k]) <= 1e-11 * max(abs(ro[k]), 1e-12), (k, gr[k], ro[k])
