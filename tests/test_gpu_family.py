"""GPU tests of the parametric-family solver (one A, many b) against the
CPU oracle run on each member alone."""
import sys

import numpy as np
import pytest

import oracle
from paper_2203_05027_amd import instances as I
from paper_2203_05027_amd.solver import Family

pytestmark = pytest.mark.gpu
KEYS = ("x", "z", "delta", "lambda")


def say(msg):
    sys.__stderr__.write(f"[gpu-test] {msg}\n")
    sys.__stderr__.flush()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


def family_members(fam, thetas):
    return [fam.instance(t) for t in thetas]


@pytest.fixture(scope="module")
def small_family():
    return I.ParametricFamily(m=300, n=600, k=5, p=8, seed=7)


@pytest.mark.parametrize("B,nb", [(64, 5), (128, 70), (192, 150), (512, 300)])
def test_fp64_family_matches_oracle(small_family, B, nb):
    fam = small_family
    thetas = [fam.theta(1000 + i, p=8) for i in range(nb)]
    insts = family_members(fam, thetas)
    say(f"family B={B} nb={nb}")
    with Family(fam.m, fam.n, fam.row_ptr, fam.col_idx, fam.val, fam.c, B=B, precision="fp64",
                eps=0.0, check_every=7) as F:
        F.set_rhs(np.stack([i["b"] for i in insts]))
        F.iterate(200)
        sol = F.solution()
        res = F.residuals()
    for l in (0, 1, nb // 2, nb - 1):
        o = oracle.Oracle.from_instance(insts[l])
        o.iterate(200)
        s = o.state()
        errs = {k: rel(sol[k][l], s[k]) for k in KEYS}
        assert max(errs.values()) <= 1e-9, (l, errs)
        r = o.residuals()
        assert res[l]["iter"] == 200 or res[l]["status"] == "running"


def test_fp64_family_convergence_matches_oracle(small_family):
    fam = small_family
    insts = family_members(fam, [fam.theta(2000 + i, p=8) for i in range(3)])
    with Family(fam.m, fam.n, fam.row_ptr, fam.col_idx, fam.val, fam.c, B=64, precision="fp64",
                eps=1e-4) as F:
        F.set_rhs(np.stack([i["b"] for i in insts]))
        assert F.iterate(300_000) == 0
        res = F.residuals()
    for l, inst in enumerate(insts):
        ro = oracle.Oracle.from_instance(inst).solve(1e-4, check_every=10, max_iter=300_000)
        say(f"member {l}: family {res[l]['iter']} oracle {ro['iter']}")
        assert res[l]["status"] == "converged" and res[l]["iter"] == ro["iter"]
        assert abs(res[l]["pobj"] - ro["pobj"]) <= 1e-9 * abs(ro["pobj"])


def test_warm_start_at_solution_is_converged(small_family):
    """Starting from a solution (x*, lambda*) the predicted-start mapping
    (z = max(x, 0), delta = max(c + A'lambda, 0)) is converged at once."""
    import torch
    assert torch.cuda.is_available()
    fam = small_family
    insts = family_members(fam, [fam.theta(3000 + i, p=8) for i in range(4)])
    b = np.stack([i["b"] for i in insts])
    with Family(fam.m, fam.n, fam.row_ptr, fam.col_idx, fam.val, fam.c, B=64, precision="mixed",
                eps=1e-5) as F:
        F.set_rhs(b)
        assert F.iterate(400_000) == 0
        cold = [r["iter"] for r in F.residuals()]
        sol = F.solution()
        xl = np.concatenate([sol["z"], sol["lambda"]], axis=1).astype(np.float32)
        dev = torch.from_numpy(xl).cuda()
        F.set_rhs(b)
        F.set_start_predicted(dev.data_ptr(), xl.shape[1], "both")
        torch.cuda.synchronize()
        s0 = F.solution()
        np.testing.assert_allclose(s0["z"], np.maximum(xl[:, :fam.n], 0), rtol=1e-6, atol=1e-6)
        A = np.zeros((fam.m, fam.n))
        A[np.repeat(np.arange(fam.m), np.diff(fam.row_ptr)), fam.col_idx] = fam.val
        dl = np.maximum(fam.c[None, :] + xl[:, fam.n:].astype(np.float64) @ A, 0)
        np.testing.assert_allclose(s0["delta"], dl, rtol=1e-9, atol=1e-9)
        F.iterate(400_000)
        warm = [r["iter"] for r in F.residuals()]
    say(f"cold {cold} warm {warm}")
    assert all(w <= 0.1 * c + 20 for w, c in zip(warm, cold))


def test_mixed_family_reaches_optimum(small_family):
    fam = small_family
    thetas = [fam.theta(4000 + i, p=8) for i in range(64)]
    insts = family_members(fam, thetas)
    with Family(fam.m, fam.n, fam.row_ptr, fam.col_idx, fam.val, fam.c, B=64, precision="mixed",
                eps=1e-4) as F:
        F.set_rhs(np.stack([i["b"] for i in insts]))
        assert F.iterate(400_000) == 0
        res = F.residuals()
    for l in range(0, 64, 9):
        ro = oracle.Oracle.from_instance(insts[l]).solve(1e-5, check_every=50, max_iter=400_000)
        assert res[l]["kkt"] <= 1e-4
        assert abs(res[l]["pobj"] - ro["pobj"]) <= 2e-3 * (1 + abs(ro["pobj"]))


def _fam(fam, B=64, **kw):
    return Family(fam.m, fam.n, fam.row_ptr, fam.col_idx, fam.val, fam.c, B=B, **kw)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_refilled_member_equals_a_fresh_run(small_family, precision):
    """A member that enters a stopped slot mid-run (family_refill) follows
    bitwise the trajectory it has alone in a fresh family: same stopping
    iteration, residuals and iterates, whatever its slot and start time."""
    fam = small_family
    first = [fam.instance(fam.theta(3000 + i, p=8)) for i in range(6)]
    late = [fam.instance(fam.theta(3100 + i, p=8)) for i in range(4)]
    kw = dict(precision=precision, eps=1e-4, check_every=10, max_iter=20_000)
    with _fam(fam, **kw) as F:
        F.set_rhs(np.stack([i["b"] for i in first]))
        owner = list(range(6))          # member index per slot (late members are 100 + q)
        queue = list(range(4))
        res_late = {}
        sol_late = {}
        while True:
            active = F.iterate(50)
            res = F.residuals()
            stopped = [sl for sl in range(6) if res[sl]["status"] != "running" and owner[sl] is not None]
            for sl in stopped:
                if owner[sl] >= 100:
                    res_late[owner[sl] - 100] = res[sl]
                    sol_late[owner[sl] - 100] = {k: v[sl].copy() for k, v in F.solution().items()}
                owner[sl] = None
            take = [sl for sl in stopped][: len(queue)]
            if take:
                qs = [queue.pop(0) for _ in take]
                say(f"{precision}: refill slots {take} with late members {qs}")
                F.refill(take, np.stack([late[q]["b"] for q in qs]))
                for sl, q in zip(take, qs):
                    owner[sl] = 100 + q
                continue
            if active == 0 and not queue:
                break
    assert len(res_late) == 4
    for q in range(4):
        with _fam(fam, **kw) as G:
            G.set_rhs(late[q]["b"][None, :])
            while G.iterate(2000):
                pass
            r = G.residuals()[0]
            s = G.solution()
        say(f"late member {q}: refilled iter {res_late[q]['iter']} fresh iter {r['iter']}")
        assert res_late[q]["status"] == r["status"] == "converged"
        for k in ("iter", "kkt", "r_prim", "r_dual", "r_gap", "pobj", "dobj", "res_ax_b"):
            assert res_late[q][k] == r[k], k
        for k in KEYS:
            assert np.array_equal(sol_late[q][k], s[k][0]), k


def test_refill_with_predicted_start_matches_set_start_predicted(small_family):
    """The predicted start a refill gives a slot is the start
    family_set_start_predicted gives a fresh family: bitwise the same member
    after its 30 iterations (max_iter counts the member's own iterations)."""
    import torch
    fam = small_family
    a, b = fam.instance(fam.theta(3200, p=8)), fam.instance(fam.theta(3201, p=8))
    rng = np.random.default_rng(8)
    D = fam.n + fam.m
    xl = torch.from_numpy(rng.standard_normal((1, D)).astype(np.float32)).cuda()
    kw = dict(precision="fp64", eps=0.0, check_every=10, max_iter=30)
    with _fam(fam, **kw) as F:
        F.set_rhs(np.stack([a["b"], a["b"]]))
        assert F.iterate(100) == 0                   # both stop at max_iter 30
        F.refill([1], b["b"][None, :], dev_ptr=xl.data_ptr(), ld=D)
        assert F.iterate(100) == 0
        rr = F.residuals()[1]
        sr = {k: v[1] for k, v in F.solution().items()}
    with _fam(fam, **kw) as G:
        G.set_rhs(b["b"][None, :])
        G.set_start_predicted(xl.data_ptr(), D, "both")
        assert G.iterate(100) == 0
        rg = G.residuals()[0]
        sg = {k: v[0] for k, v in G.solution().items()}
    assert rr["status"] == rg["status"] == "max_iter" and rr["iter"] == rg["iter"] == 30
    for k in ("kkt", "pobj", "dobj", "res_ax_b"):
        assert rr[k] == rg[k], k
    for k in KEYS:
        assert np.array_equal(sr[k], sg[k]), k


def test_refilled_fp64_member_matches_oracle(small_family):
    fam = small_family
    a, b = fam.instance(fam.theta(3300, p=8)), fam.instance(fam.theta(3301, p=8))
    with _fam(fam, precision="fp64", eps=0.0, check_every=10, max_iter=200) as F:
        F.set_rhs(np.stack([a["b"], a["b"], a["b"]]))
        assert F.iterate(1000) == 0
        F.refill([2], b["b"][None, :])
        assert F.iterate(1000) == 0
        res = F.residuals()
        s = {k: v[2] for k, v in F.solution().items()}
    o = oracle.Oracle.from_instance(b)
    o.iterate(200)
    st = o.state()
    errs = {k: rel(s[k], st[k]) for k in KEYS}
    say(f"refilled member vs oracle after 200: {errs}")
    assert max(errs.values()) <= 1e-9
    assert res[2]["iter"] == 200 and res[0]["iter"] == 200


def test_refill_rejects_running_and_repeated_slots(small_family):
    fam = small_family
    a = fam.instance(fam.theta(3400, p=8))
    with _fam(fam, precision="fp64", eps=0.0, check_every=10, max_iter=20) as F:
        F.set_rhs(np.stack([a["b"]] * 3))
        with pytest.raises(Exception):
            F.refill([0], a["b"][None, :])                 # slot 0 still running
        F.iterate(100)
        with pytest.raises(Exception):
            F.refill([1, 1], np.stack([a["b"]] * 2))       # the same slot twice
        with pytest.raises(Exception):
            F.refill([3], a["b"][None, :])                 # beyond the current members
        F.refill([0, 2], np.stack([a["b"]] * 2))
        assert F.iterate(5) == 2


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_member_state_is_the_members_row_of_the_solution(small_family, precision):
    fam = small_family
    insts = family_members(fam, [fam.theta(4000 + i, p=8) for i in range(7)])
    with _fam(fam, precision=precision, eps=0.0, check_every=10) as F:
        F.set_rhs(np.stack([i["b"] for i in insts]))
        F.iterate(130)
        sol = F.solution()
        for sl in (0, 3, 6):
            st = F.member_state(sl)
            for k in KEYS:
                assert np.array_equal(st[k], sol[k][sl]), (sl, k)
        with pytest.raises(Exception):
            F.member_state(7)


def test_member_continues_on_the_single_problem_solver(small_family):
    """Hand-over of a running member: its state (family_member_state) taken
    into a solver_create handle of the same A and c whose b is the member's
    (solver_set_rhs + solver_resume) continues the run: after 150 more
    iterations it agrees with the member kept in the family, and with the
    oracle run on the member alone for all 270 iterations (FP64, 1e-9)."""
    from paper_2203_05027_amd.solver import Solver
    fam = small_family
    insts = family_members(fam, [fam.theta(4100 + i, p=8) for i in range(5)])
    with _fam(fam, precision="fp64", eps=0.0, check_every=10) as F:
        F.set_rhs(np.stack([i["b"] for i in insts]))
        F.iterate(120)
        st = F.member_state(2)
        F.iterate(150)
        kept = {k: v[2].copy() for k, v in F.solution().items()}
    other = insts[0]
    with Solver(fam.m, fam.n, fam.row_ptr, fam.col_idx, fam.val, other["b"], fam.c, fam.n, (),
                eps=0.0, check_every=10) as s:
        s.set_rhs(insts[2]["b"])
        s.resume(st["x"], st["z"], st["delta"], st["lambda"])
        s.iterate(150)
        moved = s.solution()
    o = oracle.Oracle.from_instance(insts[2])
    o.iterate(270)
    ref = o.state()
    for k in KEYS:
        assert rel(moved[k], kept[k]) <= 1e-9, (k, rel(moved[k], kept[k]))
        assert rel(moved[k], ref[k]) <= 1e-9, (k, rel(moved[k], ref[k]))


def test_stream_hand_over_keeps_every_member_and_its_count(small_family):
    """The streaming driver with the last running members handed to the
    single-problem solver against the driver without it: every member
    converges in both, and each member's iteration count agrees to within
    two checks (the hand-over continues the same iteration; only the order
    of FP32 additions differs)."""
    import torch  # noqa: F401
    from paper_2203_05027_amd.warmstart import WarmStart
    fam = small_family
    ws = WarmStart(fam, k=8, hidden=(32, 32), B=64, log=say)
    thetas = np.stack([fam.theta(5000 + i, p=8) for i in range(150)])
    b_all = np.ascontiguousarray(fam.b_many(thetas))
    with_h = ws.solve_stream(b_all, eps=1e-4, max_iter=100_000, tail_slots=16)
    without = ws.solve_stream(b_all, eps=1e-4, max_iter=100_000, tail_slots=0)
    say(f"hand-over: {with_h['handed_over']} members, {with_h['handover_iters']} iterations alone; "
        f"group iterations {with_h['group_iters']} vs {without['group_iters']}; "
        f"{with_h['seconds']:.2f} s vs {without['seconds']:.2f} s")
    assert with_h["converged"].all() and without["converged"].all()
    assert without["handed_over"] == 0 and with_h["handed_over"] >= 1
    assert np.abs(with_h["iters"] - without["iters"]).max() <= 20
    assert with_h["group_iters"] <= without["group_iters"]


def test_hand_over_falls_back_to_a_cold_solve(small_family):
    """A warm-started member handed to the single-problem solver that does
    not converge within the iterations it has left is solved again from the
    zero start, as in the group: its iterations add up, and the cold part
    is exactly a fresh handle's count."""
    import torch  # noqa: F401
    from paper_2203_05027_amd.solver import Solver
    from paper_2203_05027_amd.warmstart import WarmStart
    fam = small_family
    ws = WarmStart(fam, k=8, hidden=(32, 32), B=64, log=say)
    insts = family_members(fam, [fam.theta(6000 + i, p=8) for i in range(3)])
    b = np.stack([i["b"] for i in insts])
    tail = ws._tail_solver(b[0], 1e-4)
    try:
        with _fam(fam, precision="mixed", eps=1e-4, check_every=10) as F:
            F.set_rhs(b)
            F.iterate(20)
            ok, more = ws._finish_alone(tail, F, 1, b[1], 1e-4, 10, True, 100_000)
    finally:
        tail.close()
    with Solver(fam.m, fam.n, fam.row_ptr, fam.col_idx, fam.val, b[1], fam.c, fam.n, (), eps=1e-4,
                precision="mixed", check_every=10) as s:
        while not s.iterate(5000):
            pass
        cold = s.residuals()["iter"]
    say(f"hand-over fallback: {more} iterations alone, a fresh cold solve {cold}")
    assert ok and more == 10 + cold


def test_stream_hand_over_keeps_solutions():
    """The solutions the streaming driver keeps ([z ; lambda] rows, the
    training data of the learned start): members that stopped in the group
    are bitwise those of the driver without the hand-over; members finished
    on the single-problem solver are converged points of the same problems,
    z in the cone, and within the stopping tolerance's reach of the other
    run's point."""
    import torch
    from paper_2203_05027_amd.warmstart import WarmStart
    fam = I.ParametricFamily(m=300, n=600, k=5, p=8, seed=7)
    ws = WarmStart(fam, k=8, hidden=(32, 32), B=64, log=say)
    thetas = np.stack([fam.theta(7000 + i, p=8) for i in range(150)])
    b_all = np.ascontiguousarray(fam.b_many(thetas))
    keeps, runs = [], []
    for tail in (16, 0):
        keep = torch.zeros((len(thetas), ws.D), dtype=torch.float32, device="cuda")
        runs.append(ws.solve_stream(b_all, eps=1e-4, max_iter=100_000, keep=keep, tail_slots=tail))
        keeps.append(keep.cpu().numpy())
    with_h, without = runs
    assert with_h["handed_over"] >= 1 and with_h["converged"].all() and without["converged"].all()
    handed = np.zeros(len(thetas), bool)
    handed[with_h["handed_members"]] = True
    n = fam.n
    assert (keeps[0][:, :n] >= 0).all()
    # members that stopped in the group: the same iterates, bit for bit
    assert np.array_equal(keeps[0][~handed], keeps[1][~handed])
    assert np.array_equal(with_h["iters"][~handed], without["iters"][~handed])
    # members finished alone: the same iteration continued with another order of FP32 sums
    scale = np.abs(keeps[1][handed]).max(axis=1)
    diff = np.abs(keeps[0][handed] - keeps[1][handed]).max(axis=1) / scale
    say(f"kept rows: {int(handed.sum())} handed over, largest relative difference {diff.max():.2e}")
    assert diff.max() <= 5e-2, float(diff.max())
