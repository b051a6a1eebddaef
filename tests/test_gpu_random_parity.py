"""Randomised GPU parity: many small problems drawn by hypothesis (shapes,
cone mixes with sizes 1..300, empty rows, mu, launch options, start points),
the HIP solver against the FP64 oracle after a few dozen iterations at the
1e-9 bar, and batches of such problems in every pass form.

The bar is relative to the largest entry of the oracle's whole state
(x, z, delta, lambda) rather than of each vector: after a step in which the
projection is the identity, delta = delta + mu (z - x) cancels to rounding
noise of the previous delta on both sides, and a per-vector ratio of two
such noises says nothing."""
import sys

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import oracle
from paper_2203_05027_amd import instances as I
from paper_2203_05027_amd.solver import Batch, Solver

pytestmark = pytest.mark.gpu
KEYS = ("x", "z", "delta", "lambda")
SETTINGS = settings(max_examples=200, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])


def say(msg):
    sys.__stderr__.write(f"[gpu-test] {msg}\n")
    sys.__stderr__.flush()


def errors(g, o):
    scale = max(max((float(np.abs(o[k]).max()) if o[k].size else 0.0) for k in KEYS), 1e-30)
    return {k: (float(np.abs(g[k] - o[k]).max()) / scale if o[k].size else 0.0) for k in KEYS}


def empty_rows(inst, rows):
    """The instance with the listed rows emptied (b kept consistent with x0)."""
    m = inst["m"]
    r = np.repeat(np.arange(m), np.diff(inst["row_ptr"]))
    keep = ~np.isin(r, rows)
    rr, cc, vv = r[keep], inst["col_idx"][keep], inst["val"][keep]
    row_ptr = np.zeros(m + 1, np.int64)
    np.cumsum(np.bincount(rr, minlength=m), out=row_ptr[1:])
    b = np.zeros(m)
    np.add.at(b, rr, vv * inst["x0"][cc])
    return dict(inst, row_ptr=row_ptr, col_idx=cc.astype(np.int32), val=vv, nnz=int(rr.size), b=b)


@st.composite
def problems(draw):
    n_orth = draw(st.integers(0, 300))
    sizes = draw(st.lists(st.integers(1, 300), max_size=6))
    if n_orth + sum(sizes) == 0:
        n_orth = 1
    n = n_orth + sum(sizes)
    m = draw(st.integers(1, max(1, min(400, n - 1)) if n > 1 else 1))
    k = draw(st.integers(1, min(4, m)))
    seed = draw(st.integers(0, 10_000))
    inst = I.conic_instance(m, n_orth, sizes, k, seed=seed)
    if m > 2 and draw(st.booleans()):
        inst = empty_rows(inst, draw(st.lists(st.integers(0, m - 1), max_size=3)))
    return inst


@SETTINGS
@given(inst=problems(), mu=st.sampled_from([0.3, 1.0, 2.5]), opts=st.sampled_from([
    {}, {"slabs_row": 2, "slabs_col": 4}, {"slabs_row": 8, "slabs_col": 2, "slab_kernel": "chunked4"},
    {"lanes_row": 1, "lanes_col": 64, "unroll_row": 1, "unroll_col": 4}, {"use_graph": False},
    {"slabs_row": 4, "slabs_col": 1, "slab_kernel": "lanes"}]), warm=st.booleans(), data=st.data())
def test_random_problems_match_oracle(inst, mu, opts, warm, data):
    iters = data.draw(st.integers(1, 40), "iters")
    say(f"m={inst['m']} n={inst['n']} nnz={inst['nnz']} cones={len(inst['soc_sizes'])} mu={mu} {opts} "
        f"warm={warm} iters={iters}")
    orc = oracle.Oracle.from_instance(inst, mu=mu)
    with Solver.from_instance(inst, mu=mu, eps=0.0, check_every=7, **opts) as s:
        if warm:
            rng = np.random.default_rng(inst["seed"])
            start = (rng.standard_normal(inst["n"]), rng.standard_normal(inst["n"]),
                     rng.standard_normal(inst["n"]), rng.standard_normal(inst["m"]))
            orc.set_start(*start)
            s.set_start(*start)
        orc.iterate(iters)
        s.iterate(iters)
        g = s.solution()
    errs = errors(g, orc.state())
    assert max(errs.values()) <= 1e-9, errs


@SETTINGS
@given(data=st.data(), mu=st.sampled_from([0.3, 1.0, 2.5]), warm=st.booleans(),
       precision=st.sampled_from(["fp64", "mixed"]))
def test_random_resident_problems_match_oracle(data, mu, warm, precision):
    """The resident path on drawn orthant problems (ragged shapes, emptied
    rows, any check interval), warm or cold: FP64 at the 1e-9 bar, the mixed
    form against its own sweep kernels (resident off) at FP32 rounding."""
    m = data.draw(st.integers(1, 450), "m")
    n = data.draw(st.integers(1, 900), "n")
    k = data.draw(st.integers(1, min(4, m)), "k")
    inst = I.lp_instance(m, n, k, seed=data.draw(st.integers(0, 10_000), "seed"))
    if m > 2 and data.draw(st.booleans(), "holes"):
        inst = empty_rows(inst, data.draw(st.lists(st.integers(0, m - 1), max_size=3), "rows"))
    iters = data.draw(st.integers(1, 60), "iters")
    ce = data.draw(st.integers(1, 12), "check_every")
    say(f"resident m={m} n={n} nnz={inst['nnz']} mu={mu} warm={warm} {precision} iters={iters} ce={ce}")
    start = None
    if warm:
        rng = np.random.default_rng(inst["seed"])
        start = (rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(m))
    outs = {}
    for path in ("required", "never") if precision == "mixed" else ("required",):
        with Solver.from_instance(inst, mu=mu, eps=0.0, check_every=ce, precision=precision, resident=path) as s:
            assert s.launch_shape()["resident"] == (path == "required")
            if start is not None:
                s.set_start(*start)
            s.iterate(iters)
            outs[path] = s.solution()
    if precision == "fp64":
        orc = oracle.Oracle.from_instance(inst, mu=mu)
        if start is not None:
            orc.set_start(*start)
        orc.iterate(iters)
        errs = errors(outs["required"], orc.state())
        assert max(errs.values()) <= 1e-9, errs
    else:
        errs = errors(outs["required"], outs["never"])
        assert max(errs.values()) <= 1e-4, errs


@SETTINGS
@given(data=st.data())
def test_random_batches_match_oracle(data):
    count = data.draw(st.integers(1, 6), "count")
    insts = []
    for q in range(count):
        m = data.draw(st.integers(1, 700), "m")
        n = data.draw(st.integers(max(1, m // 2), 2 * m + 3), "n")
        k = data.draw(st.integers(1, min(5, m)), "k")
        inst = I.lp_instance(m, n, k, seed=data.draw(st.integers(0, 10_000), "seed"))
        if m > 2 and data.draw(st.booleans(), "holes"):
            inst = empty_rows(inst, data.draw(st.lists(st.integers(0, m - 1), max_size=3), "rows"))
        insts.append(inst)
    threads = data.draw(st.sampled_from([64, 256, 1024]), "threads")
    lanes = [data.draw(st.sampled_from([1, 2, 4, 8]), "lr") if i % 2 == 0
             else data.draw(st.sampled_from([0, 1, 2, 4]), "lc") for i in range(8)]
    lanes = [min(v, threads) for v in lanes]
    iters = data.draw(st.integers(1, 40), "iters")
    say(f"batch of {count}: m={[i['m'] for i in insts]} threads={threads} lanes={lanes} iters={iters}")
    with Batch(insts, precision="fp64", eps=0.0, check_every=6) as b:
        b.set_tiles(threads, lanes)
        b.iterate(iters)
        for i, inst in enumerate(insts):
            o = oracle.Oracle.from_instance(inst)
            o.iterate(iters)
            errs = errors(b.solution(i), o.state())
            assert max(errs.values()) <= 1e-9, (i, errs)


STD_KEYS = ("x1", "x2", "lam", "nu", "delta")


@settings(max_examples=100, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(data=st.data())
def test_random_standard_problems_match_oracle(data):
    """The standard-ADMM + CG baseline on drawn problems with m well below n
    (A A' nonsingular: a singular one makes the CG solve ill-posed, see the
    baseline's own tests), cone mixes, CG depth and mu, against its oracle."""
    from oracle import standard as std_oracle
    from paper_2203_05027_amd.solver import Standard
    m = data.draw(st.integers(1, 150), "m")
    n_orth = data.draw(st.integers(0, 200), "n_orth")
    sizes = data.draw(st.lists(st.integers(1, 120), max_size=4), "sizes")
    short = 2 * m + 1 - (n_orth + sum(sizes))
    if short > 0:
        n_orth += short
    k = data.draw(st.integers(2, min(4, m)) if m >= 2 else st.just(1), "k")
    inst = I.conic_instance(m, n_orth, sizes, k, seed=data.draw(st.integers(0, 10_000), "seed"))
    mu = data.draw(st.sampled_from([0.5, 1.0, 3.0]), "mu")
    cg = data.draw(st.sampled_from([1, 2, 5]), "cg")
    iters = data.draw(st.integers(1, 20), "iters")
    orc = std_oracle.StandardADMM.from_instance(inst, mu=mu, cg_iters=cg, cg_tol=0.0)
    orc.iterate(iters)
    o = orc.state()
    with Standard.from_instance(inst, mu=mu, cg_iters=cg, cg_tol=0.0, eps=0.0, check_every=5) as s:
        s.iterate(iters)
        g = s.solution()
    scale = max(max(float(np.abs(o[key]).max()) for key in STD_KEYS), 1e-30)
    errs = {key: float(np.abs(g[key] - o[key]).max()) / scale for key in STD_KEYS}
    assert max(errs.values()) <= 1e-9, (inst["m"], inst["n"], errs)


@settings(max_examples=40, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(data=st.data())
def test_random_families_match_oracle(data):
    """Parametric families (one A and c, many b) of drawn shapes, group sizes
    and member counts, every member against its own oracle run."""
    from paper_2203_05027_amd.solver import Family
    m = data.draw(st.integers(1, 200), "m")
    n = data.draw(st.integers(m + 1, 2 * m + 50), "n")
    k = data.draw(st.integers(1, min(4, m)), "k")
    fam = I.ParametricFamily(m=m, n=n, k=k, p=4, seed=data.draw(st.integers(0, 10_000), "seed"))
    B = data.draw(st.sampled_from([64, 128]), "B")
    nb = data.draw(st.integers(1, B), "nb")
    iters = data.draw(st.integers(1, 30), "iters")
    insts = [fam.instance(fam.theta(5000 + i, p=4)) for i in range(nb)]
    with Family(fam.m, fam.n, fam.row_ptr, fam.col_idx, fam.val, fam.c, B=B, precision="fp64",
                eps=0.0, check_every=4) as F:
        F.set_rhs(np.stack([i["b"] for i in insts]))
        F.iterate(iters)
        sol = F.solution()
    for l in sorted({0, nb // 2, nb - 1}):
        o = oracle.Oracle.from_instance(insts[l])
        o.iterate(iters)
        st_ = o.state()
        errs = errors({key: sol[key][l] for key in KEYS}, st_)
        assert max(errs.values()) <= 1e-9, (l, errs)


@settings(max_examples=100, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])
@given(data=st.data())
def test_random_literal_problems_match_oracle(data):
    """Algorithm 1 as printed (y and gamma per nonzero) on drawn LPs, emptied
    rows included, against the oracle, y and gamma compared too."""
    from paper_2203_05027_amd.solver import Literal
    m = data.draw(st.integers(1, 400), "m")
    n = data.draw(st.integers(1, 2 * m + 20), "n")
    k = data.draw(st.integers(1, min(5, m)), "k")
    inst = I.lp_instance(m, n, k, seed=data.draw(st.integers(0, 10_000), "seed"))
    if m > 2 and data.draw(st.booleans(), "holes"):
        inst = empty_rows(inst, data.draw(st.lists(st.integers(0, m - 1), max_size=3), "rows"))
    mu = data.draw(st.sampled_from([0.4, 1.0, 2.0]), "mu")
    iters = data.draw(st.integers(1, 30), "iters")
    orc = oracle.Oracle.from_instance(inst, mu=mu)
    orc.iterate(iters)
    o = orc.state()
    with Literal.from_instance(inst, mu=mu) as L:
        L.iterate(iters)
        g = L.solution()
    keys = ("x", "z", "delta", "lambda", "y", "gamma")
    scale = max(max((float(np.abs(o[key]).max()) if o[key].size else 0.0) for key in keys), 1e-30)
    errs = {key: (float(np.abs(g[key] - o[key]).max()) / scale if o[key].size else 0.0) for key in keys}
    assert max(errs.values()) <= 1e-9, errs
