"""solver_solve_noalloc (every device buffer in a fixed scratch array, no
allocation) against solver_solve through the C ABI: bitwise the same
outputs and residuals on two calls in a row, the second with a smaller
problem, in both precisions; FP64 iterates against the oracle; a problem
beyond the scratch is rejected with UV_ENOSCRATCH before any device work,
and calls after a rejection still work."""
import sys

import numpy as np
import pytest

import oracle
from paper_2203_05027_amd import instances as I
from paper_2203_05027_amd.solver import UV_ENOSCRATCH, UV_ENUMERIC, solve

pytestmark = pytest.mark.gpu
KEYS = ("x", "z", "delta", "lambda")


def say(msg):
    sys.__stderr__.write(f"[gpu-test] {msg}\n")
    sys.__stderr__.flush()


def _same(a, b):
    rc_a, sa, ra = a
    rc_b, sb, rb = b
    assert rc_a == rc_b
    for k in KEYS:
        assert np.array_equal(sa[k], sb[k]), k
    assert ra == rb


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_equals_solve_on_two_calls(precision):
    big = I.config_instance("lp_small")
    small = I.lp_instance(120, 260, 3, seed=5)
    for inst in (big, small):   # the second call is the smaller one
        say(f"noalloc {precision} m={inst['m']} n={inst['n']} nnz={inst['nnz']}")
        a = solve(inst, 3000, precision=precision, eps=1e-4)
        b = solve(inst, 3000, noalloc=True, precision=precision, eps=1e-4)
        assert a[0] == 0
        _same(a, b)
        say(f"  iter {b[2]['iter']} status {b[2]['status']} kkt {b[2]['kkt']:.3e}")


def test_noalloc_matches_oracle():
    inst = I.lp_instance(333, 777, 4, seed=17)
    orc = oracle.Oracle.from_instance(inst, mu=0.8)
    orc.iterate(200)
    o = orc.state()
    rc, g, r = solve(inst, 200, noalloc=True, mu=0.8, eps=0.0)
    assert rc == 0 and r["iter"] == 200
    for k in KEYS:
        err = float(np.abs(g[k] - o[k]).max() / max(np.abs(o[k]).max(), 1e-30))
        assert err <= 1e-9, (k, err)


def test_noalloc_rejects_what_does_not_fit():
    big = I.lp_instance(5000, 10_000, 6, seed=1)
    rc, _, _ = solve(big, 10, noalloc=True)
    assert rc == UV_ENOSCRATCH
    soc = I.socp_instance(20, 4, seed=2)
    rc, _, _ = solve(soc, 10, noalloc=True)
    assert rc == UV_ENOSCRATCH
    inst = I.lp_instance(60, 130, 4, seed=2)
    _same(solve(inst, 500, eps=1e-4), solve(inst, 500, noalloc=True, eps=1e-4))


def test_noalloc_max_iter_and_numeric_stop():
    inst = I.lp_instance(60, 130, 4, seed=2)
    a = solve(inst, 1000, eps=1e-12, max_iter=25)
    b = solve(inst, 1000, noalloc=True, eps=1e-12, max_iter=25)
    _same(a, b)
    assert b[2]["status"] == "max_iter" and b[2]["iter"] == 25
    c = inst["c"].copy()
    c[17] = np.nan
    bad = dict(inst, c=c)
    a = solve(bad, 100, eps=1e-4)
    b = solve(bad, 100, noalloc=True, eps=1e-4)
    assert a[0] == b[0] == UV_ENUMERIC
    assert b[2]["status"] == "numeric" and b[2]["iter"] == 10
