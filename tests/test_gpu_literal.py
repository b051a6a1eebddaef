"""The literal (o-space) GPU form of Algorithm 1 against the oracle, which
runs the same algebra on the CPU, including y and gamma."""
import sys

import numpy as np
import pytest

import oracle
from paper_2203_05027_amd import instances as I
from paper_2203_05027_amd.solver import Literal, Solver

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30)) if b.size else 0.0


@pytest.mark.parametrize("shape", [(500, 1000, 5), (333, 777, 4), (2000, 4100, 10)])
def test_literal_matches_oracle(shape):
    inst = I.lp_instance(*shape, seed=31)
    orc = oracle.Oracle.from_instance(inst, mu=0.8)
    orc.iterate(200)
    o = orc.state()
    with Literal.from_instance(inst, mu=0.8) as L:
        L.iterate(200)
        g = L.solution()
    errs = {k: rel(g[k], o[k]) for k in ("x", "z", "delta", "lambda", "y", "gamma")}
    sys.__stderr__.write(f"[gpu-test] literal vs oracle {errs}\n")
    assert max(errs.values()) <= 1e-9, errs


def test_literal_equals_reduced_form():
    inst = I.lp_instance(800, 1700, 6, seed=32)
    with Literal.from_instance(inst) as L, Solver.from_instance(inst, eps=0.0) as S:
        L.iterate(300)
        S.iterate(300)
        a, b = L.solution(), S.solution()
    for k in ("x", "z", "delta", "lambda"):
        assert rel(a[k], b[k]) <= 1e-9, k
