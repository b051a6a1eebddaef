"""The residual history: every check of the iteration (Section V-B's
residuals) recorded on the device, read back oldest first.  Records match
the oracle's residuals at the same iterations, the ring keeps the latest
records when it wraps, a new start clears it, and the times are the GPU's
clock in order."""
import sys

import numpy as np
import pytest

import oracle
from paper_2203_05027_amd import instances as I
from paper_2203_05027_amd.solver import Solver

pytestmark = pytest.mark.gpu

FIELDS = ("r_prim", "r_dual", "r_gap", "kkt", "pobj", "dobj", "res_ax_b", "gap_x")


def say(msg):
    sys.__stderr__.write(f"[gpu-test] {msg}\n")
    sys.__stderr__.flush()


def _instances():
    return {"lp": I.lp_instance(300, 700, 5, seed=31),
            "socp": I.socp_instance(60, 6, seed=32)}


_INST = {}


def inst_of(kind):
    if not _INST:
        _INST.update(_instances())
    return _INST[kind]


@pytest.mark.parametrize("kind,resident", [("lp", "auto"), ("lp", "never"), ("socp", "auto")])
def test_history_matches_oracle_checks(kind, resident):
    inst = inst_of(kind)
    every, checks = 10, 12
    orc = oracle.Oracle.from_instance(inst)
    want = []
    for _ in range(checks):
        orc.iterate(every)
        want.append(orc.residuals())
    orc.close()
    with Solver.from_instance(inst, eps=0.0, check_every=every, resident=resident, history=64) as s:
        say(f"history {kind} {resident}: shape {s.launch_shape()}")
        s.iterate(every * checks)
        h = s.history()
    assert [r["iter"] for r in h] == [every * (q + 1) for q in range(checks)]
    for q, (got, ref) in enumerate(zip(h, want)):
        for f in FIELDS[:-1]:
            assert got[f] == pytest.approx(ref[f], rel=1e-9, abs=1e-12), (q, f, got[f], ref[f])
        # gap_x = |c'x + b'lambda| = |pobj_x - dobj|, a difference of two
        # objectives: its error is theirs
        scale = 1.0 + abs(ref["pobj_x"]) + abs(ref["dobj"])
        assert abs(got["gap_x"] - abs(ref["pobj_x"] - ref["dobj"])) <= 1e-9 * scale, (q, got["gap_x"])
    t = [r["seconds"] for r in h]
    assert t[0] >= 0.0 and all(b >= a for a, b in zip(t, t[1:])), t


@pytest.mark.parametrize("resident", ["auto", "never"])
def test_ring_keeps_the_latest_records(resident):
    inst = inst_of("lp")
    with Solver.from_instance(inst, eps=0.0, check_every=10, resident=resident, history=256) as s:
        s.iterate(230)
        full = s.history()
    with Solver.from_instance(inst, eps=0.0, check_every=10, resident=resident, history=5) as s:
        s.iterate(230)
        ring = s.history()
        part = s.history(3)
        assert s.history(0) == []
    assert len(full) == 23 and [r["iter"] for r in ring] == [190, 200, 210, 220, 230]
    for a, b in zip(ring, full[-5:]):
        assert all(a[f] == b[f] for f in FIELDS + ("iter",))
    assert [r["iter"] for r in part] == [210, 220, 230]


def test_history_records_checks_only_and_a_new_start_clears_it():
    """Records come from the iteration's own checks: a residual query between
    checks adds none; set_start begins a new history; the last record is the
    check that stopped the run."""
    inst = inst_of("lp")
    with Solver.from_instance(inst, eps=1e-3, check_every=10, resident="never", history=4096) as s:
        s.iterate(25)
        s.residuals()
        assert [r["iter"] for r in s.history()] == [10, 20]
        s.set_start()
        assert s.history() == []
        done = s.iterate(100_000)
        h = s.history()
        r = s.residuals()
    assert done and r["status"] == "converged"
    assert h[-1]["iter"] == r["iter"] and h[-1]["kkt"] == r["kkt"] and h[-1]["kkt"] <= 1e-3
    assert all(x["kkt"] > 1e-3 for x in h[:-1])


def test_no_history_without_the_option():
    with Solver.from_instance(inst_of("lp"), eps=0.0, check_every=10) as s:
        s.iterate(50)
        assert s.history(10) == []
