"""End-to-end learned warm start on a small parametric family: the plain
method's solutions train the network, and its starts must cut the median
and the total iteration count to the 1e-4 KKT residual below the cold
start's on held-out members (every member still converges, the cold solve
being the fallback).  Members stream through the family solver's slots
(a stopped member's slot takes the next one), so the total iteration count
is what the wall time follows; both times are reported."""
import sys

import numpy as np
import pytest

from paper_2203_05027_amd import instances as I

pytestmark = pytest.mark.gpu


def say(msg):
    sys.__stderr__.write(f"[gpu-test] {msg}\n")
    sys.__stderr__.flush()


def test_learned_start_beats_cold_start():
    import torch
    from paper_2203_05027_amd.warmstart import WarmStart
    fam = I.ParametricFamily(m=400, n=800, k=5, p=16, seed=11)
    ws = WarmStart(fam, k=32, hidden=(128, 128), B=64, log=say)
    train = np.stack([fam.theta(10_000 + i, p=16) for i in range(1024)])
    test = np.stack([fam.theta(20_000 + i, p=16) for i in range(128)])
    Y, st = ws.solve_members(train, eps=1e-4, max_iter=200_000)
    say(f"training solves: {st['converged'].mean():.3f} converged, median iters {np.median(st['iters'])}")
    Yt = Y.clone()
    coef = ws.fit_basis(Y)
    hist = ws.train(train, coef, epochs=60, batch=128, lr=2e-3)
    assert hist[-1] < 0.5 * hist[0]
    err = ws.model_error(ws.predict(train[:128]), Yt[:128])
    say(f"train-set reconstruction error (median rel) {err:.3f}")
    cmp = ws.compare_stream(test, eps=1e-4, max_iter=200_000, parts=("both", "dual"), projection=True)
    cold, warm = cmp["cold"], cmp["both"]
    cm, wm = np.median(cold["iters"]), np.median(warm["iters"])
    say(f"held-out: cold median {cm} total {cold['iters'].sum()}, warm median {wm} total {warm['iters'].sum()}, "
        f"dual-only median {np.median(cmp['dual']['iters'])}, "
        f"basis projection of the solution median {np.median(cmp['projection']['iters'])}; "
        f"cold {cold['seconds']:.2f} s, warm {warm['seconds']:.2f} s (prediction {cmp['predict_seconds']:.3f} s)")
    for v in ("cold", "both", "dual", "projection"):
        assert cmp[v]["converged"].all(), v
    assert wm < cm
    assert warm["iters"].sum() < cold["iters"].sum()
    # the start a perfect network would give with this basis is at least as good
    assert np.median(cmp["projection"]["iters"]) <= cm
