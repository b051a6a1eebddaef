"""Launch-shape searches, with a JSON cache: tiles of the batched solver
(``tune``) and XCD slab counts of the single-problem solver (``tune_slabs``).

The measurement runs in the library (``batch_time``: one timed launch of a
size bucket's instances from a saved copy of the state, put back after); the
search here picks, per size bucket, the lanes per row and per column that
give the shortest launch, then the workgroup size that gives the shortest
launch over all buckets.  Results are cached by precision and by the
bucket mix of the batch (counts rounded to powers of two), so a batch of the
same shape reuses them.
"""
from __future__ import annotations

import json
import math
import os

DEFAULT_CACHE = os.environ.get(
    "UVADMM_TILE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "uvadmm", "tiles.json"))

THREADS = (256, 512, 1024)
# (lanes per row, lanes per column); lanes per column 0 = the sliced column
# copy (a wavefront per 64 columns, coalesced entry loads)
LANE_PAIRS = ((1, 1), (2, 1), (4, 1), (2, 2), (4, 2), (8, 2), (8, 4), (1, 0), (2, 0), (4, 0), (8, 0))


def signature(batch) -> str:
    counts = batch.bucket_counts()
    rounded = [0 if c == 0 else 2 ** round(math.log2(c)) for c in counts]
    return f"{batch.precision}|buckets={rounded}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tune(batch, iters: int = 20, cache_path: str | None = DEFAULT_CACHE, threads=THREADS,
         lane_pairs=LANE_PAIRS, log=None) -> dict:
    """Chooses and applies tiles for ``batch``; returns the record."""
    key = signature(batch)
    cache = _load(cache_path) if cache_path else {}
    if key in cache:
        rec = cache[key]
        batch.set_tiles(rec["threads"], rec["lanes"])
        rec = dict(rec, cached=True)
        return rec
    counts = batch.bucket_counts()
    best_overall = None
    trials = []
    for t in threads:
        lanes = [2, 1] * 4
        for bk in range(4):
            if counts[bk] == 0:
                continue
            best = None
            for lr, lc in lane_pairs:
                if lr > t or lc > t:
                    continue
                trial = list(lanes)
                trial[2 * bk], trial[2 * bk + 1] = lr, lc
                batch.set_tiles(t, trial)
                ms = batch.time(bk, iters)
                trials.append({"threads": t, "bucket": bk, "lanes": [lr, lc], "ms": ms})
                if best is None or ms < best[0]:
                    best = (ms, lr, lc)
            lanes[2 * bk], lanes[2 * bk + 1] = best[1], best[2]
        batch.set_tiles(t, lanes)
        total = batch.time(-1, iters)
        trials.append({"threads": t, "bucket": -1, "lanes": lanes, "ms": total})
        if log:
            log(f"threads={t} lanes={lanes} all-bucket launch {total:.3f} ms")
        if best_overall is None or total < best_overall["ms"]:
            best_overall = {"threads": t, "lanes": lanes, "ms": total, "iters": iters}
    batch.set_tiles(best_overall["threads"], best_overall["lanes"])
    if cache_path:
        cache = _load(cache_path)
        cache[key] = best_overall
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return dict(best_overall, cached=False, trials=trials)


SLABS = (1, 2, 4, 8)


def slab_signature(inst, precision: str) -> str:
    """Shape key of a single problem: sizes rounded to powers of two, cone mix."""
    def r(v):
        return 0 if v <= 0 else 2 ** round(math.log2(v))
    soc = inst.get("soc_sizes")
    cones = "orthant" if soc is None or len(soc) == 0 else f"soc{r(len(soc))}"
    return f"slabs|{precision}|m={r(inst['m'])}|n={r(inst['n'])}|nnz={r(inst['nnz'])}|{cones}"


def tune_slabs(inst, precision: str = "fp64", iters: int = 20, cache_path: str | None = DEFAULT_CACHE,
               slabs=SLABS, log=None) -> dict:
    """Times the column and row passes of ``inst`` (solver_time_kernels) for
    every slab count of the gathered vectors and returns the fastest pair
    {"slabs_row", "slabs_col", "ms_row", "ms_col"}; the two passes are
    independent, so each count is chosen on its own pass.  Cached by shape."""
    from .solver import Solver

    key = slab_signature(inst, precision)
    cache = _load(cache_path) if cache_path else {}
    if key in cache:
        return dict(cache[key], cached=True)
    best_row = best_col = None
    trials = []
    for S in slabs:
        if S > 1 and (S > inst["m"] or S > inst["n"]):
            continue
        with Solver.from_instance(inst, precision=precision, eps=0.0, slabs_row=S, slabs_col=S) as s:
            s.iterate(2)
            ms_col, ms_row = s.time_kernels(iters)
        trials.append({"slabs": S, "ms_row": ms_row, "ms_col": ms_col})
        if log:
            log(f"slabs={S}: row pass {ms_row:.4f} ms, column pass {ms_col:.4f} ms")
        if best_row is None or ms_row < best_row[1]:
            best_row = (S, ms_row)
        if best_col is None or ms_col < best_col[1]:
            best_col = (S, ms_col)
    rec = {"slabs_row": best_row[0], "slabs_col": best_col[0], "ms_row": best_row[1], "ms_col": best_col[1],
           "iters": iters}
    if cache_path:
        cache = _load(cache_path)
        cache[key] = rec
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return dict(rec, cached=False, trials=trials)
