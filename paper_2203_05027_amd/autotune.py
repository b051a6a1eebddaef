"""Tile search for the batched solver, with a JSON cache.

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
LANE_PAIRS = ((1, 1), (2, 1), (4, 1), (2, 2), (4, 2), (8, 2), (8, 4))


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
