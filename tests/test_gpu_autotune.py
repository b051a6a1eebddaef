"""The launch-shape searches: slab counts of the single-problem solver."""
import pytest

from paper_2203_05027_amd import autotune
from paper_2203_05027_amd import instances as I

pytestmark = pytest.mark.gpu


def test_slab_search_picks_the_fastest_measured_count(tmp_path):
    inst = I.lp_instance(300_000, 600_000, 8, seed=51)
    cache = str(tmp_path / "tiles.json")
    rec = autotune.tune_slabs(inst, "fp64", iters=10, cache_path=cache)
    assert not rec["cached"]
    trials = rec["trials"]
    assert {t["slabs"] for t in trials} == {1, 2, 4, 8}
    assert rec["ms_row"] == min(t["ms_row"] for t in trials)
    assert rec["ms_col"] == min(t["ms_col"] for t in trials)
    again = autotune.tune_slabs(inst, "fp64", iters=10, cache_path=cache)
    assert again["cached"] and again["slabs_row"] == rec["slabs_row"] and again["slabs_col"] == rec["slabs_col"]
