"""The random-gather probe behind the gather floor of the benchmark."""
import math

import pytest

from paper_2203_05027_amd.solver import probe_gather

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fp64", [True, False])
def test_probe_times_a_launch(fp64):
    ms = probe_gather(1_000_003, 262_147, 4, fp64, reps=5)
    assert math.isfinite(ms) and 0.0 < ms < 100.0


def test_probe_rate_falls_with_the_table():
    """Gathers from a part that fits one XCD's L2 are served faster than
    gathers spread over 128 MiB (the premise of the slab layout)."""
    small = probe_gather(20_000_000, 1 << 18, 1, True)      # 2 MiB table
    large = probe_gather(20_000_000, 1 << 24, 1, True)      # 128 MiB table
    assert small < large
