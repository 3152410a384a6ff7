"""The trace's algorithmic FLOP model in bench.py: the alive fractions and
Newton iteration counts it takes for each workload equal what the oracle
counts on the same sample (CPU only)."""
import numpy as np
import pytest

import bench
from flop_counts import count, paper_map_sample
from workloads import configs


@pytest.mark.parametrize("name", ["config5", "config2", "paper_map"])
def test_trace_counts_match_the_oracle(name):
    if name == "paper_map":
        lens, query = paper_map_sample()
        alive, newton = count(lens, query, per_axis=(96, 8))
    else:
        lens, sensor, query = getattr(configs, name)(rays=64)
        alive, newton = count(lens, query)
    c = bench.TRACE_COUNTS[name]
    assert len(c["alive"]) == len(lens.surfaces)
    assert np.allclose(alive, c["alive"], atol=1e-4)
    assert newton == pytest.approx(c["newton_per_ray"], abs=2e-3)
    # launched rays die, they are not created: the fractions never rise
    assert np.all(np.diff(alive) <= 0) and alive[0] == 1.0


def test_flop_per_ray_of_a_spherical_lens():
    # every ray alive at every surface: 60 + 56 per sphere + 10 per stop
    kinds = [0, 0, 2, 0]
    assert bench.trace_flop_per_ray(kinds, [1.0] * 4, 0.0) == 60 + 3 * 56 + 10
    # an asphere adds its fixed part and 48 per Newton iteration
    assert bench.trace_flop_per_ray([3], [1.0], 2.5) == 60 + 78 + 2.5 * 48
