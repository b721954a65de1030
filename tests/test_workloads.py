"""The synthetic workload definitions: sizes and parameter ranges of the
batch, the 4x circuit and the full-scale circuit, and reproducible draws."""
import numpy as np

from paper_2405_02019_amd import workloads


def test_batch_draws_are_in_range_and_reproducible():
    a = workloads.batch()
    b = workloads.batch()
    assert len(a) == 64
    assert [x.seed for x in a] == [x.seed for x in b]
    assert len({x.seed for x in a}) == 64
    s = np.array([x.scale for x in a])
    g = np.array([x.g for x in a])
    nu = np.array([x.bg_rate_hz for x in a])
    assert s.min() >= 0.05 and s.max() <= 0.2
    assert g.min() >= -6.0 and g.max() <= -3.0
    assert nu.min() >= 6.0 and nu.max() <= 10.0
    assert all(x.indegree_mode == 1 for x in a)
    assert workloads.batch(master_seed=2)[0].seed != a[0].seed


def test_full_and_x4():
    (f,) = workloads.full_scale()
    assert f.scale == 1.0 and f.indegree_mode == 0
    (x,) = workloads.stress_x4()
    assert x.scale == 4.0 and x.indegree_mode == 1
