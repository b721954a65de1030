"""Pins of the spike statistics helpers on rasters with known answers."""
import numpy as np

from spike_stats import cv_isi, first_divergence, rates_hz


def test_rates_and_cv_of_known_trains():
    rng = np.random.default_rng(0)
    off = np.array([0, 100, 300])
    steps, ids = [], []
    for i in range(100):                   # population 0: regular, every 50 steps (200 Hz)
        s = np.arange(7 + i % 50, 100000, 50)
        steps.append(s); ids.append(np.full(len(s), i))
    for i in range(100, 300):              # population 1: Poisson at 20 Hz
        n = rng.poisson(20 * 10.0)
        s = np.sort(rng.choice(100000, n, replace=False))
        steps.append(s); ids.append(np.full(len(s), i))
    s = np.concatenate(steps).astype(np.uint32)
    i = np.concatenate(ids).astype(np.uint32)
    o = np.lexsort((i, s))
    s, i = s[o], i[o]
    r = rates_hz(s, i, off, 0, 100000)
    assert abs(r[0] - 200.0) < 0.5 and abs(r[1] - 20.0) < 1.0
    c = cv_isi(s, i, off, 0, 100000)
    assert c[0] == 0.0 and abs(c[1] - 1.0) < 0.05


def test_first_divergence():
    a_s = np.array([1, 2, 2, 5], np.uint32); a_i = np.array([3, 1, 4, 0], np.uint32)
    assert first_divergence(a_s, a_i, a_s.copy(), a_i.copy()) is None
    b_i = a_i.copy(); b_i[2] = 5
    assert first_divergence(a_s, a_i, a_s, b_i) == 2
    assert first_divergence(a_s[:3], a_i[:3], a_s, a_i) == 5


def test_step_digest_locates_first_difference():
    from spike_stats import first_digest_divergence, step_digest
    s = np.array([0, 0, 3, 3, 4], np.uint32); i = np.array([1, 2, 0, 7, 5], np.uint32)
    d = step_digest(s, i, 6)
    assert d.tolist() == [[2, 3, 5], [0, 0, 0], [0, 0, 0], [2, 7, 49], [1, 5, 25], [0, 0, 0]]
    assert first_digest_divergence(d, d.copy()) is None
    i2 = i.copy(); i2[3] = 6
    assert first_digest_divergence(d, step_digest(s, i2, 6)) == 3
    assert first_digest_divergence(d, step_digest(s[:4], i[:4], 6)) == 4


def test_kde_and_kl_against_closed_forms():
    from spike_stats import kde_on_grid, kl_divergence
    rng = np.random.default_rng(1)
    grid = np.linspace(-8, 10, 4001)
    a = kde_on_grid(rng.normal(0.0, 1.0, 20000), grid)
    b = kde_on_grid(rng.normal(1.0, 1.0, 20000), grid)
    assert abs(np.trapezoid(a, grid) - 1.0) < 1e-9
    assert kl_divergence(a, a, grid) == 0.0
    # KL(N(0,1) || N(1,1)) = 1/2; the KDE widens both by the same bandwidth
    assert abs(kl_divergence(a, b, grid) - 0.5) < 0.06


def test_pearson_of_identical_and_independent_trains():
    from spike_stats import pearson_samples
    rng = np.random.default_rng(2)
    steps, ids = [], []
    base = np.sort(rng.choice(100000, 800, replace=False))
    for i in range(10):                      # ten copies of one train: r = 1
        steps.append(base); ids.append(np.full(len(base), i))
    for i in range(10, 40):                  # independent Poisson trains: r ~ 0
        s = np.sort(rng.choice(100000, 800, replace=False))
        steps.append(s); ids.append(np.full(len(s), i))
    s = np.concatenate(steps); i = np.concatenate(ids)
    r = pearson_samples(s, i, 0, 10, 0, 100000, n_sample=10)
    np.testing.assert_allclose(r, 1.0, atol=1e-12)
    r = pearson_samples(s, i, 10, 40, 0, 100000, n_sample=30)
    assert abs(r.mean()) < 0.01 and r.std() < 0.05


def test_kde_bandwidth_is_scotts_rule():
    """A Gaussian KDE is a mixture of N(x_i, h^2): its variance is the sample
    variance plus h^2, with Scott's h^2 = n^(-2/5) times the unbiased sample
    variance in one dimension."""
    from spike_stats import kde_on_grid
    rng = np.random.default_rng(3)
    x = rng.gamma(2.0, 1.0, 500)
    grid = np.linspace(x.min() - 10, x.max() + 10, 20001)
    p = kde_on_grid(x, grid)
    mean = np.trapezoid(p * grid, grid)
    var = np.trapezoid(p * (grid - mean) ** 2, grid)
    expect = x.var() + len(x) ** -0.4 * x.var(ddof=1)
    assert abs(mean - x.mean()) < 1e-6
    assert abs(var / expect - 1.0) < 1e-5
