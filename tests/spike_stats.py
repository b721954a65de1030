"""Spike-train statistics used to compare simulations that are not expected to
agree spike for spike (the FP64 oracle against the FP32/int32 paths): the
population rates and coefficients of variation of inter-spike intervals of
Sec. 4.1, and the first step at which two rasters differ."""
import numpy as np

DT_S = 1e-4


def population_of(ids, offsets):
    return np.searchsorted(offsets, ids, side="right") - 1


def rates_hz(steps, ids, offsets, t0, t1):
    """Mean firing rate per population over steps [t0, t1)."""
    m = (steps >= t0) & (steps < t1)
    pop = population_of(ids[m], offsets)
    counts = np.bincount(pop, minlength=len(offsets) - 1)[: len(offsets) - 1]
    sizes = np.diff(offsets)
    return counts / sizes / ((t1 - t0) * DT_S)


def cv_isi(steps, ids, offsets, t0, t1, min_spikes=3):
    """Mean over neurons (with >= min_spikes spikes in the window) of the
    coefficient of variation of their inter-spike intervals, per population."""
    m = (steps >= t0) & (steps < t1)
    s, i = steps[m].astype(np.int64), ids[m].astype(np.int64)
    order = np.lexsort((s, i))
    s, i = s[order], i[order]
    out = np.full(len(offsets) - 1, np.nan)
    if len(s) == 0:
        return out
    bounds = np.flatnonzero(np.diff(i)) + 1
    starts = np.concatenate([[0], bounds])
    ends = np.concatenate([bounds, [len(i)]])
    cv_per_pop = [[] for _ in range(len(offsets) - 1)]
    for a, b in zip(starts, ends):
        if b - a < min_spikes:
            continue
        isi = np.diff(s[a:b]).astype(np.float64)
        cv_per_pop[population_of(np.array([i[a]]), offsets)[0]].append(isi.std() / isi.mean())
    for p, v in enumerate(cv_per_pop):
        if v:
            out[p] = float(np.mean(v))
    return out


def first_divergence(steps_a, ids_a, steps_b, ids_b):
    """First step at which the two sorted rasters differ (None if equal)."""
    n = min(len(steps_a), len(steps_b))
    a = steps_a[:n].astype(np.int64) * (1 << 32) + ids_a[:n]
    b = steps_b[:n].astype(np.int64) * (1 << 32) + ids_b[:n]
    diff = np.flatnonzero(a != b)
    if len(diff):
        k = diff[0]
        return int(min(steps_a[k], steps_b[k]))
    if len(steps_a) != len(steps_b):
        return int(steps_a[n] if len(steps_a) > n else steps_b[n])
    return None


def step_digest(steps, ids, n_steps):
    """Per step t < n_steps: [spike count, sum of ids, sum of ids^2] (int64),
    a compact fingerprint of a raster's first steps."""
    m = steps < n_steps
    s, i = steps[m].astype(np.int64), ids[m].astype(np.int64)
    out = np.zeros((n_steps, 3), dtype=np.int64)
    np.add.at(out[:, 0], s, 1)
    np.add.at(out[:, 1], s, i)
    np.add.at(out[:, 2], s, i * i)
    return out


def first_digest_divergence(dig_a, dig_b):
    """First step whose fingerprints differ (None if all equal)."""
    n = min(len(dig_a), len(dig_b))
    diff = np.flatnonzero(np.any(np.asarray(dig_a[:n]) != np.asarray(dig_b[:n]), axis=1))
    return int(diff[0]) if len(diff) else None


# ---------------------------------------------------------------------------
# Distribution comparison of Sec. 4.1: per population, the distributions of
# single-neuron firing rates, CVs of inter-spike intervals and Pearson
# correlation coefficients between binned spike trains of a neuron sample,
# each smoothed by a Gaussian kernel density estimate (Scott's rule) and
# compared by the Kullback-Leibler divergence.
# ---------------------------------------------------------------------------

def neuron_rates(steps, ids, lo, hi, t0, t1):
    """Firing rate (Hz) of every neuron in [lo, hi) over steps [t0, t1)."""
    m = (steps >= t0) & (steps < t1) & (ids >= lo) & (ids < hi)
    return np.bincount(ids[m].astype(np.int64) - lo, minlength=hi - lo) / ((t1 - t0) * DT_S)


def neuron_cvs(steps, ids, lo, hi, t0, t1, min_spikes=3):
    """CV of inter-spike intervals of every neuron in [lo, hi) with at least
    min_spikes spikes in [t0, t1)."""
    m = (steps >= t0) & (steps < t1) & (ids >= lo) & (ids < hi)
    s, i = steps[m].astype(np.int64), ids[m].astype(np.int64)
    order = np.lexsort((s, i))
    s, i = s[order], i[order]
    if len(s) == 0:
        return np.zeros(0)
    bounds = np.flatnonzero(np.diff(i)) + 1
    out = []
    for a, b in zip(np.concatenate([[0], bounds]), np.concatenate([bounds, [len(i)]])):
        if b - a >= min_spikes:
            isi = np.diff(s[a:b]).astype(np.float64)
            out.append(isi.std() / isi.mean())
    return np.array(out)


def pearson_samples(steps, ids, lo, hi, t0, t1, n_sample=200, bin_steps=20, seed=0):
    """Pearson correlation coefficients between the binned spike trains
    (bins of bin_steps steps) of every pair in a sample of n_sample neurons
    of [lo, hi) drawn with a fixed seed; pairs with a silent neuron excluded."""
    rng = np.random.default_rng(seed)
    n = hi - lo
    sample = np.sort(rng.choice(n, size=min(n_sample, n), replace=False)) + lo
    nb = (t1 - t0) // bin_steps
    m = (steps >= t0) & (steps < t0 + nb * bin_steps) & np.isin(ids, sample)
    row = np.searchsorted(sample, ids[m])
    col = (steps[m].astype(np.int64) - t0) // bin_steps
    counts = np.zeros((len(sample), nb))
    np.add.at(counts, (row, col), 1.0)
    active = counts.std(axis=1) > 0
    c = np.corrcoef(counts[active])
    iu = np.triu_indices(c.shape[0], k=1)
    return c[iu]


def kde_on_grid(samples, grid):
    """Gaussian kernel density estimate (Scott's rule bandwidth) on a grid,
    normalised to integrate to one over the grid."""
    from scipy.stats import gaussian_kde
    samples = np.asarray(samples, np.float64)
    if len(samples) < 2 or samples.std() == 0:
        raise ValueError("need at least two distinct samples")
    p = gaussian_kde(samples, bw_method="scott")(grid)
    return p / np.trapezoid(p, grid)


def kl_divergence(p, q, grid, floor=1e-12):
    """KL(P || Q) of two densities on the same grid (trapezoidal rule)."""
    p = np.maximum(np.asarray(p, np.float64), floor)
    q = np.maximum(np.asarray(q, np.float64), floor)
    return float(np.trapezoid(p * np.log(p / q), grid))


STAT_NAMES = ("rate", "cv", "pearson")


def population_distributions(steps, ids, offsets, t0, t1):
    """Samples of the three statistics per population."""
    out = []
    for p in range(len(offsets) - 1):
        lo, hi = int(offsets[p]), int(offsets[p + 1])
        out.append({"rate": neuron_rates(steps, ids, lo, hi, t0, t1),
                    "cv": neuron_cvs(steps, ids, lo, hi, t0, t1),
                    "pearson": pearson_samples(steps, ids, lo, hi, t0, t1, seed=p)})
    return out
