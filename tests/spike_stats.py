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
