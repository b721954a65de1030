"""Writes f64_full_scale_seed1.json: spike statistics of the FP64 oracle on
the full-scale microcircuit (10 s of biological time), the reference of the
precision comparison (Sec. 4.1: statistics over [1 s, 10 s)).  Calls only the
oracle.

Stored:
  rates_hz, cv_isi   seed 1, per population: mean rate and mean CV of ISIs
  digest             seed 1, per step t < 3000: [spike count, sum of ids,
                     sum of ids^2], to locate the first step at which another
                     raster differs from it
  dist               per population and statistic (single-neuron rate, CV of
                     ISIs, Pearson coefficient of 2 ms binned trains of 200
                     sampled neurons): an evaluation grid spanning the values
                     of seeds 1-4 and the Gaussian KDE density of seed 1 on it
  seed_kl            per statistic, the population-mean KL divergence
                     KL(seed a || seed b) for the twelve ordered pairs of
                     seeds 1-4, with their mean and maximum: the seed-to-seed
                     yardstick of Sec. 4.1

Usage: python tests/golden/make_f64_stats.py   (about 20 minutes)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import pyoracle as O  # noqa: E402
from spike_stats import (STAT_NAMES, cv_isi, kde_on_grid, kl_divergence,  # noqa: E402
                         population_distributions, rates_hz, step_digest)

STEPS = 100_000
T0 = 10_000
DIGEST_STEPS = 3000
GRID_POINTS = 128
SEEDS = (1, 2, 3, 4)


def run(seed):
    t = time.time()
    net = O.Net(O.Config(scale=1.0, seed=seed))
    sim = O.Sim(net, arith=O.ARITH_F64).run(STEPS)
    steps, ids = sim.raster()
    print("seed", seed, "ran in", round(time.time() - t, 1), "s", flush=True)
    return steps, ids, net.pop_offsets()


def grid_for(samples):
    lo = min(a.min() for a in samples)
    hi = max(a.max() for a in samples)
    pad = 0.1 * (hi - lo) + 1e-9
    return np.linspace(lo - pad, hi + pad, GRID_POINTS)


def main():
    runs = {sd: run(sd) for sd in SEEDS}
    s1, i1, off = runs[1]
    for sd in SEEDS:
        assert np.array_equal(runs[sd][2], off)
    dists = {sd: population_distributions(runs[sd][0], runs[sd][1], off, T0, STEPS) for sd in SEEDS}
    npop = len(off) - 1
    dist = []
    kl = {name: {} for name in STAT_NAMES}
    for p in range(npop):
        entry = {}
        for name in STAT_NAMES:
            g = grid_for([dists[sd][p][name] for sd in SEEDS])
            k = {sd: kde_on_grid(dists[sd][p][name], g) for sd in SEEDS}
            entry[name] = {"grid": [round(float(x), 7) for x in g],
                           "seed1": [float("%.6g" % x) for x in k[1]]}
            for a in SEEDS:
                for b in SEEDS:
                    if a != b:
                        kl[name].setdefault("%d-%d" % (a, b), []).append(kl_divergence(k[a], k[b], g))
        dist.append(entry)
    seed_kl = {}
    for name in STAT_NAMES:
        pairs = {key: float(np.mean(v)) for key, v in kl[name].items()}
        seed_kl[name] = {"pairs": pairs, "mean": float(np.mean(list(pairs.values()))),
                         "max": float(np.max(list(pairs.values())))}
    out = {
        "what": "FP64 oracle, full-scale microcircuit, seeds 1-4, 100000 steps of 0.1 ms",
        "seed": 1,
        "scale": 1.0,
        "steps": STEPS,
        "window": [T0, STEPS],
        "pop_offsets": [int(x) for x in off],
        "n_spikes": int(len(s1)),
        "rates_hz": [float(x) for x in rates_hz(s1, i1, off, T0, STEPS)],
        "cv_isi": [float(x) for x in cv_isi(s1, i1, off, T0, STEPS)],
        "digest": step_digest(s1, i1, DIGEST_STEPS).tolist(),
        "dist": dist,
        "seed_kl": seed_kl,
    }
    with open(os.path.join(HERE, "f64_full_scale_seed1.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))
        f.write("\n")
    for name in STAT_NAMES:
        print(name, "population-mean KL between seeds: mean %.5f max %.5f"
              % (seed_kl[name]["mean"], seed_kl[name]["max"]), flush=True)


if __name__ == "__main__":
    main()
