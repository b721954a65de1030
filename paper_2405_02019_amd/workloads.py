"""Synthetic workloads: the instance configurations of the benchmark and the
tests.  Only configuration draws live here, none of the model's arithmetic.

* full:  the full-scale microcircuit (77,169 neurons), one seed.
* x4:    four times the neurons of every population with full-scale in-degrees
         kept (308,676 neurons, ~1.2e9 synapses).
* batch: independent instances of uneven size and parameters: scale uniform
         in [5 %, 20 %], g uniform in [-6, -3], background rate uniform in
         [6, 10] Hz, distinct seeds, in-degrees kept at full scale so every
         instance stays near the full-scale regime.  The draws come from a
         Philox generator seeded with the master seed.
"""
import numpy as np

from .snn import Instance


def full_scale(seed=1):
    return [Instance(scale=1.0, seed=seed)]


def stress_x4(seed=1):
    return [Instance(scale=4.0, indegree_mode=1, seed=seed)]


def batch(n=64, master_seed=1, scale=(0.05, 0.20), g=(-6.0, -3.0), rate_hz=(6.0, 10.0)):
    rng = np.random.Generator(np.random.Philox(master_seed))
    s = rng.uniform(scale[0], scale[1], n)
    gg = rng.uniform(g[0], g[1], n)
    nu = rng.uniform(rate_hz[0], rate_hz[1], n)
    seeds = rng.integers(1, 2**62, n)
    return [Instance(scale=float(s[i]), indegree_mode=1, g=float(gg[i]), bg_rate_hz=float(nu[i]),
                     seed=int(seeds[i])) for i in range(n)]


WORKLOADS = {"full": full_scale, "x4": stress_x4, "batch": batch}
