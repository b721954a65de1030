"""Writes f64_full_scale_seed1.json: spike statistics of the FP64 oracle on
the full-scale microcircuit (seed 1, 10 s of biological time), the reference
of the precision comparison (Sec. 4.1: rates and CV of inter-spike intervals
over [1 s, 10 s)).  Calls only the oracle.

Stored:
  rates_hz, cv_isi   per population over steps [10000, 100000)
  digest             per step t < 3000: [spike count, sum of ids, sum of ids^2]
                     of the FP64 raster, used to locate the first step at
                     which another raster differs from it.

Usage: python tests/golden/make_f64_stats.py   (about 5 minutes on 8 cores)
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
from spike_stats import cv_isi, rates_hz, step_digest  # noqa: E402

SEED = 1
STEPS = 100_000
T0 = 10_000
DIGEST_STEPS = 3000


def main():
    t = time.time()
    net = O.Net(O.Config(scale=1.0, seed=SEED))
    print("build", round(time.time() - t, 1), "s", flush=True)
    t = time.time()
    sim = O.Sim(net, arith=O.ARITH_F64).run(STEPS)
    print("run", round(time.time() - t, 1), "s", flush=True)
    steps, ids = sim.raster()
    off = net.pop_offsets()
    out = {
        "what": "FP64 oracle, full-scale microcircuit, seed 1, 100000 steps of 0.1 ms",
        "seed": SEED,
        "scale": 1.0,
        "steps": STEPS,
        "window": [T0, STEPS],
        "pop_offsets": [int(x) for x in off],
        "n_spikes": int(len(steps)),
        "rates_hz": [float(x) for x in rates_hz(steps, ids, off, T0, STEPS)],
        "cv_isi": [float(x) for x in cv_isi(steps, ids, off, T0, STEPS)],
        "digest": step_digest(steps, ids, DIGEST_STEPS).tolist(),
    }
    with open(os.path.join(HERE, "f64_full_scale_seed1.json"), "w") as f:
        json.dump(out, f, separators=(",", ":"))
        f.write("\n")
    print("rates", np.round(out["rates_hz"], 3), "cv", np.round(out["cv_isi"], 3), flush=True)


if __name__ == "__main__":
    main()
