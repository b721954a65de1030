"""Writes orientation_full_scale.json: spiking neurons per step of the
full-scale microcircuit (seed 1) under both readings of the orientation of
the connection-probability table (tab:params3: rows as target populations,
the reading taken, or rows as source populations), simulated by the int32
oracle for 5,000 steps and averaged over steps [1000, 5000) (after the
onset transient).  Sec. 3.3 reports that on average 23 neurons spike per
step, which tells the two readings apart.  Calls only the oracle.

Usage: python tests/golden/make_orientation.py   (about 2 minutes, 10 GB)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import pyoracle as O  # noqa: E402

STEPS, T0 = 5000, 1000


def main():
    out = {"what": "int32 oracle, full-scale microcircuit, seed 1, spikes per step over "
                   "steps [1000, 5000)", "steps": STEPS, "window": [T0, STEPS], "readings": {}}
    for name, ras in [("rows_are_targets", 0), ("rows_are_sources", 1)]:
        net = O.Net(O.Config(scale=1.0, seed=1, rows_are_sources=ras))
        sim = O.Sim(net).run(STEPS)
        s, i = sim.raster()
        m = s >= T0
        off = net.pop_offsets()
        pop = np.searchsorted(off, i[m], side="right") - 1
        rates = np.bincount(pop, minlength=8) / np.diff(off) / ((STEPS - T0) * 1e-4)
        out["readings"][name] = {"spikes_per_step": float(m.sum()) / (STEPS - T0),
                                 "rates_hz": [round(float(r), 4) for r in rates]}
        print(name, out["readings"][name], flush=True)
        sim.close()
        net.close()
    with open(os.path.join(HERE, "orientation_full_scale.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
