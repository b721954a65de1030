"""Writes the int32 oracle's fingerprints of 10 s of the full-scale
microcircuit (seed 1), in the plain (2^-8 pA), the compressed (16-bit,
2^-5 pA) and the dev8 (pair mean plus an 8-bit deviation, Sec. 5.3) weight
modes: the reference of the bit-exact GPU tests over the whole
run (eqn:mem, eqn:psc, eqn:ref with the int32 input sum; Sec. 4.1 motivates
spike-for-spike agreement).  Calls only the oracle.

Stored, per weight mode:
  int32_full_scale_seed1_<mode>.digest.gz
      gzip of little-endian int64 [steps][3]: per step t, the spike count,
      the sum of the spiking ids and the sum of their squares
  int32_full_scale_seed1.json
      per mode: the SHA-256 of the final U (float32), I (float32), R (int32)
      and ring W (int64, 64 rows x N, row-major), the counters, the number
      of spikes, and the SHA-256 of the digest file's contents

Usage: python tests/golden/make_int32_digests.py [mode ...]
(about 4 minutes per mode; named modes are recomputed and merged into the
existing JSON, no names recompute every mode)
"""
import gzip
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import pyoracle as O  # noqa: E402
from spike_stats import step_digest  # noqa: E402

STEPS = 100_000
SEED = 1
MODES = {"plain": O.W_PLAIN, "compressed": O.W_COMPRESSED, "dev8": O.W_DEV8}
BASENAME = "int32_full_scale_seed1"


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main(names):
    out = {"what": "int32 oracle, full-scale microcircuit, seed 1, 100000 steps of 0.1 ms",
           "seed": SEED, "scale": 1.0, "steps": STEPS, "modes": {}}
    meta = os.path.join(HERE, f"{BASENAME}.json")
    if names and os.path.exists(meta):
        with open(meta) as f:
            out = json.load(f)
    for name in names or list(MODES):
        wmode = MODES[name]
        t = time.time()
        net = O.Net(O.Config(scale=1.0, seed=SEED, weight_mode=wmode))
        sim = O.Sim(net).run(STEPS)
        steps, ids = sim.raster()
        st = sim.state()
        dig = step_digest(steps, ids, STEPS).astype("<i8")
        raw = dig.tobytes()
        path = os.path.join(HERE, f"{BASENAME}_{name}.digest.gz")
        with gzip.GzipFile(path, "wb", mtime=0) as f:
            f.write(raw)
        out["modes"][name] = {
            "digest_file": os.path.basename(path),
            "digest_sha256": hashlib.sha256(raw).hexdigest(),
            "n_neurons": net.N,
            "n_synapses": net.nsyn,
            "n_spikes": int(len(steps)),
            "counters": sim.counters(),
            "sha256": {"U": sha(st["U"].astype("<f4")), "I": sha(st["I"].astype("<f4")),
                       "R": sha(st["R"].astype("<i4")), "W": sha(st["W"].astype("<i8"))},
        }
        print(name, len(steps), "spikes in", round(time.time() - t, 1), "s", flush=True)
        sim.close()
        net.close()
    with open(os.path.join(HERE, f"{BASENAME}.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:])
