import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def oracle():
    """The CPU oracle's ctypes front end (built on first use)."""
    from oracle import build_oracle, pyoracle
    if not os.path.exists(pyoracle.LIB_PATH):
        build_oracle.build()
    return pyoracle


@pytest.fixture(scope="session")
def full_scale_runs():
    """The full-scale microcircuit (seed 1) simulated for 10 s of biological
    time (100,000 steps) on the GPU in the plain, the compressed and the
    deviation (dev8) synapse formats, in the launch configuration the
    benchmark times (10,000-step chunks).  Per format: the raster, the final
    state with the ring buffer, and the library's launch description."""
    import hashlib

    import numpy as np
    import paper_2405_02019_amd as P

    def sha(a):
        return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()

    out = {}
    for fmt in ["plain", "compressed", "dev8"]:
        print(f"[full-scale run] {fmt}: 100000 steps in 10000-step launches", flush=True)
        with P.Simulator(P.Instance(scale=1.0, seed=1), syn_format=fmt, chunk_steps=10000) as sim:
            for k in range(10):
                sim.step(10000)
                print(f"[full-scale run] {fmt}: {(k + 1) * 10000} steps queued", flush=True)
            steps, ids = sim.spikes()
            st = sim.state(ring=True)
            out[fmt] = {"steps": steps, "ids": ids, "info": sim.info(),
                        "sha256": {"U": sha(st["U"].astype("<f4")), "I": sha(st["I"].astype("<f4")),
                                   "R": sha(st["R"].astype("<i4")),
                                   "W": sha(st["W"].astype("<i8"))},
                        "counters": {k: st[k] for k in ("spikes", "events", "poisson", "consumed")},
                        "t": st["t"]}
    return out
