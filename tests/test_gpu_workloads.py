"""Parity at the benchmark's own workloads, on the layout, engine and launch
length the benchmark uses (the layout from the committed tuning cache --
timed anew if the cache has no entry for this GPU --, 10,000-step chunks,
after the launch-shape tuner has run):

* the batch of 64 independent instances of uneven scale (5-20 %), g,
  background rate and seed (576,807 neurons, 2.2e9 synapses): every
  instance equals its own oracle run spike for spike, with its state (the
  banded engine's 1,024-thread variant, 8 ring rows, windows sized per
  instance by its measured load);
* the 4x circuit with full-scale in-degrees (308,676 neurons, 1.2e9
  synapses), whose 64-row ring exceeds the chip's LDS: the banded engine
  (Sec. 3.4's horizon with 16 ring rows) against the oracle.

Both networks hold more than 2^31 record slots, so these are also the
regression tests of 64-bit record addressing.  Each case builds the oracle
network of the same configuration on the host (about 40 GB for the 4x
circuit)."""
import os
import sys

import numpy as np
import pytest

from test_gpu_parity import assert_parity, run_oracle

pytestmark = pytest.mark.gpu

CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_2405_02019_amd", "tune_cache.txt")


def say(*a):
    print("[gpu-workloads]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2405_02019_amd as P
    P.lib()
    return P


def snapshot(sim, k, ring):
    """Everything assert_parity reads, so the handle can be freed first."""
    steps, ids = sim.spikes(k)
    st = sim.state(k, ring=ring)

    class Frozen:
        def spikes(self, kk):
            return steps, ids

        def state(self, kk, ring=False):
            return st
    return Frozen()


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("fmt,wmode", [("compressed", 1), ("plain", 0)])
def test_batch_of_64_bit_exact(P, oracle, fmt, wmode):
    from paper_2405_02019_amd import workloads
    insts = workloads.batch()
    say("batch", fmt, "building")
    with P.Simulator(insts, syn_format=fmt, chunk_steps=10000, tune_steps=2000,
                     tune_cache=CACHE) as sim:
        info = sim.info()
        say("batch info", info, sim.tune_report)
        assert info["engine"] == P.ENGINE_BAND
        rep = sim.autotune(50)
        say("batch autotune", rep)
        total = rep["candidates"] * 50 + 250
        sim.step(250)
        snaps = [snapshot(sim, k, ring=(k % 8 == 0)) for k in range(len(insts))]
    n_spikes = 0
    for k, inst in enumerate(insts):
        net, osim = run_oracle(oracle, inst, wmode, total)
        n_spikes += assert_parity(snaps[k], k, net, osim, ring=(k % 8 == 0))
        osim.close()
        net.close()
    say("batch", fmt, "spikes", n_spikes, "in", total, "steps: every instance bit-exact")
    assert n_spikes > 1000


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("fmt,wmode", [("plain", 0), ("compressed", 1)])
def test_x4_circuit_bit_exact(P, oracle, fmt, wmode):
    from paper_2405_02019_amd import workloads
    inst = workloads.stress_x4()[0]
    say("x4", fmt, "building")
    with P.Simulator(inst, syn_format=fmt, chunk_steps=10000, tune_steps=2000,
                     tune_cache=CACHE) as sim:
        info = sim.info()
        say("x4 info", info, sim.tune_report)
        assert info["engine"] == P.ENGINE_BAND and info["ring_rows"] < 64
        rep = sim.autotune(40)
        total = rep["candidates"] * 40 + 160
        sim.step(160)
        snap = snapshot(sim, 0, ring=True)
    say("x4 oracle", total, "steps")
    net, osim = run_oracle(oracle, inst, wmode, total)
    n = assert_parity(snap, 0, net, osim)
    say("x4", fmt, "spikes", n, "in", total, "steps: bit-exact")
    assert n > 1000
