"""The allocation-free step call (snn_step_n_noalloc) against snn_step_n.

Two twin handles of the same configuration are advanced by the same number
of steps, one through each call: spike rasters (sorted), membrane
potentials, currents, refractory counters, the whole ring buffer and the
counters must be equal bit for bit.  Two calls in a row on different
handles, the second on a smaller network with the other LDS engine, so the
shared static scratch is reused at a different size; then a further call
continues the first handle."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-noalloc]", *a, flush=True)
    sys.stdout.flush()


def gpu_raster(torch, sim, n_steps):
    """Runs snn_step_n_noalloc and returns its raster as sorted (step, id)."""
    n = sum(s["n_neurons"] for s in [sim.state(k) for k in range(len(sim.instances))])
    cap = n * ((n_steps + 20) // 21)
    raster = torch.full((cap,), -1, dtype=torch.int64, device="cuda")
    status = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    # The fills run on torch's stream, the call on the handle's stream.
    torch.cuda.synchronize()
    sim.step_noalloc(n_steps, raster, status)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    assert st[1] == 0, st
    r = raster[: int(st[0])].cpu().numpy().view(np.uint64)
    assert np.all(raster[int(st[0]):].cpu().numpy() == -1)
    r = np.sort(r)
    return (r >> np.uint64(32)).astype(np.uint32), (r & np.uint64(0xFFFFFFFF)).astype(np.uint32)


def compare(sim_a, sim_b, steps_a, ids_a, t0, t1):
    steps_b, ids_b = sim_b.spikes(0, t0, t1)
    assert len(steps_a) == len(steps_b) and len(steps_a) > 100
    np.testing.assert_array_equal(steps_a, steps_b)
    np.testing.assert_array_equal(ids_a, ids_b)
    a = sim_a.state(ring=True)
    b = sim_b.state(ring=True)
    for k in ["U", "I", "R", "W"]:
        np.testing.assert_array_equal(a[k], b[k])
    for k in ["t", "spikes", "events", "poisson", "consumed"]:
        assert a[k] == b[k], k


def test_noalloc_matches_step_n():
    import torch
    import paper_2405_02019_amd as P
    cases = [(P.Instance(scale=0.05, seed=31), "compressed", "band", 300),
             (P.Instance(scale=0.01, seed=32), "plain", "lds", 150)]
    sims = []
    for inst, fmt, engine, n in cases:
        say("case", engine, fmt, inst.scale, n)
        a = P.Simulator(inst, syn_format=fmt, engine=engine, chunk_steps=70)
        b = P.Simulator(inst, syn_format=fmt, engine=engine, chunk_steps=70)
        steps, ids = gpu_raster(torch, a, n)
        b.step(n)
        compare(a, b, steps, ids, 0, n)
        sims.append((a, b, n))
    a, b, n = sims[0]
    say("continuing the first handle")
    steps, ids = gpu_raster(torch, a, 111)
    b.step(111)
    compare(a, b, steps, ids, n, n + 111)
    for a, b, _ in sims:
        a.close()
        b.close()


def test_noalloc_burst_reaches_every_sender_history_tier():
    """The banded engine's 512-thread variant under a burst (half-scale
    circuit, g = -2, 16 Hz background): steps of more than 320 senders fill
    the LDS history (128 ids per step), the block's private history (192
    more) and the shared one, all three carved from the static scratch area
    by the allocation-free call; it equals snn_step_n bit for bit."""
    import torch
    import paper_2405_02019_amd as P
    inst = P.Instance(scale=0.5, seed=7, g=-2.0, bg_rate_hz=16.0)
    say("burst case, band 512")
    a = P.Simulator(inst, syn_format="compressed", engine="band", block_size=512, chunk_steps=60)
    b = P.Simulator(inst, syn_format="compressed", engine="band", block_size=512, chunk_steps=60)
    assert a.info()["ring_rows"] == 16
    steps, ids = gpu_raster(torch, a, 150)
    b.step(150)
    compare(a, b, steps, ids, 0, 150)
    assert np.bincount(steps, minlength=150).max() > 320
    a.close()
    b.close()
