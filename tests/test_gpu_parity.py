"""GPU parity: the HIP path through the C ABI against the CPU oracle, element
by element.  The plain and compressed paths must reproduce the oracle's spike
rasters, membrane potentials, currents, refractory counters, ring buffers and
counters bit for bit: every FP32 operation is separately rounded on both sides
and all synaptic input is an exact int32 sum."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-parity]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2405_02019_amd as P
    P.lib()
    return P


def oracle_cfg(oracle, inst, wmode):
    return oracle.Config(seed=inst.seed, scale=inst.scale, indegree_mode=inst.indegree_mode,
                         count_rule=inst.count_rule, rows_are_sources=inst.rows_are_sources,
                         g=inst.g, bg_rate_hz=inst.bg_rate_hz, psp_ext_mv=inst.psp_ext_mv,
                         bg_const_T=inst.bg_const_T, conn=inst.conn, weight_mode=wmode)


def run_oracle(oracle, inst, wmode, steps):
    net = oracle.Net(oracle_cfg(oracle, inst, wmode))
    sim = oracle.Sim(net).run(steps)
    return net, sim


def assert_parity(sim, k, net, osim, ring=True):
    gs, gi = sim.spikes(k)
    os_, oi = osim.raster()
    assert len(gs) == len(os_), (len(gs), len(os_))
    np.testing.assert_array_equal(gs, os_)
    np.testing.assert_array_equal(gi, oi)
    st = sim.state(k, ring=ring)
    ost = osim.state()
    assert st["t"] == ost["t"]
    np.testing.assert_array_equal(st["U"], ost["U"])
    np.testing.assert_array_equal(st["I"], ost["I"])
    np.testing.assert_array_equal(st["R"], ost["R"])
    if ring:
        np.testing.assert_array_equal(st["W"].astype(np.int64), ost["W"])
    c = osim.counters()
    assert st["spikes"] == c["spikes"]
    assert st["events"] == c["events"]
    assert st["poisson"] == c["poisson"]
    assert st["consumed"] == c["consumed"]
    return len(gs)


def test_propagators_on_gpu(P, oracle):
    with P.Simulator(P.Instance(scale=0.01)) as sim:
        st = sim.state()
    k = oracle.constants()
    assert st["p11"] == np.float32(k["p11f"])
    assert st["p22"] == np.float32(k["p22f"])
    assert st["p21"] == np.float32(k["p21f"])
    assert st["w_ext_q"] == k["w_ext_q"] and st["w_f"] == k["w_f"]


@pytest.mark.parametrize("engine", ["stepwise", "persistent", "lds"])
@pytest.mark.parametrize("fmt,wmode", [("plain", 0), ("compressed", 1)])
def test_tiny_circuit_bit_exact(P, oracle, engine, fmt, wmode):
    """1 % circuit (772 neurons), 0.1 s of biological time in ragged pieces
    (1, 99, 100, 63, 65, 672 steps) across graph-chunk boundaries."""
    inst = P.Instance(scale=0.01, seed=1)
    say("tiny", engine, fmt)
    with P.Simulator(inst, syn_format=fmt, engine=engine) as sim:
        for n in [1, 99, 100, 63, 65, 672]:
            sim.step(n)
        net, osim = run_oracle(oracle, inst, wmode, 1000)
        n = assert_parity(sim, 0, net, osim)
    assert n > 5000


def test_tiny_without_graphs_and_odd_chunks(P, oracle):
    inst = P.Instance(scale=0.01, seed=2)
    for kw in [dict(use_graphs=False), dict(chunk_steps=7)]:
        say("tiny", kw)
        with P.Simulator(inst, **kw) as sim:
            sim.step(300)
            sim.step(33)
            net, osim = run_oracle(oracle, inst, 0, 333)
            assert_parity(sim, 0, net, osim)


@pytest.mark.parametrize("scale,block,grid,chunk", [(0.05, 256, 1, 100), (0.05, 128, 2, 7),
                                                    (0.05, 512, 1, 1), (0.05, 1024, 1, 33),
                                                    (0.05, 256, 3, 64), (0.08, 256, 1, 50)])
def test_persistent_shapes(P, oracle, scale, block, grid, chunk):
    """Persistent engine with forced shapes: grids of 1-3 blocks, so every
    thread owns up to 7 quads and every block many senders, and chunks of 1
    to 100 steps (one grid barrier per step)."""
    inst = P.Instance(scale=scale, seed=21)
    say("persistent shape", block, grid, chunk)
    with P.Simulator(inst, engine="persistent", block_size=block, grid_blocks=grid,
                     chunk_steps=chunk) as sim:
        info = sim.info()
        assert info["engine"] == P.ENGINE_PERSISTENT and info["grid_blocks"] == grid
        sim.step(211)
        net, osim = run_oracle(oracle, inst, 0, 211)
        assert_parity(sim, 0, net, osim)


@pytest.mark.parametrize("grid", [8, 16])
@pytest.mark.parametrize("fmt,wmode", [("plain", 0), ("compressed", 1)])
def test_lds_windows(P, oracle, grid, fmt, wmode):
    """LDS engine with 512-neuron (8 blocks) and 256-neuron (16 blocks)
    windows on the 5 % circuit (3,859 neurons, 0.75 M synapses)."""
    inst = P.Instance(scale=0.05, seed=31)
    say("lds windows", grid, fmt)
    with P.Simulator(inst, syn_format=fmt, engine="lds", grid_blocks=grid, chunk_steps=37) as sim:
        info = sim.info()
        assert info["engine"] == P.ENGINE_LDS and info["grid_blocks"] == grid
        sim.step(150)
        sim.step(100)
        net, osim = run_oracle(oracle, inst, wmode, 250)
        assert_parity(sim, 0, net, osim)


@pytest.mark.parametrize("fmt,wmode", [("plain", 0), ("compressed", 1)])
def test_lds_high_activity(P, oracle, fmt, wmode):
    """LDS engine under a burst: the half-scale circuit with weak inhibition
    (g = -2) and a 16 Hz background opens with steps of several hundred
    spikes.  Covers windows with more than four spikes in a step (list
    entries), more senders in a step than a polling wave stages (search
    over the windows with senders), both polling waves (more than 128
    windows) and senders whose segments span several pieces."""
    inst = P.Instance(scale=0.5, seed=7, g=-2.0, bg_rate_hz=16.0)
    say("lds high activity", fmt)
    with P.Simulator(inst, syn_format=fmt, engine="lds", chunk_steps=50) as sim:
        info = sim.info()
        assert info["engine"] == P.ENGINE_LDS and info["grid_blocks"] > 128
        sim.step(150)
        net, osim = run_oracle(oracle, inst, wmode, 150)
        steps, _ = osim.raster()
        per_step = np.bincount(steps, minlength=150)
        say("spikes per step: max", per_step.max(), "mean", per_step.mean())
        assert per_step.max() > 2 * 128
        assert_parity(sim, 0, net, osim)


def test_degenerate_drives(P, oracle):
    """No synapses and no thalamic input; then a constant count of one
    thalamic spike per step at a sub-threshold amplitude; then no drive at
    all on the full tables."""
    cases = [P.Instance(scale=0.01, seed=3, bg_rate_hz=0.0, conn=np.zeros(64)),
             P.Instance(scale=0.01, seed=3, bg_const_T=1, psp_ext_mv=0.07),
             P.Instance(scale=0.01, seed=4, bg_rate_hz=0.0)]
    for inst in cases:
      for engine in ["stepwise", "persistent", "lds"]:
        say("degenerate", engine, inst)
        with P.Simulator(inst, engine=engine) as sim:
            sim.step(250)
            net, osim = run_oracle(oracle, inst, 0, 250)
            assert_parity(sim, 0, net, osim)


def test_batched_instances_each_bit_exact(P, oracle):
    """Several independent instances of uneven scale, seed, g and thalamic
    rate in one handle: each matches its own oracle run."""
    insts = [P.Instance(scale=0.01, seed=11),
             P.Instance(scale=0.023, seed=12, g=-5.0, bg_rate_hz=9.0),
             P.Instance(scale=0.013, seed=13, g=-3.5, bg_rate_hz=6.5, indegree_mode=1),
             P.Instance(scale=0.002, seed=14)]
    for fmt, wmode in [("plain", 0), ("compressed", 1)]:
      for engine in ["stepwise", "persistent", "lds"]:
        say("batch", fmt, engine)
        with P.Simulator(insts, syn_format=fmt, engine=engine) as sim:
            sim.step(400)
            for k, inst in enumerate(insts):
                net, osim = run_oracle(oracle, inst, wmode, 400)
                assert_parity(sim, k, net, osim)


def test_minimum_raster_capacity(P, oracle):
    """A raster capacity of one entry is raised to the library's minimum
    (twice the neurons plus 64 entries), so the step loop drains the device
    raster every few steps.  The drain schedule bounds the spikes pending on
    the device by the refractory period (a neuron spikes at most once in 21
    steps), so the device raster cannot overflow and the results stay exact;
    reading spikes in pieces and discarding them keeps the host store
    bounded."""
    inst = P.Instance(scale=0.01, seed=5)
    net, osim = run_oracle(oracle, inst, 0, 500)
    os_, oi = osim.raster()
    for engine in ["stepwise", "persistent", "lds"]:
        say("minimum raster capacity", engine)
        with P.Simulator(inst, engine=engine, raster_capacity=1, chunk_steps=50) as sim:
            sim.step(237)
            sim.step(263)
            assert_parity(sim, 0, net, osim)
            s1, i1 = sim.spikes(0, 0, 250)
            sim.discard_spikes(250)
            s2, i2 = sim.spikes(0, 0, 500)
            m = os_ < 250
            np.testing.assert_array_equal(s1, os_[m])
            np.testing.assert_array_equal(i1, oi[m])
            np.testing.assert_array_equal(s2, os_[~m])
            np.testing.assert_array_equal(i2, oi[~m])


@pytest.mark.parametrize("fmt,wmode", [("plain", 0), ("compressed", 1)])
def test_band_tiny_bit_exact(P, oracle, fmt, wmode):
    """Banded engine with all 64 ring rows in LDS: the delay-1 band is
    delivered when the flags arrive, the other delays one step later.  The
    1 % circuit in ragged pieces (1, 99, 100, 63, 65, 672 steps)."""
    inst = P.Instance(scale=0.01, seed=1)
    say("band tiny", fmt)
    with P.Simulator(inst, syn_format=fmt, engine="band") as sim:
        info = sim.info()
        assert info["engine"] == P.ENGINE_BAND and info["ring_rows"] == 64
        for n in [1, 99, 100, 63, 65, 672]:
            sim.step(n)
        net, osim = run_oracle(oracle, inst, wmode, 1000)
        assert assert_parity(sim, 0, net, osim) > 5000


@pytest.mark.parametrize("scale,block,grid,chunk,rows", [
    (0.05, 512, 4, 37, 16), (0.05, 512, 3, 1, 16), (0.05, 1024, 2, 50, 8),
    (0.01, 1024, 1, 7, 8), (0.05, 256, 12, 3, 64), (0.05, 512, 9, 200, 16)])
@pytest.mark.parametrize("fmt,wmode", [("plain", 0), ("compressed", 1), ("dev8", 2)])
def test_band_shapes(P, oracle, scale, block, grid, chunk, rows, fmt, wmode):
    """Banded engine with 16 (512-thread blocks) and 8 (1024-thread blocks)
    ring rows in LDS, horizon-based delivery (Sec. 3.4): launches of 1 to
    200 steps, so that slow bands still pending when a launch ends go to the
    ring in device memory and come back into LDS as their rows enter the
    horizon of the next launch.  The whole 64-row ring is compared after
    each stretch."""
    inst = P.Instance(scale=scale, seed=31)
    say("band shape", block, grid, chunk, fmt)
    with P.Simulator(inst, syn_format=fmt, engine="band", block_size=block, grid_blocks=grid,
                     chunk_steps=chunk) as sim:
        info = sim.info()
        say("band info", info)
        assert info["engine"] == P.ENGINE_BAND and info["grid_blocks"] == grid
        assert info["ring_rows"] == rows and info["block_size"] == block
        sim.step(150)
        net, osim = run_oracle(oracle, inst, wmode, 150)
        assert_parity(sim, 0, net, osim)
        sim.step(101)
        osim.run(101)
        assert_parity(sim, 0, net, osim)


@pytest.mark.parametrize("block", [256, 512, 1024])
def test_band_high_activity(P, oracle, block):
    """Banded engine under a burst (half-scale circuit, g = -2, 16 Hz
    background): steps of several hundred senders overflow the LDS sender
    history into device memory and fill the sender lists; with 64, 16 and 8
    ring rows (plain, compressed and deviation records)."""
    inst = P.Instance(scale=0.5, seed=7, g=-2.0, bg_rate_hz=16.0)
    fmt, wmode = {256: ("plain", 0), 512: ("compressed", 1), 1024: ("dev8", 2)}[block]
    say("band high activity", block, fmt)
    with P.Simulator(inst, syn_format=fmt, engine="band", block_size=block, chunk_steps=60) as sim:
        info = sim.info()
        say("band info", info)
        assert info["engine"] == P.ENGINE_BAND and info["block_size"] == block
        sim.step(150)
        net, osim = run_oracle(oracle, inst, wmode, 150)
        steps, _ = osim.raster()
        assert np.bincount(steps, minlength=150).max() > 256
        assert_parity(sim, 0, net, osim)


@pytest.mark.parametrize("block", [256, 1024])
def test_band_batched_instances(P, oracle, block):
    """Independent instances of uneven scale, seed, g and thalamic rate in
    one banded launch: each matches its own oracle run."""
    insts = [P.Instance(scale=0.01, seed=11),
             P.Instance(scale=0.023, seed=12, g=-5.0, bg_rate_hz=9.0),
             P.Instance(scale=0.013, seed=13, g=-3.5, bg_rate_hz=6.5, indegree_mode=1),
             P.Instance(scale=0.002, seed=14)]
    for fmt, wmode in [("plain", 0), ("compressed", 1), ("dev8", 2)]:
        say("band batch", block, fmt)
        with P.Simulator(insts, syn_format=fmt, engine="band", block_size=block,
                         chunk_steps=90) as sim:
            sim.step(400)
            for k, inst in enumerate(insts):
                net, osim = run_oracle(oracle, inst, wmode, 400)
                assert_parity(sim, k, net, osim)


def test_lds_instance_groups_bit_exact(P, oracle):
    """Instances beyond one co-resident grid (18 x 10 % circuits, 139k
    neurons) run as several LDS launches per chunk (groups of whole
    instances, requested explicitly), each instance still equal to its own
    oracle run, across ragged chunk pieces."""
    rng = np.random.default_rng(5)
    insts = [P.Instance(scale=0.1, seed=40 + i, g=float(rng.uniform(-6, -3)),
                        bg_rate_hz=float(rng.uniform(6, 10))) for i in range(18)]
    for fmt, wmode, graphs in [("plain", 0, True), ("compressed", 1, False)]:
        say("lds groups", fmt, "graphs", graphs)
        with P.Simulator(insts, syn_format=fmt, engine="lds", chunk_steps=50,
                         use_graphs=graphs) as sim:
            info = sim.info()
            say("lds groups info", info)
            assert info["engine"] == P.ENGINE_LDS and info["launches_per_chunk"] >= 2
            sim.step(70)
            sim.step(80)
            for k, inst in enumerate(insts):
                net, osim = run_oracle(oracle, inst, wmode, 150)
                assert_parity(sim, k, net, osim, ring=(k % 5 == 0))


@pytest.mark.parametrize("engine", ["persistent", "stepwise", "lds"])
def test_autotune_keeps_results_bit_exact(P, oracle, engine):
    """The shape tuner runs its trials on the live simulation: afterwards the
    state equals the oracle's after the same number of steps."""
    insts = [P.Instance(scale=0.02, seed=21), P.Instance(scale=0.01, seed=22, g=-5.0)]
    say("autotune", engine)
    with P.Simulator(insts, engine=engine, chunk_steps=40) as sim:
        rep = sim.autotune(25)
        say("autotune report", rep)
        assert rep["candidates"] >= (1 if engine == "lds" else 2)
        assert rep["us_per_step_best"] > 0 and rep["us_per_step_best"] <= rep["us_per_step_first"]
        total = rep["candidates"] * 25 + 60
        sim.step(60)
        for k, inst in enumerate(insts):
            net, osim = run_oracle(oracle, inst, 0, total)
            assert_parity(sim, k, net, osim)


def test_tuned_build_bit_exact_and_cached(P, oracle, tmp_path):
    """snn_build_tuned times the LDS engines' candidate layouts (LDS and
    banded engine, several window lengths), rebuilds the fastest from step 0
    and records the choice; a second build of the same configuration takes
    it from the cache without timing.  Either way the results equal the
    oracle's."""
    inst = P.Instance(scale=0.05, seed=41)
    cache = str(tmp_path / "tune.txt")
    with P.Simulator(inst, chunk_steps=100, tune_steps=200, tune_cache=cache) as sim:
        rep = sim.tune_report
        say("tuned build", rep, sim.info())
        assert rep["candidates"] >= 3 and rep["us_per_step_best"] <= rep["us_per_step_first"]
        assert rep["window_neurons"] == sim.info()["window_neurons"]
        sim.step(300)
        net, osim = run_oracle(oracle, inst, 0, 300)
        assert_parity(sim, 0, net, osim)
    assert len(open(cache).read().splitlines()) == 1
    with P.Simulator(inst, chunk_steps=100, tune_steps=200, tune_cache=cache) as sim:
        rep2 = sim.tune_report
        assert rep2["candidates"] == 0 and rep2["window_neurons"] == rep["window_neurons"]
        assert rep2["engine"] == rep["engine"]
        sim.step(300)
        assert_parity(sim, 0, net, osim)


def _windows(n, L):
    """Windows of an instance of n neurons at window length L (the plan's
    rule: balanced windows of whole quads)."""
    nq = (n + 3) // 4
    nw = -(-nq // (L // 4))
    wq = -(-nq // nw)
    return -(-nq // wq)


UNEVEN = [dict(scale=0.01, seed=11), dict(scale=0.023, seed=12, g=-5.0, bg_rate_hz=9.0),
          dict(scale=0.013, seed=13, g=-3.5, bg_rate_hz=6.5, indegree_mode=1),
          dict(scale=0.002, seed=14)]


@pytest.mark.parametrize("engine,block,each", [("band", 256, [128, 256, 64, 40]),
                                               ("band", 1024, [600, 96, 1500, 4]),
                                               ("lds", 256, [200, 120, 320, 44])])
def test_per_instance_windows_bit_exact(P, oracle, engine, block, each):
    """One window length per instance (windows sized by load, Sec. 3.6's
    destination classes): the plan cuts each instance at its own length, and
    every instance still matches its own oracle run."""
    insts = [P.Instance(**kw) for kw in UNEVEN]
    for fmt, wmode in [("plain", 0), ("compressed", 1)]:
        say("per-instance windows", engine, block, each, fmt)
        with P.Simulator(insts, syn_format=fmt, engine=engine, block_size=block, chunk_steps=70,
                         inst_window_neurons=each) as sim:
            info = sim.info()
            say("per-instance windows info", info)
            n = [len(sim.state(k)["U"]) for k in range(len(insts))]
            assert info["grid_blocks"] == sum(_windows(nk, L) for nk, L in zip(n, each))
            assert info["window_neurons"] <= max(each)
            sim.step(300)
            for k, inst in enumerate(insts):
                net, osim = run_oracle(oracle, inst, wmode, 300)
                assert_parity(sim, k, net, osim)


def test_tuned_build_balances_instances(P, oracle, tmp_path):
    """With several instances the tuner also times the winning kernel with
    windows sized by each instance's measured events; the cache keeps
    per-instance lengths and a cached line with them rebuilds that layout."""
    insts = [P.Instance(scale=0.02, seed=51, g=-3.0, bg_rate_hz=10.0),
             P.Instance(scale=0.03, seed=52, g=-6.0, bg_rate_hz=6.0),
             P.Instance(scale=0.01, seed=53)]
    cache = str(tmp_path / "tune.txt")
    with P.Simulator(insts, engine="band", chunk_steps=100, tune_steps=400, tune_cache=cache) as sim:
        rep = sim.tune_report
        say("tuned batch", rep, sim.info())
        assert rep["candidates"] >= 2 and rep["us_per_step_best"] <= rep["us_per_step_first"]
        n = [len(sim.state(k)["U"]) for k in range(len(insts))]
        sim.step(200)
        for k, inst in enumerate(insts):
            net, osim = run_oracle(oracle, inst, 0, 200)
            assert_parity(sim, k, net, osim)
    line = open(cache).read().split()
    assert len(line) in (6, 7)
    # A hand-written per-instance choice for the same key is taken from the
    # cache (the last matching line wins).
    each = [64, 512, 128]
    with open(cache, "a") as f:
        f.write(" ".join(line[:2] + [str(P.ENGINE_BAND), "0", "1.0", "1.0",
                                     ",".join(map(str, each))]) + "\n")
    with P.Simulator(insts, engine="band", chunk_steps=100, tune_steps=400, tune_cache=cache) as sim:
        rep2 = sim.tune_report
        info = sim.info()
        say("cached per-instance layout", rep2, info)
        assert rep2["candidates"] == 0 and info["engine"] == P.ENGINE_BAND
        assert info["grid_blocks"] == sum(_windows(nk, L) for nk, L in zip(n, each))
        sim.step(200)
        for k, inst in enumerate(insts):
            net, osim = run_oracle(oracle, inst, 0, 200)
            assert_parity(sim, k, net, osim)


@pytest.fixture(scope="module")
def full_oracle(oracle):
    """Oracle run of the full-scale microcircuit, 300 steps."""
    say("full scale: building oracle network")
    return run_oracle(oracle, oracle_stub_instance(), 0, 300)


def oracle_stub_instance():
    import paper_2405_02019_amd as P
    return P.Instance(scale=1.0, seed=1)


@pytest.mark.parametrize("insts,chunk,pieces", [
    ([(0.01, 7, -4.0)], 37, [1, 99, 100, 300]),
    ([(0.05, 8, -4.0)], 100, [250, 50]),
    ([(0.02, 9, -5.5), (0.01, 10, -3.0), (0.03, 11, -4.5)], 64, [130, 70]),
])
def test_dev8_bit_exact(P, oracle, insts, chunk, pieces):
    """The deviation format (Sec. 5.3: each weight stored as its population
    pair's mean plus an 8-bit deviation) on the LDS engine equals the oracle's
    dev8 mode spike for spike, with the state and the whole ring, across
    ragged launches; instances of different g carry their own means and
    steps."""
    inst = [P.Instance(scale=s, seed=sd, g=g) for s, sd, g in insts]
    say("dev8", insts, chunk)
    with P.Simulator(inst, syn_format="dev8", chunk_steps=chunk) as sim:
        assert sim.info()["engine"] == P.ENGINE_LDS
        for n in pieces:
            sim.step(n)
        total = 0
        for k, x in enumerate(inst):
            net, osim = run_oracle(oracle, x, 2, sum(pieces))
            total += assert_parity(sim, k, net, osim)
    assert total > 1000


def test_dev8_full_scale_window_bit_exact(P, oracle):
    """Full scale in the benchmark's launch length (10,000-step chunks), the
    first 300 steps in the deviation format, against the oracle's dev8 mode."""
    inst = oracle_stub_instance()
    with P.Simulator(inst, syn_format="dev8", chunk_steps=10000) as sim:
        assert sim.info()["engine"] == P.ENGINE_LDS
        sim.step(300)
        net, osim = run_oracle(oracle, inst, 2, 300)
        n = assert_parity(sim, 0, net, osim)
        say("dev8 full scale spikes", n)
    assert n > 5000


@pytest.mark.parametrize("engine", ["stepwise", "persistent", "lds", "band"])
def test_full_scale_window_bit_exact(P, full_oracle, engine):
    """Full-scale microcircuit (77,169 neurons, 2.99e8 synapses): the first
    300 steps match the oracle spike for spike, with the whole state."""
    say("full scale: building GPU network", engine)
    with P.Simulator(oracle_stub_instance(), engine=engine) as sim:
        sim.step(300)
        say("full scale: comparing")
        net, osim = full_oracle
        n = assert_parity(sim, 0, net, osim)
        say("full scale spikes", n, sim.info())
