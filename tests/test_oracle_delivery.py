"""Pins of the oracle's spike delivery and step loop (CPU only).

The brute force is the paper's PULL formulation (lst:pull): every receiver
sums, over a dense [delay][receiver][sender] weight tensor, the weights of the
senders that spiked `delay` steps ago.  It shares nothing with the oracle's
push loop and ring buffer except the sampled network and the thalamic counts,
and is run in numpy FP32 with propagators taken from the continuous LIF
solution.
"""
import math

import numpy as np
import pytest

TAU_M, TAU_S, C_M, DT = 10.0, 0.5, 250.0, 0.1
BETA = TAU_S * TAU_M / (TAU_M - TAU_S)


def kernel_u(s):
    return BETA / C_M * (np.exp(-s / TAU_M) - np.exp(-s / TAU_S))


def independent_constants():
    t_peak = math.log(TAU_M / TAU_S) * BETA
    w_f = 1.0 / kernel_u(t_peak)                       # pA per mV of PSP peak
    return dict(p11=np.float32(math.exp(-DT / TAU_S)), p22=np.float32(math.exp(-DT / TAU_M)),
                p21=np.float32(kernel_u(DT)), w_ext_q=int(round(w_f * 0.15 * 256)))


def pull_simulation(net, T_rec, n_steps):
    row_ptr, post, delay, w, wq = net.csr()
    N = net.N
    pre = np.repeat(np.arange(N), np.diff(row_ptr).astype(np.int64))
    Wd = np.zeros((64, N, N), np.int32)           # [delay][receiver][sender]
    np.add.at(Wd, (delay.astype(np.int64), post.astype(np.int64), pre), wq)
    k = independent_constants()
    U = net.u0().copy()
    I = np.zeros(N, np.float32)
    R = np.zeros(N, np.int64)
    hist = []                                     # spiking senders of each past step
    raster, inputs = [], []
    for t in range(n_steps):
        refr = R > 0
        x = k["p22"] * U + k["p21"] * I
        spike = (~refr) & (x >= np.float32(15.0))
        U = np.where(refr | spike, np.float32(0.0), x).astype(np.float32)
        R = np.where(refr, R - 1, np.where(spike, 20, 0))
        s = np.zeros(N, np.int64)
        for d in range(1, 64):
            if t - d < 0:
                break
            src = hist[t - d]
            if len(src):
                s += Wd[d][:, src].astype(np.int64).sum(axis=1)
        hist.append(np.nonzero(spike)[0])
        raster.extend((t, i) for i in hist[-1])
        inputs.append(s)
        q = T_rec[t].astype(np.int64) * k["w_ext_q"] + s
        I = (k["p11"] * I + q.astype(np.float32) * np.float32(2.0**-8)).astype(np.float32)
    return np.array(raster, dtype=np.int64).reshape(-1, 2), np.array(inputs), U, I, R


def pull_simulation_f64(net, T_rec, n_steps):
    """lst:pull in numpy float64 with the unquantised weights and FP64
    propagators from the continuous solution: the FP64 oracle's arithmetic
    up to the order of summation of a step's input."""
    row_ptr, post, delay, w, wq = net.csr()
    N = net.N
    pre = np.repeat(np.arange(N), np.diff(row_ptr).astype(np.int64))
    Wd = np.zeros((64, N, N), np.float64)         # [delay][receiver][sender]
    np.add.at(Wd, (delay.astype(np.int64), post.astype(np.int64), pre), w)
    p11, p22, p21 = math.exp(-DT / TAU_S), math.exp(-DT / TAU_M), kernel_u(DT)
    w_ext = 0.15 / kernel_u(math.log(TAU_M / TAU_S) * BETA)
    U = net.u0_f64().copy()
    I = np.zeros(N)
    R = np.zeros(N, np.int64)
    hist, raster, inputs, margin = [], [], [], np.inf
    for t in range(n_steps):
        refr = R > 0
        x = p22 * U + p21 * I
        margin = min(margin, float(np.abs(x[~refr] - 15.0).min()) if (~refr).any() else np.inf)
        spike = (~refr) & (x >= 15.0)
        U = np.where(refr | spike, 0.0, x)
        R = np.where(refr, R - 1, np.where(spike, 20, 0))
        s = np.zeros(N)
        for d in range(1, 64):
            if t - d < 0:
                break
            src = hist[t - d]
            if len(src):
                s += Wd[d][:, src].sum(axis=1)
        hist.append(np.nonzero(spike)[0])
        raster.extend((t, i) for i in hist[-1])
        inputs.append(s)
        I = p11 * I + (T_rec[t] * w_ext + s)
    return np.array(raster, dtype=np.int64).reshape(-1, 2), np.array(inputs), U, I, R, margin


def test_f64_pull_brute_force_reproduces_push(oracle):
    """The FP64 oracle (FP64 state, propagators and ring, unquantised
    weights) against an FP64 pull brute force on the 1 % circuit: the same
    raster spike for spike, and ring inputs and state equal up to the order
    of the additions.  A step's input sums at most a few hundred weights of
    at most ~1 nA, so a different order changes it by < 1e-9 pA; the state's
    recursions contract (p11, p22 < 1), so they stay within 1e-9 as well.
    Decisions flip only for a membrane value within that error of the
    threshold; the run's closest approach is reported and must be far
    larger."""
    net = oracle.Net(oracle.Config(scale=0.01, seed=3))
    sim = oracle.Sim(net, arith=oracle.ARITH_F64, record_inputs=True).run(1500)
    T_rec, w_rec = sim.recorded_inputs()
    raster, inputs, U, I, R, margin = pull_simulation_f64(net, T_rec, 1500)
    steps, ids = sim.raster()
    assert len(steps) > 10000 and margin > 1e-7, margin
    np.testing.assert_array_equal(raster[:, 0], steps)
    np.testing.assert_array_equal(raster[:, 1], ids)
    np.testing.assert_allclose(inputs, w_rec, rtol=0, atol=1e-9)
    st = sim.state()
    np.testing.assert_allclose(st["U"], U, rtol=0, atol=1e-9)
    np.testing.assert_allclose(st["I"], I, rtol=0, atol=1e-9)
    np.testing.assert_array_equal(st["R"], R)


@pytest.fixture(scope="module")
def tiny(oracle):
    net = oracle.Net(oracle.Config(scale=0.01, seed=3))
    sim = oracle.Sim(net, record_inputs=True).run(1500)
    return net, sim


def test_pull_brute_force_reproduces_push(oracle, tiny):
    net, sim = tiny
    T_rec, w_rec = sim.recorded_inputs()
    raster, inputs, U, I, R = pull_simulation(net, T_rec, 1500)
    steps, ids = sim.raster()
    assert len(steps) > 10000
    np.testing.assert_array_equal(inputs, w_rec)
    np.testing.assert_array_equal(raster[:, 0], steps)
    np.testing.assert_array_equal(raster[:, 1], ids)
    st = sim.state()
    np.testing.assert_array_equal(st["U"], U)
    np.testing.assert_array_equal(st["I"], I)
    np.testing.assert_array_equal(st["R"], R)


def test_pull_brute_force_reproduces_push_dev8(oracle):
    """The same dense lst:pull check on the dev8 weights (pair mean plus an
    8-bit deviation): the push delivery of the oracle does not depend on how
    the weights were quantised."""
    net = oracle.Net(oracle.Config(scale=0.01, seed=4, weight_mode=oracle.W_DEV8))
    sim = oracle.Sim(net, record_inputs=True).run(400)
    T_rec, w_rec = sim.recorded_inputs()
    raster, inputs, U, I, R = pull_simulation(net, T_rec, 400)
    steps, ids = sim.raster()
    assert len(steps) > 1000
    np.testing.assert_array_equal(inputs, w_rec)
    np.testing.assert_array_equal(raster[:, 0], steps)
    np.testing.assert_array_equal(raster[:, 1], ids)
    st = sim.state()
    np.testing.assert_array_equal(st["U"], U)
    np.testing.assert_array_equal(st["I"], I)


@pytest.mark.parametrize("scale,seed,steps,threads", [(0.05, 12, 600, 4), (0.01, 13, 900, 3)])
def test_threaded_step_loop_equals_serial(oracle, scale, seed, steps, threads):
    """The all-cores baseline loop (neurons in parallel, atomic int64 ring
    adds) gives the serial loop's raster, state, ring and counters bit for
    bit: every ring entry is an exact integer sum."""
    net = oracle.Net(oracle.Config(scale=scale, seed=seed))
    a = oracle.Sim(net).run(steps)
    b = oracle.Sim(net).run_threads(steps // 3, threads).run_threads(steps - steps // 3, threads)
    sa, ia = a.raster()
    sb, ib = b.raster()
    assert len(sa) > 1000
    np.testing.assert_array_equal(sa, sb)
    np.testing.assert_array_equal(ia, ib)
    x, y = a.state(), b.state()
    for k in ["U", "I", "R", "W"]:
        np.testing.assert_array_equal(x[k], y[k])
    assert a.counters() == b.counters()


def test_threaded_step_loop_refuses_what_it_does_not_do(oracle):
    net = oracle.Net(oracle.Config(scale=0.01, seed=1))
    with pytest.raises(oracle.OracleError):
        oracle.Sim(net, arith=oracle.ARITH_F64).run_threads(10, 2)
    with pytest.raises(oracle.OracleError):
        oracle.Sim(net, record_inputs=True).run_threads(10, 2)
    with pytest.raises(oracle.OracleError):
        oracle.Sim(net).run_threads(10, 0)


def test_delivered_events_and_charge_conservation(oracle, tiny):
    """Every spike activates each outgoing synapse exactly once: delivered
    events = sum of sender out-degrees, and the charge injected equals what
    was read from the ring plus what is still in it (int64, exact)."""
    net, sim = tiny
    row_ptr, post, delay, w, wq = net.csr()
    steps, ids = sim.raster()
    c = sim.counters()
    outdeg = np.diff(row_ptr.astype(np.int64))
    assert c["spikes"] == len(ids)
    assert c["events"] == int(outdeg[ids].sum())
    rowsum = np.add.reduceat(wq.astype(np.int64), row_ptr[:-1].astype(np.int64)) * (outdeg > 0)
    assert c["injected"] == int(rowsum[ids].sum())
    assert c["consumed"] + int(sim.state()["W"].sum()) == c["injected"]
    T, _ = sim.recorded_inputs()
    assert c["poisson"] == int(T.sum())


def test_raster_is_sorted_and_refractory(oracle, tiny):
    net, sim = tiny
    steps, ids = sim.raster()
    key = steps.astype(np.int64) * net.N + ids
    assert np.all(np.diff(key) > 0)
    order = np.lexsort((steps, ids))
    s2, i2 = steps[order].astype(np.int64), ids[order]
    same = i2[1:] == i2[:-1]
    assert np.all(np.diff(s2)[same] >= 21)


def test_resume_equals_one_run(oracle):
    """Splitting a run into pieces changes nothing (state carries over)."""
    net = oracle.Net(oracle.Config(scale=0.01, seed=5))
    a = oracle.Sim(net).run(700)
    b = oracle.Sim(net)
    for n in [1, 63, 64, 65, 7, 500]:
        b.run(n)
    for x, y in zip(a.raster(), b.raster()):
        np.testing.assert_array_equal(x, y)


def test_f64_and_int32_agree_statistically(oracle):
    """The FP64 oracle (unquantised weights, FP64 state) and the FP32/int32
    oracle give the same population rates on the tiny circuit."""
    net = oracle.Net(oracle.Config(scale=0.01, seed=11))
    a = oracle.Sim(net).run(5000)
    b = oracle.Sim(net, arith=oracle.ARITH_F64).run(5000)
    off = net.pop_offsets()
    ra = np.bincount(np.searchsorted(off, a.raster()[1], side="right") - 1, minlength=8)
    rb = np.bincount(np.searchsorted(off, b.raster()[1], side="right") - 1, minlength=8)
    np.testing.assert_allclose(ra, rb, rtol=0.05)


def test_degenerate_drives(oracle):
    """No synapses and no thalamic input: only neurons that start above
    threshold fire, once, at step 0 (p22 U0 >= 15 mV); a constant thalamic
    count gives exactly that count every step."""
    net = oracle.Net(oracle.Config(scale=0.01, bg_rate_hz=0.0, conn=np.zeros(64)))
    assert net.nsyn == 0
    sim = oracle.Sim(net).run(300)
    st, ids = sim.raster()
    k = independent_constants()
    expect = np.nonzero(k["p22"] * net.u0() >= np.float32(15.0))[0]
    np.testing.assert_array_equal(ids, expect)
    assert np.all(st == 0)
    assert sim.counters()["poisson"] == 0 and sim.counters()["events"] == 0
    net = oracle.Net(oracle.Config(scale=0.01, bg_const_T=1))
    sim = oracle.Sim(net, record_inputs=True).run(50)
    T, _ = sim.recorded_inputs()
    assert np.all(T == 1)
