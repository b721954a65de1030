"""Pins of the oracle's neuron update (eqn:mem, eqn:psc, eqn:ref) on one
synapse-less neuron driven by a chosen per-step input (CPU only).

References are written from the LIF ODE, not from the propagators: a current
kick J at time 0 gives I(s) = J exp(-s/tau_syn) and
U(s) = J/C_m * beta * (exp(-s/tau_m) - exp(-s/tau_syn)), beta =
tau_syn tau_m / (tau_m - tau_syn); inputs superpose.  In the discrete loop the
input of step k enters I after step k and reaches U one step later, so the
state stored after step t sees kick k at elapsed time (t - k) * dt.
"""
import numpy as np
import pytest

TAU_M, TAU_S, C_M, DT = 10.0, 0.5, 250.0, 0.1
BETA = TAU_S * TAU_M / (TAU_M - TAU_S)


def kernel_u(s):
    return BETA / C_M * (np.exp(-s / TAU_M) - np.exp(-s / TAU_S))


def superposed(q_pA):
    """U and I after each step for a per-step input sequence (pA), by
    superposing the continuous single-kick responses."""
    n = len(q_pA)
    t = np.arange(n)
    U = np.zeros(n)
    I = np.zeros(n)
    for k in np.nonzero(q_pA)[0]:
        s = (t[k:] - k) * DT
        U[k:] += q_pA[k] * kernel_u(s)
        I[k:] += q_pA[k] * np.exp(-s / TAU_S)
    return U, I


def test_single_kick_f64(oracle):
    q = np.zeros(400)
    q[3] = 123.4
    u, i, r = oracle.single_neuron(q, arith=oracle.ARITH_F64)
    U, I = superposed(q)
    assert np.all(r == 0)
    np.testing.assert_allclose(i, I, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(u, U, rtol=1e-11, atol=1e-16)


def test_single_kick_f32(oracle):
    q = np.zeros(400, dtype=np.int64)
    q[0] = 22479                       # one thalamic kick, 2^-8 pA units
    u, i, r = oracle.single_neuron(q)
    U, I = superposed(q.astype(np.float64) / 256.0)
    # FP32 state accumulates a few ulps of rounding per step
    np.testing.assert_allclose(i, I, rtol=2e-6 * 50, atol=1e-30)
    np.testing.assert_allclose(u[1:200], U[1:200], rtol=2e-5)


def test_psp_peak_is_the_psp_amplitude(oracle):
    """A kick of w_f * 0.15 pA peaks at 0.15 mV near 1.58 ms (definition of
    w_f, Sec. 2.2); the grid maximum sits at 1.5 or 1.6 ms just below it."""
    k = oracle.constants()
    q = np.zeros(300)
    q[0] = k["w_f"] * 0.15
    u, _, _ = oracle.single_neuron(q, arith=oracle.ARITH_F64)
    assert int(np.argmax(u)) in (15, 16)
    assert 0.15 * (1 - 2e-3) < u.max() <= 0.15
    qq = np.zeros(300, dtype=np.int64)
    qq[0] = k["w_ext_q"]
    uf, _, _ = oracle.single_neuron(qq)
    assert abs(float(uf.max()) - u.max()) < 1e-5


@pytest.mark.parametrize("arith", ["f32", "f64"])
def test_step_drive_closed_form(oracle, arith):
    """Constant drive below threshold: J = w_f * 0.07 mV every step gives the
    superposed response, approaching p21 J / ((1-p11)(1-p22)) ~ 8.2 mV."""
    k = oracle.constants()
    n = 3000
    if arith == "f32":
        jq = int(round(k["w_f"] * 0.07 * 256))
        q = np.full(n, jq, dtype=np.int64)
        u, i, r = oracle.single_neuron(q)
        U, I = superposed(np.full(n, jq / 256.0))
        tol = 1e-5
    else:
        q = np.full(n, k["w_f"] * 0.07)
        u, i, r = oracle.single_neuron(q, arith=oracle.ARITH_F64)
        U, I = superposed(q)
        tol = 1e-11
    assert np.all(r == 0) and u.max() < 15.0
    np.testing.assert_allclose(i, I, rtol=tol)
    np.testing.assert_allclose(u[5:], U[5:], rtol=tol)
    assert 8.0 < u[-1] < 8.4


@pytest.mark.parametrize("arith", ["f32", "f64"])
def test_refractory_and_reset_invariants(oracle, arith):
    """Strong drive: each spike stores U = 0 and starts 20 refractory steps
    during which U stays 0 and R counts down (eqn:ref, lst:push), so the
    inter-spike interval is at least 21 steps; no stored U reaches 15 mV."""
    n = 4000
    if arith == "f32":
        q = np.full(n, 60000, dtype=np.int64)
        u, i, r = oracle.single_neuron(q)
    else:
        q = np.full(n, 60000 / 256.0)
        u, i, r = oracle.single_neuron(q, arith=oracle.ARITH_F64)
    spikes = np.nonzero(r == 20)[0]
    assert len(spikes) > 20
    assert np.all(np.diff(spikes) >= 21)
    assert np.all(u < 15.0)
    for s in spikes[:-1]:
        assert np.all(u[s:s + 21] == 0.0)
        np.testing.assert_array_equal(r[s:s + 21], np.arange(20, -1, -1))
    # The first crossing happens where the superposed continuous solution
    # first reaches 15 mV (well separated from the grid neighbours here).
    U, _ = superposed(np.full(n, 60000 / 256.0))
    first = int(np.argmax(U >= 15.0))
    assert spikes[0] == first
    assert U[first - 1] < 15.0 - 1e-3 and U[first] > 15.0 + 1e-3
