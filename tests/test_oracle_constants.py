"""Pins of the oracle's model constants and random streams (CPU only).

Each check compares the oracle with something other than itself: values the
paper prints, the LIF ODE solved numerically, or published known answers.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.optimize import minimize_scalar
from scipy.stats import norm

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_values.json")))

TAU_M, TAU_S, C_M, DT = 10.0, 0.5, 250.0, 0.1   # Table tab:params


def _ode(i0, u0, t_end, dense=False):
    """LIF membrane with an exponentially decaying current (eqn:lif plus the
    synaptic current): dI/dt = -I/tau_syn, dU/dt = -U/tau_m + I/C_m
    (pA, pF, ms, mV), integrated to 1e-13 relative accuracy."""
    return solve_ivp(lambda t, y: [-y[0] / TAU_S, -y[1] / TAU_M + y[0] / C_M], (0.0, t_end),
                     [i0, u0], method="DOP853", rtol=1e-13, atol=1e-18, dense_output=dense)


def test_constants_match_printed_values(oracle):
    k = oracle.constants()
    for name in ["w_f", "p11", "p22", "p21"]:
        assert abs(k[name] - GOLD[name]["value"]) <= GOLD[name]["abs_tol"], name


def test_propagators_are_the_exact_ode_solution(oracle):
    """p11, p21, p22 advance (I, U) by one step of 0.1 ms exactly (eqn:p11p22,
    eqn:p21): a unit current gives (p11, p21), a unit potential (0, p22)."""
    k = oracle.constants()
    sol = _ode(1.0, 0.0, DT)
    assert sol.y[0, -1] == pytest.approx(k["p11"], rel=1e-12)
    assert sol.y[1, -1] == pytest.approx(k["p21"], rel=1e-11)
    sol = _ode(0.0, 1.0, DT)
    assert sol.y[1, -1] == pytest.approx(k["p22"], rel=1e-12)
    assert abs(sol.y[0, -1]) == 0.0


def test_wf_maps_psp_amplitude_to_current(oracle):
    """w_f is the PSC amplitude (pA) whose PSP peaks at 1 mV (Sec. 2.2)."""
    k = oracle.constants()
    sol = _ode(k["w_f"] * 0.15, 0.0, 5.0, dense=True)
    res = minimize_scalar(lambda t: -sol.sol(t)[1], bounds=(0.5, 3.0), method="bounded",
                          options={"xatol": 1e-10})
    assert -res.fun == pytest.approx(0.15, rel=1e-9)
    # the continuous peak time is ln(tau_m/tau_s) tau_s tau_m / (tau_m - tau_s)
    assert res.x == pytest.approx(math.log(TAU_M / TAU_S) * TAU_S * TAU_M / (TAU_M - TAU_S),
                                  abs=1e-6)


def test_fp32_propagators_are_far_from_rounding_ties(oracle):
    """Any faithfully rounded exp gives the same FP32 propagators: each FP64
    value lies well inside its FP32 rounding interval."""
    k = oracle.constants()
    for name in ["p11", "p22", "p21"]:
        x = k[name]
        f = np.float32(x)
        assert float(f) == k[name + "f"]
        ulp = float(np.spacing(f))
        assert abs(x - float(f)) <= 0.4 * ulp, name


def test_thalamic_weight_in_fixed_point(oracle):
    k = oracle.constants()
    # 0.15 mV thalamic PSP -> w_f * 0.15 pA = 87.8085 pA -> 22479 units of 2^-8 pA
    assert k["w_ext"] == pytest.approx(87.8085, abs=1e-4)
    assert k["w_ext_q"] == 22479


def test_ring_buffer_depth(oracle):
    """Sec. 3.2: 64 rows suffice since P(N(1.5, 0.75) <= 6.4 ms) ~ 1 - 3.2e-11."""
    g = GOLD["delay_tail_cdf"]
    assert norm.cdf(6.4, 1.5, 0.75) == pytest.approx(g["value"], abs=g["abs_tol"])
    g = GOLD["ring_bytes"]
    assert 64 * 4 * GOLD["total_neurons"]["value"] == pytest.approx(g["value"], rel=g["rel_tol"])


def test_philox_known_answers(oracle):
    with open(os.path.join(HERE, "golden", "philox_kat.txt")) as f:
        rows = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert oracle.philox4x32_10(v[0:4], v[4:6]) == v[6:10]


@pytest.mark.parametrize("lam", [0.0, 1e-12, 0.3, 1.2, 1.28, 1.52, 2.32, 5.0, 20.0])
def test_poisson_table_is_the_poisson_cdf(oracle, lam):
    """thr[k] / 2^32 is P(T <= k) to 2^-32, and the mass lumped into the last
    count (beyond the table) is below 2^-32."""
    from scipy.stats import poisson
    thr = oracle.poisson_table(lam)
    assert np.all(np.diff(thr.astype(np.int64)) >= 0)
    for k, t in enumerate(thr):
        assert abs(float(t) / 2**32 - poisson.cdf(k, lam)) <= 2**-32 + 1e-15
    assert poisson.sf(len(thr), lam) < 2**-32
    if lam == 0.0:
        assert len(thr) == 0


def test_poisson_counts_have_poisson_moments(oracle):
    """Thalamic counts T drawn in the step loop: mean and variance v_th K dt per
    population (Sec. 2.2) within 5 standard errors."""
    net = oracle.Net(oracle.Config(scale=0.01))
    sim = oracle.Sim(net, record_inputs=True).run(3000)
    T, _ = sim.recorded_inputs()
    off = net.pop_offsets()
    K = [1600, 1500, 2100, 1900, 2000, 1900, 2900, 2100]
    for p in range(8):
        x = T[:, off[p]:off[p + 1]].ravel().astype(np.float64)
        lam = 8.0 * K[p] * 1e-4
        n = x.size
        assert abs(x.mean() - lam) < 5 * math.sqrt(lam / n), p
        # Var of the sample variance of a Poisson: (mu4 - sigma^4) / n, mu4 = lam(1+3 lam)
        se_var = math.sqrt((lam * (1 + 3 * lam) - lam * lam) / n)
        assert abs(x.var() - lam) < 5 * se_var, p
    # "L23/exc neurons receive about 8 x 1,600 = 12,800 thalamic spikes per second"
    l23e = T[:, off[0]:off[1]].mean() * 1e4
    assert l23e == pytest.approx(GOLD["thalamic_rate_l23e"]["value"], rel=0.02)
