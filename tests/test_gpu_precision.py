"""Precision of the FP32/int32 paths against the FP64 oracle (Sec. 4.1).

The GPU paths reproduce their int32 oracles bit for bit (test_gpu_parity);
here the plain path, the compressed form (16-bit weights, Sec. 5.3) and the
deviation form (the pair's mean plus an 8-bit deviation, Sec. 5.3) are
compared with the FP64 oracle (FP64 state and propagators, unquantised
weights), which they are not expected to match spike for spike.  Bar:
population rates within 5 % and mean CV of inter-spike intervals within 0.05
of the FP64 run on the full-scale circuit (seed 1), over [1 s, 10 s) as in the
paper's statistics; and the paper's own comparison, the KL divergence between
the distributions (single-neuron rates, CVs of ISIs, Pearson coefficients of
binned trains) of the FP64 run and ours, averaged over populations, within
the divergence between seeds of the FP64 run.  The FP64 figures are stored in
golden/f64_full_scale_seed1.json (written by golden/make_f64_stats.py from the
oracle alone); the step of the first raster difference is reported."""
import json
import os
import sys

import numpy as np
import pytest

from spike_stats import (STAT_NAMES, cv_isi, first_digest_divergence, first_divergence,
                         kde_on_grid, kl_divergence, population_distributions, rates_hz,
                         step_digest)

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "f64_full_scale_seed1.json")


def say(*a):
    print("[gpu-precision]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ref():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def runs(ref, full_scale_runs):
    assert ref["steps"] == 100000 and ref["seed"] == 1
    return {fmt: (r["steps"], r["ids"]) for fmt, r in full_scale_runs.items()}


@pytest.mark.timeout(600)
@pytest.mark.parametrize("fmt", ["plain", "compressed", "dev8"])
def test_rates_and_cv_isi_match_f64(ref, runs, fmt):
    off = np.array(ref["pop_offsets"])
    t0, t1 = ref["window"]
    r_ref, c_ref = np.array(ref["rates_hz"]), np.array(ref["cv_isi"])
    r = rates_hz(*runs[fmt], off, t0, t1)
    c = cv_isi(*runs[fmt], off, t0, t1)
    div = first_digest_divergence(step_digest(*runs[fmt], len(ref["digest"])), ref["digest"])
    say(fmt, "rates", np.round(r, 3), "f64", np.round(r_ref, 3))
    say(fmt, "rel. rate error", np.round(np.abs(r / r_ref - 1), 4))
    say(fmt, "cv", np.round(c, 3), "f64", np.round(c_ref, 3))
    say(fmt, "first raster difference from f64 at step", div)
    assert np.all(r_ref > 0.1)
    np.testing.assert_allclose(r, r_ref, rtol=0.05)
    assert np.all(np.abs(c - c_ref) <= 0.05)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("fmt", ["compressed", "dev8"])
def test_compressed_divergence_from_plain_is_reported(runs, fmt):
    div = first_divergence(*runs[fmt], *runs["plain"])
    say("first raster difference", fmt, "vs plain at step", div)
    # Weight quantisation (2^-5 pA, or steps of 0.04 sd of the pair)
    # perturbs currents slightly: the rasters separate, but only after
    # recurrent input has arrived.
    assert div is None or div > 0


@pytest.mark.timeout(600)
@pytest.mark.parametrize("fmt", ["plain", "compressed", "dev8"])
def test_distributions_within_seed_variation(ref, runs, fmt):
    """Sec. 4.1: per statistic, the KL divergence from the FP64 run (same
    seed), averaged over the eight populations, lies within the seed-to-seed
    divergence of the FP64 model (at most the largest over the twelve
    ordered pairs of seeds 1-4)."""
    off = np.array(ref["pop_offsets"])
    t0, t1 = ref["window"]
    ours = population_distributions(*runs[fmt], off, t0, t1)
    for name in STAT_NAMES:
        kls = []
        for p, entry in enumerate(ref["dist"]):
            e = entry[name]
            g = np.array(e["grid"])
            kls.append(kl_divergence(np.array(e["seed1"]), kde_on_grid(ours[p][name], g), g))
        y = ref["seed_kl"][name]
        say(fmt, name, "KL to FP64 per population", np.round(kls, 4))
        say(fmt, name, "population mean %.4g; between FP64 seeds: mean %.4g, max %.4g"
            % (np.mean(kls), y["mean"], y["max"]))
        assert np.mean(kls) <= y["max"], (name, np.mean(kls), y["max"])
