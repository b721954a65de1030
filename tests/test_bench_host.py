"""Host-side logic of bench.py (no GPU): the algorithmic byte model, the
roofline block built from a leg's timing, the committed rocprofv3 traffic
records it attaches only while they match the kernel sources and launch
length, and the refusal of more than one GPU."""
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


class _Engines:
    ENGINE_STEPWISE, ENGINE_PERSISTENT, ENGINE_LDS, ENGINE_BAND = 1, 2, 3, 4


def _current(bench, kernel, wl, fmt):
    """The committed traffic record if its source hash matches the kernel's
    sources as they are now, else None (counters of an older kernel)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{wl}_{fmt}.json")
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(ROOT, "paper_2405_02019_amd", "csrc", f), "rb").read())
    return rec if h.hexdigest() == rec["kernel_source_sha256"] else None


def test_algorithmic_bytes(bench):
    """Per step: 8 bytes per neuron (ring word read and cleared); per
    synaptic event the record plus a 4-byte ring word; 24 bytes per spike."""
    ring, syn = bench.algorithmic_bytes(77169, 10, 1000, 8.0)
    assert ring == 8.0 * 77169
    assert syn == 12.0 * 1000 + 24.0 * 10
    assert bench.algorithmic_bytes(1, 0, 1000, 3.0)[1] == 7.0 * 1000


def test_roofline_from_a_leg(bench):
    """achieved = algorithmic bytes per launch / average launch time, against
    the 8 TB/s HBM peak; the full-scale plain record is attached, with its L2
    counters, while its hash matches the kernel sources (else traffic is
    null)."""
    leg = {"gpu_ms": 10 * 34.6, "launches": 10, "bytes": 10 * 1.77e10, "fmt": "plain",
           "info": {"engine": _Engines.ENGINE_LDS, "chunk_steps": 10000}}
    r = bench.roofline(_Engines, leg, "full")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert abs(r["avg_launch_ms"] - 34.6) < 1e-9
    assert abs(r["achieved"] - 1.77e10 / 34.6e-3 / 1e9) < 1e-6
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-12
    rec = _current(bench, "k_lds", "full", "plain")
    if rec is None:
        assert r["traffic"] is None and "cache" not in r
    else:
        assert r["traffic"] == rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
        assert 0.0 < r["cache"]["l2_hit_rate"] < 1.0
    assert r["kernel"].startswith("k_lds")


def test_traffic_records_only_for_matching_sources_and_launches(bench):
    """The traffic record is attached for the kernels and workloads the
    committed profiles cover while their sources are unchanged, and not for
    another launch length, another workload or format, or an unknown
    kernel."""
    for kernel, wl, fmt in [("k_lds", "full", "plain"), ("k_band", "x4", "plain"),
                            ("k_band", "batch", "compressed")]:
        rec = bench.profile_record(kernel, wl, fmt, 10000)
        assert (rec is None) == (_current(bench, kernel, wl, fmt) is None), (kernel, wl, fmt)
        if rec is not None:
            assert rec["fetch_bytes_per_launch"] > 0 and rec["kernel_us_per_launch"] > 0
    assert bench.profile_record("k_lds", "full", "plain", 1000) is None
    assert bench.profile_record("k_lds", "full", "dev8", 10000) is None
    assert bench.profile_record("k_update", "full", "plain", 10000) is None


def test_more_than_one_gpu_is_refused():
    """bench.py --gpus 2 exits with a message before touching a GPU."""
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert p.returncode != 0
    assert "one GPU" in p.stderr
