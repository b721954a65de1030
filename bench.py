#!/usr/bin/env python
"""Benchmark: the full-scale Potjans-Diesmann microcircuit on one MI355X.

One bench "step" is 10,000 simulation steps of 0.1 ms = 1 s of biological
time, so ms_per_step / 1000 is the real-time factor (wall / biological time,
the paper's RTF).  Defaults: 1 untimed warm-up second, then 10 timed seconds
(the paper's 10 s runs).  The timed region runs from the first step launch to
the read-back of the timed window's spike raster, bracketed by
torch.cuda.synchronize(); the network is built and uploaded before it.

Reported value: synaptic events per second (device-counted activations of
synapses by spikes) over the timed region.  The same line carries the
real-time factor, the compressed-synapse leg, the roofline of the dominant
kernel (timed live with HIP events on the library's stream) and the CPU
oracle's throughput on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

STEPS_PER_BIO_SECOND = 10000
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s


def algorithmic_bytes(n_neurons, spikes, events, rec_bytes):
    """Bytes a step loop must move at least (roofline):
    ring row read + clear per neuron and step, one record plus one 4-byte ring
    word per synaptic event, row pointers and raster entry per spike."""
    return 8.0 * n_neurons, (rec_bytes + 4.0) * events + 24.0 * spikes


def run_leg(P, fmt, engine, warm_bio_s, timed_bio_s, log):
    import torch
    t_build = time.perf_counter()
    sim = P.Simulator(P.Instance(scale=1.0, seed=1), syn_format=fmt, engine=engine)
    build_s = time.perf_counter() - t_build
    info = sim.info()
    log(f"[bench] {fmt}: built in {build_s:.1f} s ({info['n_synapses_total']} synapses, "
        f"engine {info['engine']}, block {info['block_size']}, grid {info['grid_blocks']})")
    if warm_bio_s:
        sim.step(warm_bio_s * STEPS_PER_BIO_SECOND)
    s0 = sim.state()
    t0_step = s0["t"]
    n_steps = timed_bio_s * STEPS_PER_BIO_SECOND
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    gpu_ms = sim.time_steps(n_steps)              # HIP events on the library's stream
    steps, ids = sim.spikes(0, t0_step, t0_step + n_steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    s1 = sim.state()
    events = s1["events"] - s0["events"]
    spikes = s1["spikes"] - s0["spikes"]
    assert spikes == len(ids), (spikes, len(ids))
    n = s1["n_neurons"]
    rec = 8.0 if fmt == "plain" else 5.0
    ring_b, syn_b = algorithmic_bytes(n, spikes, events, rec)
    total_bytes = ring_b * n_steps + syn_b
    chunked = info["engine"] in (P.ENGINE_PERSISTENT, P.ENGINE_LDS)
    launches = -(-n_steps // info["chunk_steps"]) if chunked else 2 * n_steps
    sim.close()
    return {
        "fmt": fmt, "wall_s": wall, "gpu_ms": gpu_ms, "events": events, "spikes": spikes,
        "n_steps": n_steps, "n_neurons": n, "build_s": build_s, "info": info,
        "bytes": total_bytes, "launches": launches,
    }


def kernel_name(P, info):
    """Name of the dominant kernel of an engine (as rocprofv3 lists it)."""
    e = info["engine"]
    if e == P.ENGINE_LDS:
        return "k_lds"
    if e == P.ENGINE_PERSISTENT:
        return "k_persistent"
    return "k_update + k_transfer"


def measured_traffic(kernel, fmt):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, scaled by the copy calibration -- only while the kernel source is
    the one the counters were taken on."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_full_scale_{fmt}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_2405_02019_amd", "csrc", "kernels.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["kernel_source_sha256"]:
        return None
    return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def cpu_baseline(n_steps, log):
    """The oracle (plain C, single-threaded step loop) on the same full-scale
    network; network sampling is not timed."""
    from oracle import pyoracle as O
    t = time.perf_counter()
    net = O.Net(O.Config(scale=1.0, seed=1))
    log(f"[bench] oracle network built in {time.perf_counter() - t:.1f} s")
    sim = O.Sim(net)
    t = time.perf_counter()
    sim.run(n_steps)
    wall = time.perf_counter() - t
    c = sim.counters()
    return {"value": c["events"] / wall, "unit": "synaptic events/s", "cores": 1, "kind": "oracle",
            "sample": f"full-scale microcircuit (77,169 neurons, {net.nsyn} synapses), steps 0-{n_steps} "
                      f"({n_steps / STEPS_PER_BIO_SECOND:.2f} s bio) of the same seed, "
                      f"{c['events']} events in {wall:.1f} s",
            "rtf": wall / (n_steps / STEPS_PER_BIO_SECOND)}


def copy_calibration(log):
    """Plain device-to-device copy of 1 GiB, for scaling the FETCH_SIZE and
    WRITE_SIZE counters (run under rocprofv3 --pmc)."""
    import torch
    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log("[bench] copied 3 x 1 GiB")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed seconds of biological time")
    ap.add_argument("--warmup", type=int, default=1, help="untimed seconds of biological time")
    ap.add_argument("--engine", default="auto", choices=["auto", "stepwise", "persistent", "lds"])
    ap.add_argument("--no-compressed", action="store_true", help="skip the compressed-synapse leg")
    ap.add_argument("--cpu-steps", type=int, default=4000,
                    help="oracle steps for the CPU baseline (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the 1 GiB copy used to scale HBM counters")
    args = ap.parse_args()

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: this build simulates one microcircuit (or one batch) "
              f"per device and has no multi-GPU path; got --gpus {args.gpus}", file=sys.stderr)
        sys.exit(2)
    if int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py is single-process; run it without torch.distributed", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(log)
        return
    import paper_2405_02019_amd as P

    plain = run_leg(P, "plain", args.engine, args.warmup, args.steps, log)
    comp = None if args.no_compressed else run_leg(P, "compressed", args.engine, args.warmup,
                                                   args.steps, log)
    bio = float(args.steps)
    value = plain["events"] / plain["wall_s"]
    avg_launch_ms = plain["gpu_ms"] / plain["launches"]
    achieved = plain["bytes"] / plain["launches"] / (avg_launch_ms * 1e-3) / 1e9
    kname = kernel_name(P, plain["info"])
    kernel = kname
    if plain["info"]["engine"] in (P.ENGINE_PERSISTENT, P.ENGINE_LDS):
        kernel += " (one cooperative launch per chunk of %d steps)" % plain["info"]["chunk_steps"]
    out = {
        "metric": "realtime factor & synaptic events/s, full PD microcircuit; plain vs compressed",
        "value": value,
        "unit": "synaptic events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * plain["wall_s"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 state, int32 fixed-point synaptic input",
        "data": "synthetic: Potjans-Diesmann network sampled from the paper's tables (seed 1)",
        "config": {"workload": "full-scale PD microcircuit, 77,169 neurons, %d synapses, "
                               "dt 0.1 ms, 10 s biological time per measurement" % plain["info"]["n_synapses_total"],
                   "steps_per_bench_step": STEPS_PER_BIO_SECOND, "syn_format": "plain8",
                   "engine": plain["info"]["engine"], "block": plain["info"]["block_size"],
                   "grid": plain["info"]["grid_blocks"], "chunk_steps": plain["info"]["chunk_steps"]},
        "rtf": plain["wall_s"] / bio,
        "bio_per_wall": bio / plain["wall_s"],
        "spikes_per_step": plain["spikes"] / plain["n_steps"],
        "events_per_step": plain["events"] / plain["n_steps"],
        "gpu_ms_timed": plain["gpu_ms"],
        "build_s": plain["build_s"],
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(kname, "plain"),
                     "kernel": kernel,
                     "avg_launch_ms": avg_launch_ms,
                     "bytes_per_launch": plain["bytes"] / plain["launches"]},
        "paper_context": {"fpga_rtf_gmem_mono_s": 4.79, "fpga_rtf_best_horiz_multi": 0.79,
                          "hardware": "1 Intel Agilex 7 FPGA (numbers quoted from the paper)"},
    }
    if comp:
        out["compressed"] = {"value": comp["events"] / comp["wall_s"], "unit": "synaptic events/s",
                             "rtf": comp["wall_s"] / bio, "ms_per_step": 1000.0 * comp["wall_s"] / args.steps,
                             "spikes_per_step": comp["spikes"] / comp["n_steps"],
                             "syn_format": "compressed5", "build_s": comp["build_s"],
                             "device_bytes": comp["info"]["device_bytes"]}
    if args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps, log)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
