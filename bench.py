#!/usr/bin/env python
"""Benchmark: the Potjans-Diesmann microcircuit on one MI355X.

One bench "step" is 10,000 simulation steps of 0.1 ms = 1 s of biological
time, so ms_per_step / 1000 is the real-time factor (wall / biological time,
the paper's RTF).  The timed region runs from the first step launch to the
read-back of the timed window's spike rasters, bracketed by
torch.cuda.synchronize(); networks are built and uploaded before it.

Workloads (--workload selects the headline one):
  full   the full-scale circuit, 77,169 neurons, ~3e8 synapses; plain,
         compressed and dev8 (pair mean plus 8-bit deviation, 3-byte
         synapses) legs; defaults 1 warm-up + 10 timed seconds (the paper's
         10 s runs).  The default.
  batch  64 independent instances of uneven scale (5-20 %), g and background
         rate, compressed synapses; 2 timed seconds.
  x4     four times the neurons, full in-degrees (308,676 neurons, ~1.2e9
         synapses); plain and compressed legs; 5 timed seconds.
With the full workload as the headline, the batch and x4 workloads run too
(unless --no-extra) and are reported under "workloads".

Reported value: synaptic events per second (device-counted activations of
synapses by spikes) of the first leg over the timed region.  The line also
carries the real-time factor, the other legs, the roofline of the dominant
kernel (timed live with HIP events on the library's stream) and, for the
full workload, the CPU oracle's throughput on a bounded sample.
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

WORKLOADS = {
    "full": {"legs": ["plain", "compressed", "dev8"], "steps": 10,
             "name": "full-scale PD microcircuit, 77,169 neurons, {syn} synapses, dt 0.1 ms"},
    "batch": {"legs": ["compressed"], "steps": 2,
              "name": "64 independent PD instances, scale U[5%,20%], g U[-6,-3], background "
                      "U[6,10] Hz, full in-degrees; {neurons} neurons, {syn} synapses, dt 0.1 ms"},
    "x4": {"legs": ["plain", "compressed"], "steps": 5,
           "name": "4x PD microcircuit with full in-degrees, {neurons} neurons, {syn} synapses, "
                   "dt 0.1 ms"},
}
# Sources whose bytes (concatenated in this order) a committed counter record
# must match: the kernel's file and the device helpers it includes.
KERNEL_SOURCES = {"k_lds": ["kernels.hip", "device.hpp", "engine.hpp"],
                  "k_persistent": ["kernels.hip", "device.hpp"],
                  "k_band": ["band.hip", "device.hpp", "engine.hpp"]}


def algorithmic_bytes(n_neurons, spikes, events, rec_bytes):
    """Bytes a step loop must move at least: ring row read + clear per neuron
    and step, one record plus one 4-byte ring word per synaptic event, row
    pointers and raster entry per spike."""
    return 8.0 * n_neurons, (rec_bytes + 4.0) * events + 24.0 * spikes


def run_leg(P, instances, fmt, engine, chunk, warm_bio_s, timed_bio_s, log, tune_steps=0,
            tune_cache=None):
    import torch
    t_build = time.perf_counter()
    sim = P.Simulator(instances, syn_format=fmt, engine=engine, chunk_steps=chunk,
                      tune_steps=tune_steps, tune_cache=tune_cache)
    build_s = time.perf_counter() - t_build
    info = sim.info()
    layout = sim.tune_report
    if layout:
        log(f"[bench] {fmt}: layout tuned over {layout['candidates']} candidates (0 = cached): "
            f"engine {layout['engine']}, window {layout['window_neurons']}, "
            f"{layout['us_per_step_first']:.2f} -> {layout['us_per_step_best']:.2f} us/step")
    log(f"[bench] {fmt}: built in {build_s:.1f} s ({info['n_synapses_total']} synapses, "
        f"engine {info['engine']}, block {info['block_size']}, grid {info['grid_blocks']}, "
        f"window {info['window_neurons']}, ring rows {info['ring_rows']}, "
        f"launches/chunk {info['launches_per_chunk']}, graphs {info['graphs']})")
    if warm_bio_s:
        sim.step(int(warm_bio_s * STEPS_PER_BIO_SECOND))
    tune = None
    if info["engine"] in (P.ENGINE_PERSISTENT, P.ENGINE_STEPWISE):   # the LDS engines' shape
        tune = sim.autotune(500)                                     # is fixed by their layout
        info = sim.info()
        log(f"[bench] {fmt}: autotuned over {tune['candidates']} shapes: block {tune['block_size']}, "
            f"grid {tune['grid_blocks']}, quads/thread {tune['quads_per_thread']}, "
            f"{tune['us_per_step_first']:.2f} -> {tune['us_per_step_best']:.2f} us/step")
    ni = len(instances)
    s0 = [sim.state(i) for i in range(ni)]
    t0_step = s0[0]["t"]
    sim.discard_spikes(t0_step)
    n_steps = int(timed_bio_s * STEPS_PER_BIO_SECOND)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    gpu_ms = sim.time_steps(n_steps)              # HIP events on the library's stream
    n_raster = 0
    for i in range(ni):
        steps, ids = sim.spikes(i, t0_step, t0_step + n_steps)
        n_raster += len(ids)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    s1 = [sim.state(i) for i in range(ni)]
    events = sum(b["events"] - a["events"] for a, b in zip(s0, s1))
    spikes = sum(b["spikes"] - a["spikes"] for a, b in zip(s0, s1))
    assert spikes == n_raster, (spikes, n_raster)
    n = sum(b["n_neurons"] for b in s1)
    windowed = info["engine"] in (P.ENGINE_LDS, P.ENGINE_BAND)
    rec = {"plain": 8.0, "dev8": 3.0}.get(fmt, 4.0 if windowed else 5.0)
    ring_b, syn_b = algorithmic_bytes(n, spikes, events, rec)
    total_bytes = ring_b * n_steps + syn_b
    chunked = info["engine"] in (P.ENGINE_PERSISTENT, P.ENGINE_LDS, P.ENGINE_BAND)
    launches = (-(-n_steps // info["chunk_steps"]) * info["launches_per_chunk"] if chunked
                else 2 * n_steps)
    sim.close()
    return {
        "fmt": fmt, "wall_s": wall, "gpu_ms": gpu_ms, "events": events, "spikes": spikes,
        "n_steps": n_steps, "n_neurons": n, "build_s": build_s, "info": info,
        "bytes": total_bytes, "launches": launches, "rec_bytes": rec, "tune": tune,
        "layout": layout,
    }


def kernel_name(P, info):
    """Name of the dominant kernel of an engine (as rocprofv3 lists it)."""
    e = info["engine"]
    if e == P.ENGINE_LDS:
        return "k_lds"
    if e == P.ENGINE_BAND:
        return "k_band"
    if e == P.ENGINE_PERSISTENT:
        return "k_persistent"
    return "k_update + k_transfer"


def profile_record(kernel, workload, fmt, chunk):
    """The committed rocprofv3 counter summary of a kernel and workload
    (profiles/traffic_<kernel>_<workload>_<fmt>.json) -- only while the
    kernel's sources are the ones the counters were taken on, for the same
    launch length."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}_{fmt}.json")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCES:
        return None
    rec = json.load(open(path))
    sha = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        sha.update(open(os.path.join(ROOT, "paper_2405_02019_amd", "csrc", f), "rb").read())
    if sha.hexdigest() != rec["kernel_source_sha256"]:
        return None
    if rec.get("chunk_steps") != chunk:
        return None
    return rec


def roofline(P, leg, workload):
    avg_launch_ms = leg["gpu_ms"] / leg["launches"]
    achieved = leg["bytes"] / leg["launches"] / (avg_launch_ms * 1e-3) / 1e9
    kname = kernel_name(P, leg["info"])
    kernel = kname
    if leg["info"]["engine"] in (P.ENGINE_PERSISTENT, P.ENGINE_LDS, P.ENGINE_BAND):
        kernel += " (cooperative launches of %d steps)" % leg["info"]["chunk_steps"]
    rec = profile_record(kname, workload, leg["fmt"], leg["info"]["chunk_steps"])
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS,
           "traffic": (rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]) if rec else None,
           "traffic_kind": "L2-to-fabric bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a 1 GiB "
                           "copy; Infinity Cache hits are included, the counters cannot separate them)",
           "kernel": kernel, "avg_launch_ms": avg_launch_ms,
           "bytes_per_launch": leg["bytes"] / leg["launches"]}
    if rec and "cache" in rec:
        out["cache"] = rec["cache"]
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


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
    out = {"value": c["events"] / wall, "unit": "synaptic events/s", "cores": 1, "kind": "oracle",
           "sample": f"full-scale microcircuit (77,169 neurons, {net.nsyn} synapses), steps 0-{n_steps} "
                     f"({n_steps / STEPS_PER_BIO_SECOND:.2f} s bio) of the same seed, "
                     f"{c['events']} events in {wall:.1f} s, one thread",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "rtf": wall / (n_steps / STEPS_PER_BIO_SECOND)}
    sim.close()
    # The same steps on every host core the process may use (OpenMP step loop
    # of the oracle: neurons in parallel, atomic integer ring adds; equal to
    # the serial loop bit for bit).
    threads = max(1, min(os.cpu_count() or 1, int(os.environ.get("OMP_NUM_THREADS", "0") or 0)
                         or (os.cpu_count() or 1)))
    sim = O.Sim(net)
    t = time.perf_counter()
    sim.run_threads(n_steps, threads)
    wall_t = time.perf_counter() - t
    ct = sim.counters()
    assert ct == c, "the threaded oracle loop must equal the serial one"
    out["all_cores"] = {"value": ct["events"] / wall_t, "unit": "synaptic events/s", "cores": threads,
                        "kind": "oracle, OpenMP step loop",
                        "sample": f"the same {n_steps} steps, {wall_t:.1f} s on {threads} threads",
                        "rtf": wall_t / (n_steps / STEPS_PER_BIO_SECOND)}
    log(f"[bench] oracle: {wall:.1f} s on one thread, {wall_t:.1f} s on {threads} threads")
    return out


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


def leg_summary(P, leg, bio, workload):
    info = leg["info"]
    return {"value": leg["events"] / leg["wall_s"], "unit": "synaptic events/s",
            "rtf": leg["wall_s"] / bio, "ms_per_step": 1000.0 * leg["wall_s"] / bio,
            "us_per_sim_step_gpu": 1000.0 * leg["gpu_ms"] / leg["n_steps"],
            "spikes_per_step": leg["spikes"] / leg["n_steps"],
            "events_per_step": leg["events"] / leg["n_steps"],
            "syn_format": {"plain": "plain8"}.get(leg["fmt"], leg["fmt"]),
            "record_bytes": leg["rec_bytes"], "build_s": leg["build_s"],
            "device_bytes": info["device_bytes"], "engine": info["engine"],
            "block": info["block_size"], "grid": info["grid_blocks"],
            "window_neurons": info["window_neurons"], "ring_rows": info["ring_rows"],
            "layout_tuning": leg["layout"], "roofline": roofline(P, leg, workload)}


def run_workload(P, workloads, name, args, log, bio_steps=None):
    wl = WORKLOADS[name]
    bio = bio_steps if bio_steps is not None else wl["steps"]
    instances = workloads.WORKLOADS[name]()
    legs = [f for f in wl["legs"] if not (f in ("compressed", "dev8") and args.no_compressed)
            and not (f == "plain" and args.no_plain)] or wl["legs"][:1]
    return bio, instances, [run_leg(P, instances, f, args.engine, args.chunk, args.warmup, bio, log,
                                    args.tune_steps, args.tune_cache) for f in legs]


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="full", choices=sorted(WORKLOADS))
    ap.add_argument("--steps", type=int, default=None,
                    help="timed seconds of biological time (default: 10 full, 2 batch, 5 x4)")
    ap.add_argument("--warmup", type=int, default=1, help="untimed seconds of biological time")
    ap.add_argument("--engine", default="auto", choices=["auto", "stepwise", "persistent", "lds", "band"])
    ap.add_argument("--chunk", type=int, default=10000, help="simulation steps per launch (chunk)")
    ap.add_argument("--no-compressed", action="store_true",
                    help="skip the compressed and dev8 synapse legs")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-synapse legs")
    ap.add_argument("--no-extra", action="store_true",
                    help="with the full workload: skip the batch and x4 workloads")
    ap.add_argument("--tune-steps", type=int, default=2000,
                    help="LDS engines: steps timed per candidate layout when the tuning cache has "
                         "no entry for the workload (0 = no layout tuning)")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_2405_02019_amd", "tune_cache.txt"),
                    help="file of earlier layout choices (read; a miss appends)")
    ap.add_argument("--cpu-steps", type=int, default=10000,
                    help="oracle steps for the CPU baseline, full workload only (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the 1 GiB copy used to scale HBM counters")
    args = ap.parse_args()

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the simulator runs one microcircuit (or one batch) "
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
    from paper_2405_02019_amd import workloads

    bio_steps, instances, results = run_workload(P, workloads, args.workload, args, log, args.steps)
    first = results[0]
    bio = float(bio_steps)
    info = first["info"]
    wl = WORKLOADS[args.workload]
    out = {
        "metric": "realtime factor & synaptic events/s, full PD microcircuit; plain vs compressed",
        "value": first["events"] / first["wall_s"],
        "unit": "synaptic events/s",
        "n_gpus": 1,
        "steps": bio_steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * first["wall_s"] / bio,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 state, int32 fixed-point synaptic input",
        "data": "synthetic: Potjans-Diesmann networks sampled from the paper's tables",
        "config": {"workload": wl["name"].format(syn=info["n_synapses_total"],
                                                 neurons=first["n_neurons"]),
                   "steps_per_bench_step": STEPS_PER_BIO_SECOND,
                   "syn_format": {"plain": "plain8"}.get(first["fmt"], first["fmt"]),
                   "instances": len(instances), "engine": info["engine"],
                   "block": info["block_size"], "grid": info["grid_blocks"],
                   "window_neurons": info["window_neurons"], "ring_rows": info["ring_rows"],
                   "chunk_steps": info["chunk_steps"],
                   "launches_per_chunk": info["launches_per_chunk"], "graphs": info["graphs"],
                   "autotuned": first["tune"] is not None or first["layout"] is not None,
                   "layout_tuning": first["layout"]},
        "rtf": first["wall_s"] / bio,
        "bio_per_wall": bio / first["wall_s"],
        "spikes_per_step": first["spikes"] / first["n_steps"],
        "events_per_step": first["events"] / first["n_steps"],
        "us_per_sim_step_gpu": 1000.0 * first["gpu_ms"] / first["n_steps"],
        "gpu_ms_timed": first["gpu_ms"],
        "build_s": first["build_s"],
        "roofline": roofline(P, first, args.workload),
        "paper_context": {"fpga_rtf_gmem_mono_s": 4.79, "fpga_rtf_best_horiz_multi": 0.79,
                          "hardware": "1 Intel Agilex 7 FPGA (numbers quoted from the paper)"},
    }
    for leg in results[1:]:
        out[leg["fmt"]] = leg_summary(P, leg, bio, args.workload)
    if args.workload == "full" and args.cpu_steps > 0:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps, log)
    if args.workload == "full" and not args.no_extra:
        out["workloads"] = {}
        for name in ["batch", "x4"]:
            wbio, winst, wres = run_workload(P, workloads, name, args, log)
            out["workloads"][name] = {
                "workload": WORKLOADS[name]["name"].format(syn=wres[0]["info"]["n_synapses_total"],
                                                           neurons=wres[0]["n_neurons"]),
                "instances": len(winst), "timed_bio_s": wbio,
                "legs": {leg["fmt"]: leg_summary(P, leg, float(wbio), name) for leg in wres}}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
