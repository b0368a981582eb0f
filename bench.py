"""Benchmark of the dense belief-tensor odometry step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--only NAME]

Headline workload: a 512x512 synthetic floor plan (0.05 m cells, rooms,
corridors and clutter, ~35 % occupied) with 72 heading bins (18.9 M states),
FP32 storage, motion noise sigma = 1 cell / 1 bin, driven by a seeded smooth
trajectory with odometry noise.  Inputs are resident in HBM before timing.
One step is one fused odometry update (warp, mask, 3-D blur, wall
normalisation, renormalising reduction) of the whole tensor.

Prints ONE JSON line: throughput in states*steps/s, per-step latency
percentiles (HIP events on the launch stream), the roofline of the step
kernel, and the FP64 oracle timed on a bounded sample on the host.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "belief states·steps/s + p50/p99 step latency; % HBM/MFMA roofline"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def headline_inputs(n_steps):
    from gen import rooms_and_corridors, smooth_trajectory
    occ = rooms_and_corridors(512, 512, seed=3)
    _, odo = smooth_trajectory(occ, 0.05, max(n_steps, 1000), seed=4)
    return occ, odo


def time_filter(f, odo, steps, warmup, latency_steps):
    """Returns (seconds for `steps` steps, per-step event latencies in ms)."""
    import torch
    n = len(odo)
    for t in range(warmup):
        f.step_odometry(*odo[t % n])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(steps):
        f.step_odometry(*odo[(warmup + t) % n])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # latency pass: an event pair around every step on the launch stream
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(latency_steps)]
    for t in range(latency_steps):
        ev[t][0].record(stream)
        f.step_odometry(*odo[(warmup + steps + t) % n])
        ev[t][1].record(stream)
    torch.cuda.synchronize()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    return elapsed, lat


def cpu_baseline(occ, odo, n_theta, sigma, steps=8):
    import oracle as O
    p = O.OracleParams(n_theta=n_theta, cell_m=0.05, sigma_xy=sigma, sigma_theta=sigma)
    st = O.init_uniform(occ, n_theta)
    M = O.free_mask(occ)
    t0 = time.perf_counter()
    for t in range(steps):
        st = O.step(st, occ, p, *odo[t], M=M)
    dt = time.perf_counter() - t0
    states = occ.size * n_theta
    return {"value": states * steps / dt, "unit": "states*steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} odometry steps of the 512x512x72 FP64 oracle (numpy, single thread), "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--latency-steps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--only", default="")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the filter step is a single-GPU kernel and this build "
              "has no multi-GPU path (see DESIGN.md, sharding).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1910_00572_amd import mcl

    torch.cuda.set_device(0)
    occ, odo = headline_inputs(args.steps + args.warmup + args.latency_steps)
    n_theta, sigma = 72, 1.0
    log("[bench] building map and filter 512x512x72 f32")
    m = mcl.Map(occ, 0.05, sigma)
    f = mcl.Filter(m, n_theta, sigma, storage="f32")
    info = f.info()
    states = occ.size * n_theta
    log(f"[bench] shape tile={info.tile_x}x{info.tile_y} chunks={info.theta_chunks} wg={info.workgroups}")
    elapsed, lat = time_filter(f, odo, args.steps, args.warmup, args.latency_steps)
    ms_per_step = elapsed * 1e3 / args.steps
    value = states * args.steps / elapsed
    kern_ms = float(lat.mean())
    algo_bytes = 2 * states * 4  # one read and one write of the FP32 belief
    achieved = algo_bytes / (kern_ms * 1e-3) / 1e9
    log(f"[bench] {ms_per_step*1e3:.1f} us/step, {value:.3e} states*steps/s, event mean {kern_ms*1e3:.1f} us")
    b, pose, _, _ = f.read_belief(want_belief=False)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "states*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512x512 floor plan (0.05 m, ~35% occupied), 72 theta bins, FP32 storage, "
                               "sigma 1 cell / 1 bin, smooth trajectory; fused odometry step",
                   "states": states, "tile": [info.tile_x, info.tile_y], "theta_chunks": info.theta_chunks,
                   "workgroups": info.workgroups},
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "mean": kern_ms, "samples": int(len(lat))},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(occ, odo, n_theta, sigma, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
