"""Benchmark of the dense belief-tensor odometry step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extra] [--only a,b]

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


def committed_traffic(kernel_source, summary):
    """HBM bytes per step launch from a committed rocprofv3 counter summary.

    The summary records the sha256 of the step-kernel source it was measured
    on; if the source has changed since, the figure is stale and None is
    returned.
    """
    import hashlib
    import re
    try:
        text = open(summary).read()
        sha = hashlib.sha256(open(kernel_source, "rb").read()).hexdigest()
    except OSError:
        return None
    m_sha = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    m_b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_sha or not m_b or m_sha.group(1) != sha:
        return None
    return float(m_b.group(1))


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


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_worker(args, progress=False):
    """One oracle filter on the headline workload: (states*steps, seconds) of `steps` timed steps."""
    import os as _os
    _os.environ.setdefault("OMP_NUM_THREADS", "1")
    import oracle as O
    from gen import rooms_and_corridors, smooth_trajectory
    size, n_theta, sigma, steps, seed = args
    occ = rooms_and_corridors(size, size, seed=seed)
    _, odo = smooth_trajectory(occ, 0.05, steps, seed=seed + 1)
    p = O.OracleParams(n_theta=n_theta, cell_m=0.05, sigma_xy=sigma, sigma_theta=sigma)
    st = O.init_uniform(occ, n_theta)
    M = O.free_mask(occ)
    t0 = time.perf_counter()
    for t in range(steps):
        st = O.step(st, occ, p, *odo[t], M=M)
        if progress:
            log(f"[bench] oracle {size}x{size}x{n_theta}: step {t + 1}/{steps}, {time.perf_counter() - t0:.1f} s")
    return occ.size * n_theta * steps, time.perf_counter() - t0


def cpu_baseline(occ, odo, n_theta, sigma, steps=8, pool_steps=3):
    """The FP64 oracle on the host: one core (one filter, `steps` steps of the
    512x512x72 workload) and all of the machine's cores (independent filters of
    the same workload on a process pool, one per core, `pool_steps` steps each)."""
    import multiprocessing as mp
    import oracle as O
    p = O.OracleParams(n_theta=n_theta, cell_m=0.05, sigma_xy=sigma, sigma_theta=sigma)
    st = O.init_uniform(occ, n_theta)
    M = O.free_mask(occ)
    t0 = time.perf_counter()
    for t in range(steps):
        st = O.step(st, occ, p, *odo[t], M=M)
    dt = time.perf_counter() - t0
    states = occ.size * n_theta
    one = states * steps / dt
    # the GPU machine grants 16 host cores per GPU, whatever the host shows
    workers = max(1, min(16, os.cpu_count() or 1))
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_worker, [(512, n_theta, sigma, pool_steps, 3)] * workers)
    wall = time.perf_counter() - t0
    work = sum(r[0] for r in res)
    compute = max(r[1] for r in res)
    return {"value": work / compute, "unit": "states*steps/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} independent FP64 oracle filters (numpy) of the 512x512x72 workload on a "
                      f"process pool, {pool_steps} steps each ({compute:.1f} s of compute, {wall:.1f} s with "
                      f"start-up); one core: {steps} steps of one filter",
            "one_core_value": one, "one_core_seconds": dt, "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


def cpu_baseline_large(steps=5):
    """The FP64 oracle on the 1024x1024x128 workload (one filter, one core), `steps` steps."""
    n, dt = _oracle_worker((1024, 128, 1.0, steps, 5), progress=True)
    return {"value": n / dt, "unit": "states*steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of the 1024x1024x128 FP64 oracle (numpy, one core), {dt:.1f} s",
            "cpu_model": _cpu_model()}


def bench_mixed_precision(steps):
    """1024x1024 map, 128 bins: FP32 vs BF16 storage on the same trajectory."""
    import torch
    from gen import rooms_and_corridors, smooth_trajectory
    from paper_1910_00572_amd import mcl
    occ = rooms_and_corridors(1024, 1024, seed=5)
    _, odo = smooth_trajectory(occ, 0.05, steps + 10, seed=6)
    m = mcl.Map(occ, 0.05, 1.0)
    states = occ.size * 128
    out = {}
    beliefs = {}
    for storage, eb in (("f32", 4), ("bf16", 2)):
        f = mcl.Filter(m, 128, 1.0, storage=storage)
        elapsed, lat = time_filter(f, odo, steps, 5, 20)
        b, pose, _, _ = f.read_belief()
        beliefs[storage] = (b, pose.as_tuple())
        kern = float(lat.mean())
        out[storage] = {"states_steps_per_s": states * steps / elapsed, "ms_per_step": elapsed * 1e3 / steps,
                        "event_mean_ms": kern,
                        "roofline_frac": 2 * states * eb / (kern * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del f
        torch.cuda.empty_cache()
    bf, f32 = beliefs["bf16"][0].astype(np.float64), beliefs["f32"][0].astype(np.float64)
    k, j, i = beliefs["bf16"][1]
    out["bf16_vs_f32_after_steps"] = {"steps": steps + 5 + 20, "l1": float(np.abs(bf - f32).sum()),
                                     "peak_normalised_max_abs": float(np.abs(bf - f32).max() / f32.max()),
                                     "argmax_in_f32_tie_set_2^-7": bool(f32[k, j, i] >= f32.max() * (1 - 2 ** -7))}
    out["speedup_bf16_over_f32"] = out["bf16"]["states_steps_per_s"] / out["f32"]["states_steps_per_s"]
    out["bf16_vs_oracle_128x128x128"] = bf16_vs_oracle()
    return out


def bf16_vs_oracle(steps=40):
    """BF16 storage against the FP64 oracle on a 128x128 plan with 128 bins (a size the oracle runs
    in seconds), at the launch shape of the 1024x1024x128 workload: L1 and argmax agreement."""
    import oracle as O
    from gen import rooms_and_corridors, smooth_trajectory
    from paper_1910_00572_amd import mcl
    occ = rooms_and_corridors(128, 128, seed=49)
    _, odo = smooth_trajectory(occ, 0.05, steps, seed=50)
    m = mcl.Map(occ, 0.05, 1.0)
    f = mcl.Filter(m, 128, 1.0, storage="bf16", launch_shape=(0, 16, 512, 1, 1, 0, 4))
    p = O.OracleParams(n_theta=128, cell_m=0.05, sigma_xy=1.0, sigma_theta=1.0)
    st = O.init_uniform(occ, 128)
    M = O.free_mask(occ)
    worst, agree = 0.0, 0
    for t, (u, v, w) in enumerate(odo):
        f.step_odometry(u, v, w)
        st = O.step(st, occ, p, u, v, w, M=M)
        if t % 10 == 9:
            b, pose, _, _ = f.read_belief()
            worst = max(worst, float(np.abs(b.astype(np.float64) - st.B).sum()))
            k, j, i = pose.as_tuple()
            agree += int(st.B[k, j, i] >= st.B.max() * (1 - 2 ** -7))
    return {"steps": steps, "checks": steps // 10, "l1_worst": worst, "argmax_in_tie_set_2^-7": agree,
            "bound": "L1 <= 1e-2, argmax in the oracle's tie set"}


def bench_scan(n_scans):
    """512x512 map, 72 bins, 360 beams: dense scan update, BF16 and FP32 matrix operands."""
    import torch
    from gen import noisy_scan, range_table, rooms_and_corridors, smooth_trajectory
    from paper_1910_00572_amd import mcl
    occ = rooms_and_corridors(512, 512, seed=3)
    poses, odo = smooth_trajectory(occ, 0.05, 100, seed=4)
    R = range_table(occ, 0.05, 360, 10.0)
    out = {}
    for name, flags in (("bf16_mfma", mcl.DEFAULT_FLAGS), ("f32_mfma", mcl.DEFAULT_FLAGS | mcl.SCAN_F32)):
        m = mcl.Map(occ, 0.05, 1.0, range_table=R, max_range_m=10.0, flags=flags)
        f = mcl.Filter(m, 72, 1.0, storage="f32")
        zs = [noisy_scan(occ, 0.05, poses[(10 * t) % 100], 360, 10.0, 0.1, seed=7 + t) for t in range(n_scans)]
        for t in range(10):
            f.step_odometry(*odo[t])
        f.apply_scan(zs[0], 0.1)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in zs]
        for t, z in enumerate(zs):
            ev[t][0].record(stream)
            f.apply_scan(z, 0.1)
            ev[t][1].record(stream)
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        useful = 2.0 * 512 * 512 * 360 * 72
        issued = 2.0 * 512 * 512 * 384 * 96
        peak = 2500e12 if name == "bf16_mfma" else 157.3e12
        # scan every 10 steps over 100 steps
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(100):
            f.step_odometry(*odo[t])
            if t % 10 == 9:
                f.apply_scan(zs[(t // 10) % len(zs)], 0.1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"scan_ms": ms, "useful_gflop": useful / 1e9, "issued_gflop": issued / 1e9,
                     "achieved_tflops_useful": useful / (ms * 1e-3) / 1e12,
                     "mfma_frac_of_peak_issued": issued / (ms * 1e-3) / peak,
                     "table_bytes_algorithmic": 512 * 512 * 360 * (2 if name == "bf16_mfma" else 4),
                     "hbm_frac_table_plus_belief_rw": (512 * 512 * 360 * (2 if name == "bf16_mfma" else 4)
                                                       + 2 * 512 * 512 * 72 * 4) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "steps_with_scan_every_10_states_steps_per_s": 512 * 512 * 72 * 100 / dt}
        del f, m
        torch.cuda.empty_cache()
    return out


def bench_sampled(n_scans, n_samples=4096):
    """512x512 map, 72 bins, 360 beams: Floyd-Steinberg sample selection and the sampled update."""
    import torch
    from gen import noisy_scan, range_table, rooms_and_corridors, smooth_trajectory
    from paper_1910_00572_amd import mcl
    occ = rooms_and_corridors(512, 512, seed=3)
    poses, odo = smooth_trajectory(occ, 0.05, 200, seed=4)
    R = range_table(occ, 0.05, 360, 10.0)
    m = mcl.Map(occ, 0.05, 1.0, range_table=R, max_range_m=10.0)
    f = mcl.Filter(m, 72, 1.0, storage="f32")
    zs = [noisy_scan(occ, 0.05, poses[(10 * t) % 200], 360, 10.0, 0.1, seed=7 + t) for t in range(n_scans)]
    mask = torch.empty((512, 512), dtype=torch.uint8, device="cuda")
    # a multimodal belief: motion from the uniform start, then a few sampled scans
    for t in range(30):
        f.step_odometry(*odo[t])
        if t % 10 == 9:
            f.sample_cells(n_samples, out=mask)
            f.apply_scan_sampled(zs[t // 10], 0.1, mask)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in zs]
    counts = []
    for t, z in enumerate(zs):
        ev[t][0].record(stream)
        f.sample_cells(n_samples, out=mask)
        ev[t][1].record(stream)
        f.apply_scan_sampled(z, 0.1, mask)
        ev[t][2].record(stream)
        if t == len(zs) - 1:
            counts.append(int(mask.sum().item()))
    torch.cuda.synchronize()
    sel_ms = float(np.mean([a.elapsed_time(b) for a, b, _ in ev]))
    upd_ms = float(np.mean([b.elapsed_time(c) for _, b, c in ev]))
    # one-wave dithering of a 512 x 512 map: eight cells per phase, cell (i, j) at step i + 9 j
    phases = (511 + 9 * 511) // 8 + 1
    # steps with a sampled scan every 10 steps, 100 steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(100):
        f.step_odometry(*odo[30 + t])
        if t % 10 == 9:
            f.sample_cells(n_samples, out=mask)
            f.apply_scan_sampled(zs[(t // 10) % len(zs)], 0.1, mask)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    states = 512 * 512 * 72
    out = {"n_samples_requested": n_samples, "cells_selected": counts[0],
           "select_ms": sel_ms, "update_ms": upd_ms,
           "select_plus_update_ms": sel_ms + upd_ms,
           "dither_phases": phases, "dither_kernel": "one wave, eight cells per phase",
           "belief_read_bytes_select": states * 4, "belief_read_bytes_update": states * 4,
           "steps_with_sampled_scan_every_10_states_steps_per_s": states * 100 / dt}
    del f, m
    torch.cuda.empty_cache()
    return out


def bench_integer_gate(n_steps=200, split=4):
    """512x512x72 FP32: bilinear warp on every step against the whole-cell warp with carry, with and
    without the sub-cell gate, on the headline trajectory at a `split`-times higher odometry rate."""
    import torch
    from gen import rooms_and_corridors, smooth_trajectory
    from paper_1910_00572_amd import mcl
    occ = rooms_and_corridors(512, 512, seed=3)
    _, odo = smooth_trajectory(occ, 0.05, n_steps, seed=4)
    sub = np.repeat(np.asarray(odo[:n_steps], dtype=np.float64) / split, split, axis=0)
    variants = {"bilinear_every_step": mcl.DEFAULT_FLAGS,
                "whole_cell_carry": mcl.DEFAULT_FLAGS | mcl.INTEGER_SHIFT,
                "gate_whole_cell_carry": mcl.DEFAULT_FLAGS | mcl.INTEGER_SHIFT | mcl.SUBCELL_GATE}
    out, beliefs = {}, {}
    states = occ.size * 72
    for name, flags in variants.items():
        m = mcl.Map(occ, 0.05, 1.0, flags=flags)
        f = mcl.Filter(m, 72, 1.0, storage="f32")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for u, v, w in sub:
            f.step_odometry(u, v, w)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        b, pose, _, _ = f.read_belief()
        beliefs[name] = (b.astype(np.float64), pose)
        out[name] = {"odometry_steps": len(sub), "states_odometry_steps_per_s": states * len(sub) / dt,
                     "ms_per_odometry_step": dt * 1e3 / len(sub)}
        del f, m
        torch.cuda.empty_cache()
    ref, rpose = beliefs["bilinear_every_step"]
    for name in ("whole_cell_carry", "gate_whole_cell_carry"):
        b, pose = beliefs[name]
        out[name]["l1_vs_bilinear"] = float(np.abs(b - ref).sum())
        out[name]["argmax_distance_m_vs_bilinear"] = 0.05 * float(np.hypot(pose.i - rpose.i, pose.j - rpose.j))
    return out


def bench_aniso(steps=100):
    """512x512x72 FP32 with anisotropic heading-rotated noise (sigma 1.0 along, 0.5 across, radius 3)."""
    import torch
    from paper_1910_00572_amd import mcl
    occ, odo = headline_inputs(steps + 10)
    m = mcl.Map(occ, 0.05, 1.0, flags=mcl.DEFAULT_FLAGS | mcl.ANISOTROPIC)
    f = mcl.Filter(m, 72, 1.0, storage="f32", sigma_lateral=0.5)
    elapsed, lat = time_filter(f, odo, steps, 5, 20)
    states = occ.size * 72
    kern = float(lat.mean())
    # two passes: read B, write the FP32 scratch; read it, write B
    algo = 4 * states * 4
    # per state: bilinear warp of 7 theta taps (7 x 4 FMA) + 49-tap blurs of the scratch and the mask
    flops = 2 * states * (7 * 4 + 2 * 49)
    out = {"states_steps_per_s": states * steps / elapsed, "ms_per_step": elapsed * 1e3 / steps,
           "event_mean_ms": kern, "hbm_frac_two_pass_bytes": algo / (kern * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "fp32_frac_of_vector_peak": flops / (kern * 1e-3) / 78.6e12}
    del f, m
    torch.cuda.empty_cache()
    return out


def bench_match(grid=256, n_theta=72, batch=256):
    """Map difficulty D_M on a grid x grid floor plan: the best match of a noisy
    scan (360 beams, sigma 0.1 m) taken at every free cell, over every free state."""
    import time
    import torch
    from gen import cell_scans, range_table, rooms_and_corridors
    from paper_1910_00572_amd import mcl
    occ = rooms_and_corridors(grid, grid, seed=5)
    R = range_table(occ, 0.05, 360, 10.0)
    m = mcl.Map(occ, 0.05, 1.0, range_table=R, max_range_m=10.0)
    qcells = np.flatnonzero(occ.reshape(-1) == 0)
    z = cell_scans(R, qcells, 0.1, 10.0, seed=6)
    mcl.best_match(m, n_theta, z[:batch], batch=batch)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cell, head, dist = mcl.best_match(m, n_theta, z, batch=batch)
    elapsed = time.perf_counter() - t0
    dm = mcl.difficulty(m, qcells, cell, 1.0)
    pitch = (grid + 7) // 8 * 8  # row pitch: a multiple of 8 cells
    cells_pad = (grid * pitch + 127) // 128 * 128
    cols = sum(((min(batch, len(z) - q0) * n_theta + 31) // 32 * 32) for q0 in range(0, len(z), batch))
    flops = 2.0 * cells_pad * 384 * cols
    out = {"queries": int(len(z)), "seconds": elapsed, "queries_per_s": len(z) / elapsed,
           "candidate_states": int(len(qcells) * n_theta), "D_M": dm,
           "gemm_tflops_wall": flops / elapsed / 1e12,
           "bf16_frac_of_mfma_peak_wall": flops / elapsed / 1e12 / 2500.0}
    del m
    torch.cuda.empty_cache()
    return out


def _serving_requests(n_requests, seed, occs, storages):
    """Seeded requests: grid 128..1024, 36/72 bins, storage drawn from `storages`, 50-500 steps of a
    smooth trajectory, a 360-beam scan from the true pose every 10 steps on half of them."""
    from gen import noisy_scan, smooth_trajectory
    from paper_1910_00572_amd.serve import Request
    rng = np.random.default_rng(seed)
    grids = sorted(occs)
    reqs = []
    total = 0.0
    for rid in range(n_requests):
        g = int(rng.choice(grids))
        n_theta = int(rng.choice([36, 72]))
        storage = str(rng.choice(storages))
        steps = int(rng.integers(50, 501))
        poses, odo = smooth_trajectory(occs[g], 0.05, steps, seed=1000 + rid)
        scans = {}
        if rid % 2 == 0:
            for t in range(9, steps, 10):
                scans[t] = noisy_scan(occs[g], 0.05, poses[t + 1], 360, 10.0, 0.1, seed=rid * 1000 + t)
        total += g * g * n_theta * steps
        reqs.append(Request(rid, 0.0, g, n_theta, storage, odo, scans))
    return reqs, total, rng


def bench_serving(n_requests, seed=8, capacity=None, plain_f32_rate=None):
    """Continuous batching of many filters (grid 128..1024, 36/72 bins, scans on half).

    poisson: a Poisson stream of FP32/BF16 requests offered at 0.7 x the plain
    single-filter rate; burst_bf16: the same requests, all stored in BF16,
    arriving at once (the GPU's aggregate capacity for the served
    mixed-precision form), against the plain FP32 single-filter rate.
    """
    import torch
    from gen import range_table, rooms_and_corridors
    from paper_1910_00572_amd import mcl
    from paper_1910_00572_amd.serve import Server
    grids = (128, 256, 512, 1024)
    maps, occs = {}, {}
    for g in grids:
        occ = rooms_and_corridors(g, g, seed=100 + g)
        occs[g] = occ
        maps[g] = mcl.Map(occ, 0.05, 1.0, range_table=range_table(occ, 0.05, 360, 10.0), max_range_m=10.0)
    out = {}
    # Poisson arrivals, mixed storage
    reqs, total, rng = _serving_requests(n_requests, seed, occs, ["f32", "bf16"])
    cap = capacity or 5e11
    span = total / (0.7 * cap)
    arr = np.cumsum(rng.exponential(span / n_requests, n_requests))
    for r, a in zip(reqs, arr):
        r.arrival_s = float(a)
    server = Server(maps, 16 << 30, max_active=256)
    _, stats = server.run(reqs)
    stats["offered_states_steps_per_s"] = total / span
    stats["hbm_budget_gib"] = 16
    out["poisson"] = stats
    del server
    # burst at t = 0, every request stored in BF16
    reqs, total, _ = _serving_requests(n_requests, seed, occs, ["bf16"])
    server = Server(maps, 16 << 30, max_active=256)
    _, stats = server.run(reqs)
    stats["hbm_budget_gib"] = 16
    if plain_f32_rate:
        stats["plain_f32_single_filter_states_steps_per_s"] = plain_f32_rate
        stats["served_bf16_over_plain_f32"] = stats["states_steps_per_s"] / plain_f32_rate
    stats["accuracy"] = ("each served result is bitwise the filter run alone (tests/test_gpu_serve.py); BF16 "
                         "storage alone stays within L1 <= 1e-2 of the FP64 oracle with the argmax in its tie "
                         "set (mixed_precision...bf16_vs_oracle, tests/test_gpu_precision.py)")
    out["burst_bf16"] = stats
    del server, maps
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--latency-steps", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=8)
    ap.add_argument("--cpu-large-steps", type=int, default=0,
                    help="also time this many oracle steps of the 1024x1024x128 workload (about 25 s each)")
    ap.add_argument("--no-extra", action="store_true", help="headline workload only")
    ap.add_argument("--calibration-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--serving-requests", type=int, default=256)
    ap.add_argument("--only", default="", help="comma-separated extra sections to run "
                    "(mixed, scan, sampled, gate, aniso, difficulty, serving); default all")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the filter step is a single-GPU kernel and there is "
              "no multi-GPU path (sharding is a design only).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1910_00572_amd import mcl

    torch.cuda.set_device(0)
    if args.calibration_copy_mib > 0:
        # a plain copy kernel of known size: FETCH_SIZE / WRITE_SIZE of this
        # dispatch calibrate the same counters on the step kernel
        n = args.calibration_copy_mib << 18
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
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
        "paper_context": {"value": 1.0e10, "unit": "states*steps/s", "hardware": "Intel i7 + NVIDIA Titan V",
                          "workload": "belief 500x500x128, odometry and map step without samples, about 3.2 ms",
                          "source": "the paper's timing paragraph (Sec. IV); 32 M states / 3.2 ms, derived",
                          "note": "another machine and another map: context only, not the target"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": committed_traffic(os.path.join(ROOT, "paper_1910_00572_amd", "csrc", "step.hip"),
                                                  os.path.join(ROOT, "profiles", "step_f32_512x512x72_counters.md"))},
    }
    del f, m
    torch.cuda.empty_cache()
    if not args.no_extra:
        only = set(x for x in args.only.split(",") if x) or {"mixed", "scan", "sampled", "gate", "aniso",
                                                                   "difficulty", "serving"}
        if "mixed" in only:
            log("[bench] 1024x1024x128 FP32 vs BF16")
            out["mixed_precision_1024x1024x128"] = bench_mixed_precision(100)
        if "scan" in only:
            log("[bench] scan update 512x512x72, 360 beams")
            out["scan_512x512x72_360beams"] = bench_scan(20)
        if "sampled" in only:
            log("[bench] sampled update 512x512x72, 360 beams, 4096 samples")
            out["sampled_scan_512x512x72_360beams"] = bench_sampled(20)
        if "aniso" in only:
            log("[bench] anisotropic noise 512x512x72")
            out["anisotropic_512x512x72"] = bench_aniso()
        if "gate" in only:
            log("[bench] whole-cell warp and sub-cell gate against bilinear, 512x512x72")
            out["whole_cell_warp_512x512x72"] = bench_integer_gate()
        if "difficulty" in only:
            log("[bench] map difficulty 256x256, 72 headings, every free cell queried")
            out["map_difficulty_256x256x72_360beams"] = bench_match()
        if "serving" in only and args.serving_requests > 0:
            log(f"[bench] serving {args.serving_requests} requests")
            out["serving"] = bench_serving(args.serving_requests, capacity=value, plain_f32_rate=value)
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(occ, odo, n_theta, sigma, args.cpu_steps)
    if args.cpu_large_steps > 0:
        log(f"[bench] timing the FP64 oracle on 1024x1024x128, {args.cpu_large_steps} steps")
        out["cpu_baseline_1024x1024x128"] = cpu_baseline_large(args.cpu_large_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
