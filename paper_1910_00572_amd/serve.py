"""Continuous-batching server for many belief-tensor filters on one GPU.

Requests (a map, a heading count, a storage type, an odometry stream and
optional scans) arrive over time.  The server admits a request as soon as its
filter workspace fits the HBM budget and a slot is free; every iteration it
advances *all* active filters by one odometry step with one batched launch per
kernel variant (mcl_step_batch: filters of different grid sizes and heading
counts share a launch), applies the scans that are due, and retires finished
requests, which frees their memory for queued ones.  Work of requests that
arrive while others run therefore overlaps on the device.

Each filter's result is bitwise identical to running it alone: the batched
kernel gives every filter its own workgroups, reduction order and final
reduction.  Latency is measured with HIP events around each iteration on the
launch stream; throughput is total states x steps over the wall-clock span.
"""

from __future__ import annotations

import dataclasses
import time
from collections import deque

import numpy as np

from . import mcl


@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    map_key: object
    n_theta: int
    storage: str
    odometry: np.ndarray                  # (steps, 3) robot-frame u, v, w
    scans: dict = dataclasses.field(default_factory=dict)  # step index -> ranges, applied after that step
    sigma_theta: float = 1.0
    scan_sigma_m: float = 0.1


@dataclasses.dataclass
class Result:
    rid: int
    admitted_s: float
    finished_s: float
    steps: int
    states: int
    belief: np.ndarray | None
    pose: tuple
    log_norm: float
    degenerate: bool = False   # a step removed all probability mass (belief kept, Sec. III-A)


class Server:
    def __init__(self, maps: dict, hbm_budget_bytes: int, max_active: int = 256, keep_beliefs: bool = False,
                 max_inflight: int = 4):
        import torch
        self.torch = torch
        self.maps = maps
        self.budget = int(hbm_budget_bytes)
        self.max_active = int(max_active)
        self.keep_beliefs = keep_beliefs
        self.max_inflight = max_inflight
        self.ws = mcl.BatchWorkspace(self.max_active)
        self.stream = torch.cuda.current_stream()

    def _workspace_bytes(self, req: Request) -> int:
        m = self.maps[req.map_key]
        prm = mcl._params(req.n_theta, m.sigma_xy, req.sigma_theta, m.radius_xy, -1, req.storage, m.flags)
        return int(mcl.load_library().mcl_filter_workspace_bytes(m.handle, mcl.byref(prm)))

    def run(self, requests):
        """Serve `requests` (arrival times relative to the start); returns (results, stats)."""
        torch = self.torch
        pending = deque(sorted(requests, key=lambda r: r.arrival_s))
        active = []       # [request, filter, position, admitted_s, bytes]
        used = 0
        results = {}
        lat_events = []   # (start event, end event, filter-steps in the iteration)
        inflight = deque()
        waits = []
        peak_used = 0
        peak_active = 0
        t0 = time.perf_counter()
        states_steps = 0
        while pending or active:
            now = time.perf_counter() - t0
            # admission: FIFO, by memory budget and slots
            while pending and pending[0].arrival_s <= now and len(active) < self.max_active:
                req = pending[0]
                need = self._workspace_bytes(req)
                if need > self.budget:
                    raise MemoryError(f"request {req.rid} needs {need} bytes, more than the whole budget")
                if used + need > self.budget:
                    break
                pending.popleft()
                f = mcl.Filter(self.maps[req.map_key], req.n_theta, req.sigma_theta, storage=req.storage)
                active.append([req, f, 0, now, need])
                used += need
                peak_used = max(peak_used, used)
                peak_active = max(peak_active, len(active))
                waits.append(now - req.arrival_s)
            if not active:
                if pending:
                    time.sleep(max(0.0, min(pending[0].arrival_s - now, 0.01)))
                continue
            # one iteration: every active filter advances one step
            filters = [a[1] for a in active]
            uvw = np.stack([a[0].odometry[a[2]] for a in active])
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(self.stream)
            mcl.step_batch(filters, uvw, self.ws)
            for a in active:
                z = a[0].scans.get(a[2])
                if z is not None:
                    a[1].apply_scan(z, a[0].scan_sigma_m)
            e1.record(self.stream)
            lat_events.append((e0, e1, len(active)))
            inflight.append(e1)
            if len(inflight) > self.max_inflight:
                inflight.popleft().synchronize()
            still = []
            for a in active:
                a[2] += 1
                req, f = a[0], a[1]
                states_steps += f.map.width * f.map.height * req.n_theta
                if a[2] == len(req.odometry):
                    b, pose, ln, degen = _final_readout(f, self.keep_beliefs)
                    results[req.rid] = Result(req.rid, a[3], time.perf_counter() - t0, a[2],
                                              f.map.width * f.map.height * req.n_theta,
                                              b, pose, ln, degen)
                    used -= a[4]
                    del f
                    a[1] = None
                else:
                    still.append(a)
            active = still
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per_step = []
        for e0, e1, n in lat_events:
            per_step.extend([e0.elapsed_time(e1)] * n)
        per_step = np.array(per_step) if per_step else np.zeros(1)
        stats = {
            "requests": len(results),
            "wall_s": wall,
            "states_steps": states_steps,
            "states_steps_per_s": states_steps / wall if wall > 0 else 0.0,
            "step_latency_ms_p50": float(np.percentile(per_step, 50)),
            "step_latency_ms_p99": float(np.percentile(per_step, 99)),
            "iterations": len(lat_events),
            "admission_wait_s_p50": float(np.percentile(waits, 50)) if waits else 0.0,
            "admission_wait_s_p99": float(np.percentile(waits, 99)) if waits else 0.0,
            "degenerate_requests": sum(1 for r in results.values() if r.degenerate),
            "peak_bytes": peak_used,
            "peak_active": peak_active,
            "budget_bytes": self.budget,
        }
        return results, stats


def _final_readout(f, want_belief):
    """Belief, argmax pose, log-normaliser and the degenerate flag of a filter.

    A filter whose mass was all removed by some step reports EDEGENERATE; its
    readout (the last belief that had mass) is still returned.
    """
    try:
        b, pose, _, ln = f.read_belief(want_belief=want_belief)
        return b, pose.as_tuple(), ln, False
    except mcl.MclError as e:
        if e.status != mcl.EDEGENERATE:
            raise
        b, pose, _, ln = e.readout
        return b, pose.as_tuple(), ln, True


def run_alone(maps, req: Request, keep_belief=True):
    """Reference: the same request on a filter of its own, one call per step.

    Returns (belief, pose, log_norm, degenerate)."""
    f = mcl.Filter(maps[req.map_key], req.n_theta, req.sigma_theta, storage=req.storage)
    for t, (u, v, w) in enumerate(req.odometry):
        f.step_odometry(u, v, w)
        z = req.scans.get(t)
        if z is not None:
            f.apply_scan(z, req.scan_sigma_m)
    return _final_readout(f, keep_belief)
