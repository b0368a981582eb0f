"""Continuous-batching server for many belief-tensor filters on one GPU.

Requests (a map, a heading count, a storage type, an odometry stream and
optional scans) arrive over time.  The server admits a request as soon as its
filter workspace fits the HBM budget and a slot is free; every iteration it
advances *all* active filters by one odometry step through a graph-replayed
batch (mcl_batch_step: the step parameters go into a pinned slot, a HIP
graph per launch structure copies them to the device and runs one launch per
kernel group, filters of any grid size and heading count sharing a launch),
applies the due scans of the filters of each map in shared launches
(mcl_apply_scan_batch), and retires finished requests, whose readout is
exported asynchronously and whose memory goes to queued requests.  Work of
requests that arrive while others run therefore overlaps on the device, and
the host never waits for the stream except to bound the iterations in
flight.

Each filter's result is bitwise identical to running it alone: the batched
kernels give every filter its own workgroups, reduction order and final
reduction.  Latency is per request step, from the host time its iteration
was enqueued to the completion of that iteration on the device (HIP events,
placed on the host clock by a reference event); throughput is total
states x steps over the wall-clock span.
"""

from __future__ import annotations

import dataclasses
import time
from collections import defaultdict, deque

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
    pose: tuple | None
    log_norm: float
    degenerate: bool = False   # a step removed all probability mass (belief kept, Sec. III-A)


class _Draining:
    """A retired filter's asynchronous readout (belief and scalars to pinned host memory)."""

    def __init__(self, torch, f, want_belief):
        self.belief = None
        dev_scalars = f.export_scalars()
        self.scalars = torch.empty(2, dtype=torch.float64, pin_memory=True)
        self.scalars.copy_(dev_scalars, non_blocking=True)
        if want_belief:
            dev_b = f.export_belief()
            self.belief = torch.empty(dev_b.shape, dtype=torch.float32, pin_memory=True)
            self.belief.copy_(dev_b, non_blocking=True)
        self.event = torch.cuda.Event()
        self.event.record()


class Server:
    def __init__(self, maps: dict, hbm_budget_bytes: int, max_active: int = 256, keep_beliefs: bool = False,
                 max_inflight: int = 3):
        import torch
        self.torch = torch
        self.maps = maps
        self.budget = int(hbm_budget_bytes)
        self.max_active = int(max_active)
        self.keep_beliefs = keep_beliefs
        self.max_inflight = max_inflight
        # a stream of its own: graphs cannot be captured on the default stream
        self.stream = torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            self.runner = mcl.BatchRunner(self.max_active)

    def _workspace_bytes(self, req: Request) -> int:
        m = self.maps[req.map_key]
        prm = mcl._params(req.n_theta, m.sigma_xy, req.sigma_theta, m.radius_xy, -1, req.storage, m.flags)
        return int(mcl.load_library().mcl_filter_workspace_bytes(m.handle, mcl.byref(prm)))

    def run(self, requests):
        """Serve `requests` (arrival times relative to the start); returns (results, stats)."""
        with self.torch.cuda.stream(self.stream):
            return self._run(requests)

    def _run(self, requests):
        torch = self.torch
        pending = deque(sorted(requests, key=lambda r: r.arrival_s))
        active = []       # [request, filter, position, admitted_s, bytes]
        used = 0
        results = {}
        draining = []     # (request, _Draining, admitted_s, steps, states)
        iters = []        # (host enqueue time, completion event, filter-steps in the iteration)
        inflight = deque()
        waits = []
        peak_used = 0
        peak_active = 0
        states_steps = 0
        ref = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ref.record(self.stream)

        def finish_drained(block):
            still = []
            for req, d, adm, steps, states in draining:
                if block:
                    d.event.synchronize()
                if not d.event.query():
                    still.append((req, d, adm, steps, states))
                    continue
                b = d.belief.numpy().copy() if d.belief is not None else None
                pose = None
                if b is not None:
                    k, j, i = np.unravel_index(int(np.argmax(b)), b.shape)  # lowest flat index wins ties
                    pose = (int(k), int(j), int(i))
                ln, status = float(d.scalars[0]), int(d.scalars[1])
                results[req.rid] = Result(req.rid, adm, time.perf_counter() - t0, steps, states, b, pose, ln,
                                          status == mcl.EDEGENERATE)
            draining[:] = still

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
                finish_drained(False)
                if pending:
                    time.sleep(max(0.0, min(pending[0].arrival_s - now, 0.01)))
                continue
            # one iteration: every active filter advances one step
            t_enq = time.perf_counter() - t0
            filters = [a[1] for a in active]
            uvw = np.stack([a[0].odometry[a[2]] for a in active])
            self.runner.step(filters, uvw)
            due = defaultdict(list)
            for a in active:
                z = a[0].scans.get(a[2])
                if z is not None:
                    due[(a[0].map_key, a[0].scan_sigma_m)].append((a[1], z))
            for (_, sig), fz in due.items():
                mcl.apply_scan_batch([f for f, _ in fz], np.stack([z for _, z in fz]), sig)
            done = torch.cuda.Event(enable_timing=True)
            done.record(self.stream)
            iters.append((t_enq, done, len(active)))
            inflight.append(done)
            if len(inflight) > self.max_inflight:
                inflight.popleft().synchronize()
            still = []
            for a in active:
                a[2] += 1
                req, f = a[0], a[1]
                states = f.map.width * f.map.height * req.n_theta
                states_steps += states
                if a[2] == len(req.odometry):
                    draining.append((req, _Draining(torch, f, self.keep_beliefs), a[3], a[2], states))
                    used -= a[4]
                    a[1] = None
                    del f
                else:
                    still.append(a)
            active = still
            finish_drained(False)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        finish_drained(True)
        lat = []
        for t_enq, ev, n in iters:
            done_s = ref.elapsed_time(ev) * 1e-3
            lat.extend([max(0.0, done_s - t_enq) * 1e3] * n)
        lat = np.array(lat) if lat else np.zeros(1)
        captures, replays = self.runner.counts()
        stats = {
            "requests": len(results),
            "wall_s": wall,
            "states_steps": states_steps,
            "states_steps_per_s": states_steps / wall if wall > 0 else 0.0,
            "step_latency_ms_p50": float(np.percentile(lat, 50)),
            "step_latency_ms_p99": float(np.percentile(lat, 99)),
            "latency": "per request step: host enqueue of its iteration to the iteration's completion on the GPU",
            "iterations": len(iters),
            "graph_captures": captures,
            "graph_replays": replays,
            "admission_wait_s_p50": float(np.percentile(waits, 50)) if waits else 0.0,
            "admission_wait_s_p99": float(np.percentile(waits, 99)) if waits else 0.0,
            "degenerate_requests": sum(1 for r in results.values() if r.degenerate),
            "peak_bytes": peak_used,
            "peak_active": peak_active,
            "budget_bytes": self.budget,
        }
        return results, stats


def run_alone(maps, req: Request, keep_belief=True):
    """Reference: the same request on a filter of its own, one call per step.

    Returns (belief, pose, log_norm, degenerate)."""
    f = mcl.Filter(maps[req.map_key], req.n_theta, req.sigma_theta, storage=req.storage)
    for t, (u, v, w) in enumerate(req.odometry):
        f.step_odometry(u, v, w)
        z = req.scans.get(t)
        if z is not None:
            f.apply_scan(z, req.scan_sigma_m)
    try:
        b, pose, _, ln = f.read_belief(want_belief=keep_belief)
        return b, pose.as_tuple(), ln, False
    except mcl.MclError as e:
        if e.status != mcl.EDEGENERATE:
            raise
        b, pose, _, ln = e.readout
        return b, pose.as_tuple(), ln, True
