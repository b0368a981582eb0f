"""Seeded odometry streams.

Odometry is a sequence of robot-frame increments (u, v, w): u forward and v
to the left in metres, w the heading change in radians (counter-clockwise).
"""

from __future__ import annotations

import math

import numpy as np


def random_odometry(n_steps: int, seed: int, *, max_step_m: float = 0.15,
                    sigma_w_deg: float = 5.0) -> np.ndarray:
    """(n, 3) float64: u, v ~ U[0, max_step_m], w ~ N(0, sigma_w_deg)."""
    rng = np.random.default_rng(seed)
    out = np.empty((n_steps, 3), np.float64)
    out[:, 0] = rng.uniform(0.0, max_step_m, n_steps)
    out[:, 1] = rng.uniform(0.0, max_step_m, n_steps)
    out[:, 2] = np.deg2rad(rng.normal(0.0, sigma_w_deg, n_steps))
    return out


def _clearance_cells(occ: np.ndarray) -> np.ndarray:
    from scipy.ndimage import distance_transform_edt
    return distance_transform_edt(occ == 0)


def smooth_trajectory(occ: np.ndarray, cell_m: float, n_steps: int, seed: int, *,
                      fwd_range=(0.04, 0.10), yaw_amp_deg: float = 3.0,
                      yaw_period: float = 200.0, noise_xy_m: float = 0.01,
                      noise_w_deg: float = 1.0, clearance_m: float = 0.25):
    """A ground-truth path that stays in free space, and its noisy odometry.

    The robot drives forward 0.04-0.10 m per step with a yaw rate of
    3 deg * sin(2 pi t / 200) per step.  When the next position would come
    closer than `clearance_m` to an obstacle it turns in place instead.
    Reported odometry = true increment + N(0, noise_xy_m) on u and v and
    N(0, noise_w_deg) on w.

    Returns (poses, odometry): poses (n+1, 3) world x, y, heading; odometry
    (n, 3) robot-frame u, v, w.
    """
    rng = np.random.default_rng(seed)
    clear = _clearance_cells(occ) * cell_m
    h, w = occ.shape
    ok = np.argwhere(clear >= max(2 * clearance_m, 3 * cell_m))
    if len(ok) == 0:
        ok = np.argwhere(occ == 0)
    j, i = ok[int(rng.integers(len(ok)))]
    x, y = (i + 0.5) * cell_m, (j + 0.5) * cell_m
    th = float(rng.uniform(-math.pi, math.pi))
    poses = np.empty((n_steps + 1, 3), np.float64)
    odo = np.empty((n_steps, 3), np.float64)
    poses[0] = (x, y, th)

    def clearance_at(px, py):
        ci, cj = int(math.floor(px / cell_m)), int(math.floor(py / cell_m))
        if not (0 <= ci < w and 0 <= cj < h):
            return 0.0
        return clear[cj, ci]

    for t in range(n_steps):
        fwd = float(rng.uniform(*fwd_range))
        dth = math.radians(yaw_amp_deg) * math.sin(2 * math.pi * t / yaw_period)
        nx = x + fwd * math.cos(th)
        ny = y + fwd * math.sin(th)
        if clearance_at(nx, ny) < clearance_m:
            fwd = 0.0
            dth = math.radians(float(rng.uniform(30.0, 90.0))) * (1 if rng.random() < 0.5 else -1)
            nx, ny = x, y
        x, y, th = nx, ny, th + dth
        poses[t + 1] = (x, y, th)
        odo[t, 0] = fwd + rng.normal(0.0, noise_xy_m)
        odo[t, 1] = rng.normal(0.0, noise_xy_m)
        odo[t, 2] = dth + math.radians(rng.normal(0.0, noise_w_deg))
    return poses, odo
