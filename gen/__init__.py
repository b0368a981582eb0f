"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds no arithmetic of the localization method itself: it only
draws occupancy maps, robot trajectories with odometry, laser scans and the
expected-range table that a scan model consumes.  Every generator takes an
explicit seed, so a (generator, seed, size) triple names one input exactly.

The paper evaluates on public floor plans with a simulated LIDAR (Sec. IV);
neither is available here, so the generators below stand in for them with
rooms, corridors, doorways and clutter at comparable sizes.
"""

from .maps import bsp_rooms, rooms_and_corridors, occupancy_fraction
from .trajectory import random_odometry, smooth_trajectory
from .raycast import range_table, scan_at, noisy_scan, cell_scans

__all__ = [
    "bsp_rooms",
    "rooms_and_corridors",
    "occupancy_fraction",
    "random_odometry",
    "smooth_trajectory",
    "range_table",
    "scan_at",
    "noisy_scan",
]
