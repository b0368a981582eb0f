"""Oracle of the map-difficulty measure D_M (Sec. IV, localisation robustness).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For every free location p the paper takes the observation z there, finds the
location p_hat whose observation matches z best, and counts the locations with
||p - p_hat|| > C (C = 1 m) among the free ones.  Readings:

  * the observation at p is a range scan at heading 0 (the table row of p,
    plus noise where the caller adds it), quantised as the scan update does;
  * "best matches" is the smallest exact squared distance D of the scan update
    (oracle.scan) over every free cell q and every heading channel k, heading
    offset 0; ties go to the lowest flat index k * (H * W) + q;
  * occupied cells are not candidates.
"""

from __future__ import annotations

import numpy as np

from .scan import beam_offsets, scan_sqdist


def best_match(Rq: np.ndarray, zq: np.ndarray, n_theta: int, free: np.ndarray):
    """(q, k, D) of the best match of one quantised scan.

    Rq: (H * W, N) quantised table in dense cell order; free: (H * W,) bool.
    """
    s = beam_offsets(0.0, n_theta, Rq.shape[1])
    D = scan_sqdist(Rq, zq, s)  # (n_theta, cells)
    big = np.iinfo(np.int64).max
    D = np.where(np.asarray(free, bool)[None, :], D, big)
    flat = int(np.argmin(D.reshape(-1)))  # argmin returns the lowest index among ties
    k, q = divmod(flat, Rq.shape[0])
    return q, k, int(D[k, q])


def difficulty(best_cells: np.ndarray, query_cells: np.ndarray, width: int, cell_m: float,
               threshold_m: float = 1.0) -> float:
    """D_M: the fraction of queried free cells whose best match lies more than threshold_m away."""
    q = np.asarray(query_cells)
    b = np.asarray(best_cells)
    e = cell_m * np.hypot(q % width - b % width, q // width - b // width)
    return float(np.count_nonzero(e > threshold_m)) / max(len(q), 1)
