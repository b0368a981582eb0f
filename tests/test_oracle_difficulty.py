"""Pins of the map-difficulty oracle (best scan match over all free states; D_M), CPU only.

Pinned by a pure-Python brute force of the best match (its own beam loop,
the stated tie order and the free-cell rule), the zero-distance limit of
noise-free scans, the exclusion of occupied cells, and a hand count of D_M.
"""

import itertools

import numpy as np
import pytest

import oracle as O
from gen import bsp_rooms, range_table


def _brute(Rq, zq, n_theta, free):
    n = Rq.shape[1]
    best = None
    for k, q in itertools.product(range(n_theta), range(Rq.shape[0])):  # flat order k * cells + q
        if not free[q]:
            continue
        s = int(np.floor(k * (n / n_theta) + 0.5)) % n  # nearest direction to k * 2 pi / n_theta
        d = sum((int(zq[b]) - int(Rq[q, (b + s) % n])) ** 2 for b in range(n))
        if best is None or d < best[2]:
            best = (q, k, d)
    return best


def _small():
    occ = bsp_rooms(14, 11, seed=101)
    R = range_table(occ, 0.2, 24, 2.5)
    return occ, O.quantize_ranges(R, 2.5)


def test_matches_a_brute_force():
    occ, Rq = _small()
    free = (occ == 0).reshape(-1)
    rng = np.random.default_rng(102)
    for p in rng.choice(np.flatnonzero(free), 6, replace=False):
        zq = np.clip(Rq[p] + rng.integers(-6, 7, Rq.shape[1]), -128, 128)
        assert O.best_match(Rq, zq, 8, free) == _brute(Rq, zq, 8, free)


def test_noise_free_scans_match_exactly():
    occ, Rq = _small()
    free = (occ == 0).reshape(-1)
    for p in np.flatnonzero(free)[::7]:
        q, k, d = O.best_match(Rq, Rq[p], 6, free)
        assert d == 0
        assert k == 0 or not np.array_equal(Rq[q], Rq[p])  # heading 0 first on ties


def test_occupied_cells_are_not_candidates():
    occ, Rq = _small()
    free = (occ == 0).reshape(-1)
    wall = int(np.flatnonzero(~free)[3])
    zq = Rq[wall].copy()  # exactly the expected scan of a wall cell
    q, k, d = O.best_match(Rq, zq, 6, free)
    assert free[q] and d > 0


def test_difficulty_counts_far_matches():
    # width 10, 0.5 m cells: errors 0, 0 and 2 cells (1.0 m)
    assert O.difficulty([0, 5, 30], [0, 5, 10], 10, 0.5) == 0.0
    assert O.difficulty([0, 5, 30], [0, 5, 10], 10, 0.5, threshold_m=0.9) == pytest.approx(1 / 3)
