"""Pins of the integer-shift option of the oracle (whole-cell warp with a carried remainder), CPU only.

The warp of Alg. 1 read as a whole-cell translation: a channel moves by its
displacement plus the remainder it carries, rounded half up, and keeps the
new remainder.  Pinned by hand-derived positions of an impulse, the remainder
bound against the summed displacement, equality with the bilinear warp when
every move is a whole cell, and the sub-cell gate firing on schedule.
"""

import math

import numpy as np

import oracle as O


def _impulse(H, W, n_theta, j, i):
    B = np.zeros((n_theta, H, W))
    B[:, j, i] = 1.0 / n_theta
    return O.FilterState(B=B)


def _params(n_theta, gate=False, sigma=0.0):
    return O.OracleParams(n_theta=n_theta, cell_m=1.0, sigma_xy=sigma, sigma_theta=sigma, radius_xy=0 if sigma == 0 else -1,
                          radius_theta=0 if sigma == 0 else -1, wall_normalize=False, subcell_gate=gate,
                          integer_shift=True)


def _where(B, k):
    j, i = np.unravel_index(int(np.argmax(B[k])), B[k].shape)
    assert B[k, j, i] > 0 and np.count_nonzero(B[k]) == 1
    return int(j), int(i)


def test_hand_derived_positions():
    # five moves of 0.35 cells forward: carried displacement 0.35, 0.70 -> 1 (rem -0.30),
    # 0.05, 0.40, 0.75 -> 1: positions +0, +1, +1, +1, +2 along the channel's heading
    # (every carried value is at least 0.05 from a rounding tie, in both directions)
    occ = np.zeros((9, 9), np.uint8)
    p = _params(4)
    st = _impulse(9, 9, 4, 4, 4)
    expect = [0, 1, 1, 1, 2]
    for t in range(5):
        st = O.step(st, occ, p, 0.35, 0.0, 0.0)
        assert _where(st.B, 0) == (4, 4 + expect[t])  # heading 0: +x
        assert _where(st.B, 1) == (4 + expect[t], 4)  # heading 90 deg: +y
        assert _where(st.B, 2) == (4, 4 - expect[t])  # heading 180 deg: -x
        assert _where(st.B, 3) == (4 - expect[t], 4)  # heading 270 deg: -y


def test_remainder_stays_within_half_a_cell_of_the_summed_displacement():
    rng = np.random.default_rng(3)
    occ = np.zeros((61, 61), np.uint8)
    n_theta = 8
    p = _params(n_theta)
    st = _impulse(61, 61, n_theta, 30, 30)
    total = np.zeros((n_theta, 2))
    theta = 0.0
    for t in range(25):
        u, v, w = rng.uniform(-0.7, 0.7), rng.uniform(-0.7, 0.7), rng.normal(0, 0.3)
        for k in range(n_theta):
            psi = theta + k * 2 * math.pi / n_theta
            total[k] += (u * math.cos(psi) - v * math.sin(psi), u * math.sin(psi) + v * math.cos(psi))
        theta += w
        st = O.step(st, occ, p, u, v, w)
        for k in range(n_theta):
            j, i = _where(st.B, k)
            assert abs((i - 30) - total[k, 0]) <= 0.5 + 1e-12
            assert abs((j - 30) - total[k, 1]) <= 0.5 + 1e-12
            assert np.allclose(st.rem[k], total[k] - (i - 30, j - 30), atol=1e-12)


def test_whole_cell_moves_equal_the_bilinear_warp():
    occ = O_map = (np.random.default_rng(4).random((20, 24)) < 0.1).astype(np.uint8)
    pb = O.OracleParams(n_theta=4, cell_m=0.5, sigma_xy=0.7, sigma_theta=0.7)
    pi = O.OracleParams(n_theta=4, cell_m=0.5, sigma_xy=0.7, sigma_theta=0.7, integer_shift=True)
    a = O.init_uniform(occ, 4)
    b = O.init_uniform(occ, 4)
    for u, v in ((1.0, 0.0), (0.5, -1.5), (0.0, 2.0)):  # whole cells at headings 0, 90, 180, 270 deg
        a = O.step(a, occ, pb, u, v, 0.0)
        b = O.step(b, occ, pi, u, v, 0.0)
        assert np.allclose(a.B, b.B, rtol=0, atol=1e-15)
        assert np.allclose(b.rem, 0.0, atol=1e-12)


def test_gate_fires_and_carries():
    # gate and whole-cell warp: 0.4-cell moves accumulate; the gate fires at
    # 1.2 cells (n = 1, carry 0.2) and again three moves later (1.2 + 0.2 -> n = 1, carry 0.4)
    occ = np.zeros((9, 13), np.uint8)
    p = _params(4, gate=True)
    st = _impulse(9, 13, 4, 4, 4)
    pos = []
    for t in range(6):
        st = O.step(st, occ, p, 0.4, 0.0, 0.0)
        pos.append(_where(st.B, 0)[1] - 4)
    assert pos == [0, 0, 1, 1, 1, 2]
    assert abs(st.rem[0, 0] - 0.4) < 1e-12
