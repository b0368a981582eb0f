"""Pins of the FP64 oracle against closed forms, invariants and a brute force.

These run on the CPU only and never touch the HIP library.  Each test names
the passage of the paper whose consequence it checks.
"""

import math
import os

import numpy as np
import pytest

import oracle as O
from gen import bsp_rooms, random_odometry
from tests.bruteforce import DenseModel

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([float(x) for x in line.split()])
    return np.array(rows)


def _delta_state(shape, n_theta, points):
    B = np.zeros((n_theta,) + shape)
    for (k, j, i) in points:
        B[k, j, i] = 1.0
    B /= B.sum()
    return O.FilterState(B=B)


def test_taps_sum_to_one_and_match_closed_form():
    # eq. (Gaussian kernel) sampled on integers; sigma = 1, radius 3
    g = O.gaussian_taps(1.0, 3)
    raw = np.array([math.exp(-m * m / 2.0) for m in range(-3, 4)])
    assert abs(g.sum() - 1.0) < 1e-15
    assert np.allclose(g, raw / raw.sum(), rtol=0, atol=1e-16)
    assert np.array_equal(O.gaussian_taps(0.0, 2), np.array([0, 0, 1.0, 0, 0]))
    assert O.default_radius(0.5) == 2 and O.default_radius(1.0) == 3


def test_integer_shift_lands_on_exact_cell():
    # Sec. III-A-1: an integer displacement moves an impulse to p + d exactly
    occ = np.zeros((16, 16), np.uint8)
    p = O.OracleParams(n_theta=1, cell_m=0.1, sigma_xy=0.0, sigma_theta=0.0)
    st = _delta_state(occ.shape, 1, [(0, 6, 5)])
    nst = O.step(st, occ, p, 2 * 0.1, 1 * 0.1, 0.0)
    assert nst.B[0, 7, 7] == pytest.approx(1.0, abs=1e-12)
    assert nst.B.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.count_nonzero(nst.B > 1e-12) == 1


def test_fractional_shift_bilinear_weights_and_mass_centre():
    # golden: bilinear weights for d = (0.25, 0.5)
    gold = _load_golden("bilinear_quarter_half.txt")
    occ = np.zeros((12, 12), np.uint8)
    p = O.OracleParams(n_theta=1, cell_m=1.0, sigma_xy=0.0, sigma_theta=0.0)
    st = _delta_state(occ.shape, 1, [(0, 4, 3)])
    nst = O.step(st, occ, p, 0.25, 0.5, 0.0)
    for di, dj, wgt in gold:
        assert nst.B[0, 4 + int(dj), 3 + int(di)] == pytest.approx(wgt, abs=1e-15)
    jj, ii = np.mgrid[0:12, 0:12]
    cx = (nst.B[0] * ii).sum()
    cy = (nst.B[0] * jj).sum()
    assert cx == pytest.approx(3.25, abs=1e-14) and cy == pytest.approx(4.5, abs=1e-14)


def test_four_heading_bins_move_in_rotated_directions():
    # golden: channel k moves by R(k * 90 deg) [u, v]
    gold = _load_golden("theta4_directions.txt")
    occ = np.zeros((11, 11), np.uint8)
    p = O.OracleParams(n_theta=4, cell_m=1.0, sigma_xy=0.0, sigma_theta=0.0)
    for u, v, k, di, dj in gold:
        st = _delta_state(occ.shape, 4, [(int(k), 5, 5)])
        nst = O.step(st, occ, p, u, v, 0.0)
        assert nst.B[int(k), 5 + int(dj), 5 + int(di)] == pytest.approx(1.0, abs=1e-12)


def test_blur_of_impulse_is_sampled_kernel():
    # Sec. III-A-2: away from walls the 3-D blur of an impulse is g_x g_y g_theta
    occ = np.zeros((25, 23), np.uint8)
    p = O.OracleParams(n_theta=16, cell_m=1.0, sigma_xy=1.0, sigma_theta=1.0)
    st = _delta_state(occ.shape, 16, [(5, 12, 11)])
    nst = O.step(st, occ, p, 0.0, 0.0, 0.0)
    g = lambda m: math.exp(-m * m / 2.0)
    z = sum(g(m) for m in range(-3, 4))
    exp = np.zeros_like(nst.B)
    for dk in range(-3, 4):
        for dj in range(-3, 4):
            for di in range(-3, 4):
                exp[5 + dk, 12 + dj, 11 + di] = g(dk) * g(dj) * g(di) / z ** 3
    assert np.abs(nst.B - exp).max() < 1e-16


def test_theta_blur_wraps_circularly():
    occ = np.zeros((9, 9), np.uint8)
    p = O.OracleParams(n_theta=8, cell_m=1.0, sigma_xy=0.0, sigma_theta=1.0)
    st = _delta_state(occ.shape, 8, [(0, 4, 4)])
    nst = O.step(st, occ, p, 0.0, 0.0, 0.0)
    b = nst.B[:, 4, 4]
    assert b[7] == pytest.approx(b[1], abs=0) and b[6] == pytest.approx(b[2], abs=0)
    assert b[5] == pytest.approx(b[3], abs=0) and b[7] > 0 and b[4] == 0.0  # 4 bins > radius


def test_theta_count_smaller_than_kernel_wraps_repeatedly():
    # Theta = 2 with radius 3: taps fold onto the two channels
    occ = np.zeros((5, 5), np.uint8)
    p = O.OracleParams(n_theta=2, cell_m=1.0, sigma_xy=0.0, sigma_theta=1.0)
    st = _delta_state(occ.shape, 2, [(0, 2, 2)])
    nst = O.step(st, occ, p, 0.0, 0.0, 0.0)
    g = O.gaussian_taps(1.0, 3)
    even = g[0::2].sum()  # offsets -3, -1, 1, 3 land on channel 1; -2, 0, 2 on channel 0
    assert nst.B[0, 2, 2] == pytest.approx(g[1] + g[3] + g[5], abs=1e-16)
    assert nst.B[1, 2, 2] == pytest.approx(even, abs=1e-16)


def test_occupied_cells_are_exactly_zero_after_every_step():
    # Alg. 1: multiplication by M after the blur
    occ = bsp_rooms(48, 40, seed=11)
    p = O.OracleParams(n_theta=12, cell_m=0.1, sigma_xy=0.5, sigma_theta=0.5)
    odo = random_odometry(10, seed=12)
    occupied = occ.astype(bool)

    def check(t, st):
        assert np.all(st.B[:, occupied] == 0.0)

    O.run(occ, p, odo, callback=check)


def test_uniform_over_free_is_a_fixed_point_of_wall_normalisation():
    # Sec. III-A-3 (the "cliff" argument): dividing by G(B_0) makes uniform
    # free space invariant under zero motion; without it mass leaks at walls.
    occ = bsp_rooms(40, 36, seed=5)
    st = O.init_uniform(occ, 6)
    p = O.OracleParams(n_theta=6, cell_m=0.1, sigma_xy=1.0, sigma_theta=1.0)
    nst = O.step(st, occ, p, 0.0, 0.0, 0.0)
    assert np.abs(nst.B - st.B).max() <= 1e-15 * st.B.max() * 10
    p_off = O.OracleParams(n_theta=6, cell_m=0.1, sigma_xy=1.0, sigma_theta=1.0,
                           wall_normalize=False)
    nst_off = O.step(st, occ, p_off, 0.0, 0.0, 0.0)
    assert np.abs(nst_off.B - st.B).max() > 1e-2 * st.B.max()


def test_mirror_symmetry():
    # Mirroring the map in x maps heading psi to pi - psi, i.e. channel k to
    # Theta/2 - k, and odometry (u, v, w) to (u, -v, -w).
    occ = bsp_rooms(30, 26, seed=7)
    p = O.OracleParams(n_theta=8, cell_m=0.1, sigma_xy=0.7, sigma_theta=0.8)
    odo = random_odometry(12, seed=8)
    a = O.run(occ, p, odo)
    odo_m = odo * np.array([1.0, -1.0, -1.0])
    b = O.run(occ[:, ::-1].copy(), p, odo_m)
    perm = [(8 // 2 - k) % 8 for k in range(8)]
    mirrored = a.B[perm][:, :, ::-1]
    assert np.abs(mirrored - b.B).max() < 1e-12 * a.B.max()
    assert a.log_norm == pytest.approx(b.log_norm, abs=1e-12)


@pytest.mark.parametrize("shape,n_theta,sxy,rxy,sth,rth,wall,maskb", [
    ((5, 6), 4, 0.8, 2, 0.7, 1, True, True),
    ((7, 8), 8, 1.0, 3, 1.0, 3, True, True),
    ((6, 5), 3, 0.5, 2, 1.3, 2, False, True),
    ((6, 6), 5, 0.6, 1, 0.9, 2, True, False),
])
def test_against_dense_brute_force(shape, n_theta, sxy, rxy, sth, rth, wall, maskb):
    rng = np.random.default_rng(hash(shape) % 1000)
    occ = (rng.random(shape) < 0.2).astype(np.uint8)
    occ[0, 0] = 0
    p = O.OracleParams(n_theta=n_theta, cell_m=0.1, sigma_xy=sxy, sigma_theta=sth,
                       radius_xy=rxy, radius_theta=rth, wall_normalize=wall,
                       mask_before_blur=maskb)
    dense = DenseModel(occ, n_theta, sxy, rxy, sth, rth, wall_normalize=wall,
                       mask_before_blur=maskb)
    odo = random_odometry(20, seed=3) * np.array([2.0, 2.0, 3.0])
    st = O.init_uniform(occ, n_theta)
    b = st.B.copy()
    theta = 0.0
    log_norm = 0.0
    for u, v, w in odo:
        st = O.step(st, occ, p, u, v, w)
        nb, mass = dense.step(b, u, v, theta, 0.1)
        b = nb / mass
        log_norm += math.log(mass)
        theta += w
        assert np.abs(st.B - b).max() <= 1e-12 * b.max()
    assert st.log_norm == pytest.approx(log_norm, rel=1e-12, abs=1e-12)
    assert st.B.sum() == pytest.approx(1.0, abs=1e-14)


def test_mass_is_one_after_every_step():
    occ = bsp_rooms(64, 64, seed=1)
    p = O.OracleParams(n_theta=36, cell_m=0.1, sigma_xy=0.5, sigma_theta=0.5)
    odo = random_odometry(5, seed=2)
    O.run(occ, p, odo, callback=lambda t, s: pytest.approx(1.0, abs=1e-14) == s.B.sum()
          or pytest.fail("mass"))


def test_subcell_gate_accumulates_until_one_cell():
    # Alg. 1 "IF |u_{t,k}| >= 1": three 0.4-cell moves act as one 1.2-cell move
    occ = np.zeros((16, 16), np.uint8)
    occ[0, :] = occ[-1, :] = occ[:, 0] = occ[:, -1] = 1
    base = dict(n_theta=4, cell_m=1.0, sigma_xy=0.6, sigma_theta=0.6)
    gated = O.OracleParams(subcell_gate=True, **base)
    plain = O.OracleParams(**base)
    st = _delta_state(occ.shape, 4, [(0, 7, 6), (1, 8, 8)])
    g1 = O.step(st, occ, gated, 0.4, 0.0, 0.0)
    assert np.array_equal(g1.B, st.B)
    g2 = O.step(g1, occ, gated, 0.4, 0.0, 0.0)
    assert np.array_equal(g2.B, st.B)
    g3 = O.step(g2, occ, gated, 0.4, 0.0, 0.0)
    ref = O.step(st, occ, plain, 1.2, 0.0, 0.0)
    assert np.abs(g3.B - ref.B).max() < 1e-14


def test_all_mass_into_wall_is_degenerate():
    occ = np.ones((10, 10), np.uint8)
    occ[4:6, 4:6] = 0
    p = O.OracleParams(n_theta=4, cell_m=1.0, sigma_xy=0.0, sigma_theta=0.0)
    st = O.init_uniform(occ, 4)
    nst = O.step(st, occ, p, 3.0, 0.0, 0.0)
    assert nst.degenerate and np.array_equal(nst.B, st.B)


def test_readout_argmax_lowest_index_wins():
    B = np.zeros((3, 4, 5))
    B[1, 2, 3] = B[2, 0, 0] = 0.5
    assert O.argmax_pose(B) == (1, 2, 3)
    assert O.belief_map(B)[2, 3] == 0.5
