"""Pins of the anisotropic, heading-rotated motion noise in the oracle (CPU only).

Eq. (Gaussian kernel) with the rotated covariance R(psi) diag(sf^2, sl^2) R(psi)^T:
forward noise along a channel's heading, lateral noise across it.  Pinned by
the isotropic limit (the separable step), an independent dense brute force
built from the unseparated 3-D quadratic form with one kernel per target
channel, and the direction a thin kernel spreads along at 0, 45 and 90 degrees.
"""

import math

import numpy as np
import pytest

import oracle as O
from gen import bsp_rooms, random_odometry
from tests.bruteforce import DenseModel


def test_isotropic_limit_is_the_separable_step():
    occ = bsp_rooms(30, 26, seed=91)
    n_theta = 8
    pi = O.OracleParams(n_theta=n_theta, cell_m=0.1, sigma_xy=0.8, sigma_theta=0.7)
    pa = O.OracleParams(n_theta=n_theta, cell_m=0.1, sigma_xy=0.8, sigma_theta=0.7, sigma_lateral=0.8)
    a = O.init_uniform(occ, n_theta)
    b = O.init_uniform(occ, n_theta)
    for u, v, w in random_odometry(4, seed=92):
        a = O.step(a, occ, pi, u, v, w)
        b = O.step(b, occ, pa, u, v, w)
        assert np.allclose(a.B, b.B, rtol=0, atol=1e-14)
        assert b.log_norm == pytest.approx(a.log_norm, abs=1e-12)


@pytest.mark.parametrize("case", [(5, 6, 4, 1.0, 0.4, 0.6, 2, 1), (4, 7, 6, 0.5, 1.1, 0.0, 2, 0)])
def test_matches_the_dense_brute_force(case):
    H, W, n_theta, sf, sl, sth, rxy, rth = case
    rng = np.random.default_rng(sum(case[:3]))
    occ = (rng.random((H, W)) < 0.15).astype(np.uint8)
    occ[H // 2, W // 2] = 0
    p = O.OracleParams(n_theta=n_theta, cell_m=0.1, sigma_xy=sf, sigma_theta=sth, radius_xy=rxy,
                       radius_theta=rth, sigma_lateral=sl)
    st = O.init_uniform(occ, n_theta)
    for u, v, w in ((0.07, 0.02, 0.3), (-0.04, 0.05, -0.2), (0.11, -0.03, 0.9)):
        model = DenseModel(occ, n_theta, sf, rxy, sth, rth, sigma_lateral=sl, theta=st.theta)
        ref, kept = model.step(st.B, u, v, st.theta, 0.1)
        st = O.step(st, occ, p, u, v, w)
        assert np.allclose(st.B, ref / kept, rtol=0, atol=1e-12)


@pytest.mark.parametrize("psi,axis", [(0.0, (1, 0)), (math.pi / 4, (1, 1)), (math.pi / 2, (0, 1))])
def test_thin_kernel_spreads_along_the_heading(psi, axis):
    # lateral sigma 0.05 cells: all but ~1e-80 of the weight lies on the line
    # through the centre along (cos psi, sin psi) sampled at whole cells
    g = O.rotated_taps(1.2, 0.05, 3, psi)
    on = np.zeros_like(g, dtype=bool)
    for t in range(-3, 4):
        on[3 + t * axis[1], 3 + t * axis[0]] = True
    assert g[~on].max() < 1e-30
    assert g[on].sum() == pytest.approx(1.0, abs=1e-12)
    # the spread along the line is the forward Gaussian, for heading 0 the 1-D taps
    if psi == 0.0:
        assert np.allclose(g[3], O.gaussian_taps(1.2, 3), atol=1e-15)


def test_channel_heading_orients_the_blur_of_an_impulse():
    # 8 channels, no motion: the impulse in channel 1 (45 deg) spreads along the
    # diagonal, in channel 2 (90 deg) along y
    occ = np.zeros((15, 15), np.uint8)
    n_theta = 8
    p = O.OracleParams(n_theta=n_theta, cell_m=1.0, sigma_xy=1.0, sigma_theta=0.0, radius_xy=3,
                       radius_theta=0, wall_normalize=False, sigma_lateral=0.05)
    B = np.zeros((n_theta, 15, 15))
    B[:, 7, 7] = 1.0 / n_theta
    st = O.step(O.FilterState(B=B), occ, p, 0.0, 0.0, 0.0)
    d = np.array([st.B[1, 7 + t, 7 + t] for t in range(-3, 4)])
    assert d.sum() == pytest.approx(st.B[1].sum(), rel=1e-12)
    y = st.B[2, :, 7]
    assert y.sum() == pytest.approx(st.B[2].sum(), rel=1e-12)
