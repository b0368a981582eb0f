"""Pins of the FP64 scan-update oracle (eq. sensor update, dense form).

CPU only.  The distance is checked against the expanded product form and a
per-beam linear-domain brute force; the posterior against the ordering
property of eq. (observation constraint) and an independent log-sum-exp.
"""

import math

import numpy as np
import pytest

import oracle as O
from gen import bsp_rooms, range_table


def test_quantised_ranges_are_exact_centred_counts():
    h = 10.0 / 256
    r = np.array([0.0, h * 0.49, h * 0.51, 128 * h, 256 * h, 300 * h, 5 * h])
    q = O.quantize_ranges(r, 10.0)
    assert q.tolist() == [-128, -128, -127, 0, 128, 128, -123]
    assert q.dtype == np.int64


def test_beam_offsets_closed_form():
    # channel k of 36 at theta = 0 looks along 10k degrees: column 10k of 360
    assert O.beam_offsets(0.0, 36, 360).tolist() == [10 * k for k in range(36)]
    s = O.beam_offsets(math.radians(0.7), 36, 360)
    assert s.tolist() == [(10 * k + 1) % 360 for k in range(36)]
    s = O.beam_offsets(math.radians(-3.2), 4, 360)
    assert s.tolist() == [357, 87, 177, 267]


def _small_table(seed=0, n=64):
    occ = bsp_rooms(20, 18, seed=seed)
    R = range_table(occ, 0.1, n, 3.0)
    return occ, R


def test_direct_distance_equals_expanded_product_form():
    # D = sum z^2 - 2 R C + sum r^2 with the circulant C[beta, k] = z[(beta - s_k) mod N]
    occ, R = _small_table()
    n = R.shape[1]
    Rq = O.quantize_ranges(R, 3.0)
    rng = np.random.default_rng(1)
    zq = rng.integers(-128, 129, n)
    s = O.beam_offsets(0.3, 12, n)
    D = O.scan_sqdist(Rq, zq, s)
    beta = np.arange(n)
    C = np.stack([zq[(beta - sk) % n] for sk in s], axis=1)  # (N, Theta)
    X = Rq @ C
    D2 = (zq * zq).sum() - 2 * X.T + (Rq * Rq).sum(axis=1)[None, :]
    assert np.array_equal(D, D2)


def test_noise_free_scan_gives_zero_distance_and_posterior_peak_at_truth():
    occ, R = _small_table(seed=2)
    H, W = occ.shape
    n = R.shape[1]
    Rq = O.quantize_ranges(R, 3.0)
    n_theta = 8
    i, j, k = 7, 9, 3
    assert occ[j, i] == 0
    s = O.beam_offsets(0.0, n_theta, n)
    cell = j * W + i
    zq = np.array([Rq[cell, (b + s[k]) % n] for b in range(n)])
    D = O.scan_sqdist(Rq, zq, s)
    assert D[k, cell] == 0
    st = O.init_uniform(occ, n_theta)
    post = O.apply_scan(st, Rq, zq, 0.1, 3.0)
    best = post.B.max()
    assert post.B[k, j, i] == best
    ties = np.argwhere(post.B == best)
    for kk, jj, ii in ties:
        assert D[kk, jj * W + ii] == 0


def test_posterior_never_demotes_a_better_match():
    # eq. (observation constraint): for D(a) <= D(b), B'(a)/B'(b) >= B(a)/B(b)
    occ, R = _small_table(seed=3)
    n = R.shape[1]
    Rq = O.quantize_ranges(R, 3.0)
    rng = np.random.default_rng(4)
    zq = rng.integers(-128, 129, n)
    n_theta = 6
    st = O.init_uniform(occ, n_theta)
    st.B = st.B * rng.uniform(0.5, 1.5, st.B.shape)
    st.B /= st.B.sum()
    post = O.apply_scan(st, Rq, zq, 0.5, 3.0)
    D = O.scan_sqdist(Rq, zq, O.beam_offsets(0.0, n_theta, n)).reshape(st.B.shape)
    nz = np.argwhere(st.B > 0)
    for _ in range(500):
        a = tuple(nz[rng.integers(len(nz))])
        b = tuple(nz[rng.integers(len(nz))])
        if D[a] > D[b]:
            a, b = b, a
        lhs = math.log(post.B[a]) - math.log(post.B[b]) if post.B[b] > 0 else math.inf
        rhs = math.log(st.B[a]) - math.log(st.B[b])
        assert lhs >= rhs - 1e-9


def test_linear_domain_brute_force_and_log_normaliser():
    # per-beam loop, nearest table direction per beam angle, linear-domain product
    occ = bsp_rooms(9, 8, seed=5)
    H, W = occ.shape
    n = 16
    R = range_table(occ, 0.25, n, 2.0)
    Rq = O.quantize_ranges(R, 2.0)
    rng = np.random.default_rng(6)
    zq = rng.integers(-60, 60, n)
    n_theta = 4
    theta = 0.41
    sigma = 2.0  # wide enough that every likelihood stays representable in linear space
    h = 2.0 / 256
    c = h * h / (2 * sigma * sigma)
    st = O.init_uniform(occ, n_theta)
    st.theta = theta
    st.B = st.B * rng.uniform(0.2, 1.0, st.B.shape)
    st.B /= st.B.sum()
    lik = np.zeros_like(st.B)
    for k in range(n_theta):
        psi = theta + k * 2 * math.pi / n_theta
        for j in range(H):
            for i in range(W):
                d = 0
                for b in range(n):
                    ang = psi + b * 2 * math.pi / n
                    beta = int(round(ang / (2 * math.pi / n))) % n
                    d += (int(zq[b]) - int(Rq[j * W + i, beta])) ** 2
                lik[k, j, i] = math.exp(-c * d)
    joint = st.B * lik
    expect = joint / joint.sum()
    post = O.apply_scan(st, Rq, zq, sigma, 2.0)
    assert np.abs(post.B - expect).max() <= 1e-12 * expect.max()
    assert post.log_norm - st.log_norm == pytest.approx(math.log(math.fsum(joint.reshape(-1))),
                                                         abs=1e-12)


def test_continuous_model_equals_the_quantised_one_on_quantised_ranges():
    # with every range a multiple of h, the continuous per-beam Gaussian is the
    # quantised model: D_continuous = h^2 D_quantised, so the posteriors agree
    occ = bsp_rooms(30, 26, seed=81)
    R = range_table(occ, 0.1, 48, 3.0)
    h = 3.0 / 256
    Rq = O.quantize_ranges(R, 3.0)
    Rh = (Rq + 128) * h                         # ranges rounded to multiples of h
    rng = np.random.default_rng(82)
    z = rng.uniform(0.0, 3.1, 48)
    zq = O.quantize_ranges(z, 3.0)
    zh = (zq + 128) * h
    st = O.init_uniform(occ, 6)
    st.theta = 0.4
    a = O.apply_scan(st, Rq, zq, 0.2, 3.0)
    b = O.apply_scan_continuous(st, Rh, zh, 0.2)
    assert np.allclose(a.B, b.B, rtol=0, atol=1e-12 * a.B.max())
    assert abs(a.log_norm - b.log_norm) < 1e-9
    # and the direct distance is h^2 times the integer one
    s = O.beam_offsets(0.4, 6, 48)
    assert np.allclose(O.scan_sqdist_continuous(Rh, zh, s), h * h * O.scan_sqdist(Rq, zq, s), rtol=1e-12, atol=0)


def test_continuous_distance_brute_force():
    # one cell, two channels, four beams written out by hand
    R = np.array([[1.0, 2.0, 3.0, 4.0]])
    z = np.array([1.5, 2.0, 2.0, 5.0])
    s = np.array([0, 1])
    # k = 0: columns 0, 1, 2, 3; k = 1: columns 1, 2, 3, 0
    d0 = 0.25 + 0.0 + 1.0 + 1.0
    d1 = (1.5 - 2.0) ** 2 + (2.0 - 3.0) ** 2 + (2.0 - 4.0) ** 2 + (5.0 - 1.0) ** 2
    assert np.allclose(O.scan_sqdist_continuous(R, z, s)[:, 0], [d0, d1], rtol=0, atol=1e-15)
