"""Pins of the sampled observation update oracle (oracle/sample.py), CPU only.

Floyd-Steinberg dithering (Sec. III-B) is pinned by hand-derived selections,
its limits (black, white), conservation of the total intensity up to the
error that leaves the grid, and equality with an independently structured
wavefront ("pull") formulation.  The sampled update is pinned by its limits:
with every cell selected it is the dense update of eq. (sensor update); with
none it changes nothing; samples never gain mass relative to the rest.
"""

import os
import zlib

import numpy as np
import pytest

import oracle as O
from gen import bsp_rooms, noisy_scan, random_odometry, range_table

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
F = np.float32


def _golden():
    out = []
    for line in open(os.path.join(GOLDEN, "floyd_steinberg_small.txt")):
        if line.startswith("#") or not line.strip():
            continue
        left, right = line.split("|")
        name, rows, cols, value = left.split()
        sel = np.array([int(x) for x in right.split()], np.uint8).reshape(int(rows), int(cols))
        out.append((name, np.full((int(rows), int(cols)), float(value), np.float32), sel))
    return out


@pytest.mark.parametrize("case", _golden(), ids=lambda c: c[0])
def test_hand_derived_selections(case):
    _, img, sel = case
    assert np.array_equal(O.floyd_steinberg(img), sel)


def test_black_and_white():
    assert O.floyd_steinberg(np.zeros((7, 9), np.float32)).sum() == 0
    assert O.floyd_steinberg(np.ones((7, 9), np.float32)).sum() == 63


@pytest.mark.parametrize("seed", [0, 1])
def test_selected_count_tracks_total_intensity(seed):
    # error only escapes through the right and bottom borders, at most 1/2 per
    # cell it leaves from, so |#selected - sum I| <= (W + H) / 2 + 1
    rng = np.random.default_rng(seed)
    img = rng.uniform(0, 1, (23, 31)).astype(np.float32)
    n = int(O.floyd_steinberg(img).sum())
    assert abs(n - float(img.sum())) <= (23 + 31) / 2 + 1


def _wavefront_pull(img):
    # cell (i, j) runs at time t = i + 2 j, after all of its sources; it pulls
    # the errors of (i-1, j-1), (i, j-1), (i+1, j-1) and (i-1, j) in the order
    # the raster scan would have pushed them
    H, W = img.shape
    e = np.zeros((H, W), np.float32)
    out = np.zeros((H, W), np.uint8)
    for t in range(W + 2 * H):
        for j in range(H):
            i = t - 2 * j
            if not 0 <= i < W:
                continue
            acc = F(0.0)
            if j > 0:
                if i > 0:
                    acc = F(acc + F(F(1 / 16) * e[j - 1, i - 1]))
                acc = F(acc + F(F(5 / 16) * e[j - 1, i]))
                if i + 1 < W:
                    acc = F(acc + F(F(3 / 16) * e[j - 1, i + 1]))
            if i > 0:
                acc = F(acc + F(F(7 / 16) * e[j, i - 1]))
            v = F(img[j, i] + acc)
            out[j, i] = 1 if v >= F(0.5) else 0
            e[j, i] = F(v - F(out[j, i]))
    return out


@pytest.mark.parametrize("shape", [(1, 17), (13, 1), (9, 14), (16, 16)])
def test_raster_push_equals_wavefront_pull(shape):
    rng = np.random.default_rng(sum(shape))
    img = (rng.uniform(0, 1, shape) ** 3).astype(np.float32)
    assert np.array_equal(O.floyd_steinberg(img), _wavefront_pull(img))


def test_intensity_targets_the_sample_count():
    rng = np.random.default_rng(5)
    m = rng.uniform(0, 1, (40, 50)) ** 4
    I = O.dither_intensity(m, 200)
    assert I.dtype == np.float32 and I.max() <= 1.0
    assert abs(float(I.sum()) - 200) < 1e-3 * 200  # no cell saturates here
    assert O.dither_intensity(np.zeros((3, 3)), 10).sum() == 0
    # a peak that would ask for more than one sample in its cell saturates at 1
    peak = np.full((4, 4), 0.01)
    peak[1, 2] = 1.0
    Ip = O.dither_intensity(peak, 8)  # 8 * 1 / 1.15 = 6.96 before clamping
    assert Ip[1, 2] == np.float32(1.0) and Ip.max() == np.float32(1.0)
    assert Ip[0, 0] == np.float32(np.float32(8 * np.float32(0.01)) / np.float32(1.15))


def _scan_setup():
    occ = bsp_rooms(24, 20, seed=61)
    n_theta = 6
    st = O.init_uniform(occ, n_theta)
    p = O.OracleParams(n_theta=n_theta, cell_m=0.1, sigma_xy=0.6, sigma_theta=0.6)
    for u, v, w in random_odometry(4, seed=62):
        st = O.step(st, occ, p, u, v, w)
    R = range_table(occ, 0.1, 36, 2.5)
    Rq = O.quantize_ranges(R, 2.5)
    free = np.argwhere(occ == 0)
    j, i = free[len(free) // 3]
    z = noisy_scan(occ, 0.1, ((i + 0.5) * 0.1, (j + 0.5) * 0.1, 0.4), 36, 2.5, 0.1, seed=63)
    return occ, st, Rq, O.quantize_ranges(z, 2.5)


def test_full_selection_is_the_dense_update():
    occ, st, Rq, zq = _scan_setup()
    dense = O.apply_scan(st, Rq, zq, 0.15, 2.5)
    full = O.apply_scan_sampled(st, Rq, zq, 0.15, 2.5, np.ones(occ.shape, np.uint8))
    assert np.allclose(full.B, dense.B, rtol=0, atol=1e-12)
    assert full.log_norm == pytest.approx(dense.log_norm, abs=1e-9)


def test_empty_selection_changes_nothing():
    occ, st, Rq, zq = _scan_setup()
    out = O.apply_scan_sampled(st, Rq, zq, 0.15, 2.5, np.zeros(occ.shape, np.uint8))
    assert np.array_equal(out.B, st.B) and out.log_norm == st.log_norm


def test_samples_never_gain_relative_to_the_rest():
    occ, st, Rq, zq = _scan_setup()
    mask = O.sample_mask(st.B, 40)
    assert 20 <= mask.sum() <= 60
    out = O.apply_scan_sampled(st, Rq, zq, 0.15, 2.5, mask)
    ratio = np.where(st.B > 0, out.B / np.where(st.B > 0, st.B, 1), 0)  # per-state gain
    sampled = np.broadcast_to(mask.astype(bool), st.B.shape) & (st.B > 0)
    unsampled = ~np.broadcast_to(mask.astype(bool), st.B.shape) & (st.B > 0)
    assert ratio[sampled].max() <= ratio[unsampled].min() * (1 + 1e-12)
    assert abs(out.B.sum() - 1.0) < 1e-12


# ---- the C form of the dithering oracle (large images) ---------------------------

@pytest.mark.parametrize("case", _golden(), ids=lambda c: c[0])
def test_c_form_hand_derived_selections(case):
    _, img, sel = case
    assert np.array_equal(O.floyd_steinberg_c(img), sel)


@pytest.mark.parametrize("shape", [(1, 1), (1, 29), (31, 1), (2, 2), (17, 23), (40, 64)])
@pytest.mark.parametrize("dist", ["uniform", "cubed", "near_half", "wide"])
def test_c_form_equals_python_form(shape, dist):
    # bit-for-bit equality with the pinned raster loop over value mixes that
    # exercise the threshold, negative errors and intensities above one
    rng = np.random.default_rng(zlib.crc32(repr((shape, dist)).encode()))
    if dist == "uniform":
        img = rng.uniform(0, 1, shape)
    elif dist == "cubed":
        img = rng.uniform(0, 1, shape) ** 3
    elif dist == "near_half":
        img = 0.5 + rng.integers(-3, 4, shape) * np.float32(2.0 ** -24)
    else:
        img = rng.uniform(-0.5, 2.0, shape)
    img = img.astype(np.float32)
    assert np.array_equal(O.floyd_steinberg_c(img), O.floyd_steinberg(img))


def test_c_form_empty_image():
    assert O.floyd_steinberg_c(np.zeros((0, 5), np.float32)).shape == (0, 5)
