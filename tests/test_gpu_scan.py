"""Dense scan update on the GPU vs the FP64 oracle (GPU only; through the C ABI).

The squared distance D is an exact integer on both sides (quantised ranges,
exact MFMA accumulation), so it is compared bit for bit, for BF16 and FP32
matrix operands.  The posterior is compared with the oracle's log-domain
update: peak-normalised max-abs error <= 1e-5 for FP32 storage, the bound
stated for FP32 results.  The FP32 arithmetic of the update stays well
inside it: each stored value is exp(L - M*) with L - M* formed from FP32
logarithms of values near the peak (abs. error ~1e-7 each) and
c (D - D_ref) with D exact and |c (D - D_ref)| of a few nats for the states
that carry mass (abs. error ~3e-7), plus the FP32 exp (~1e-7): about 5e-7
relative per value.  The log-normaliser after a scan is checked against the
oracle's scan started from the very FP32 prior the GPU holds, so the
storage's precision does not enter the comparison.
"""

import math

import numpy as np
import pytest

import oracle as O
from gen import bsp_rooms, noisy_scan, random_odometry, range_table, rooms_and_corridors, smooth_trajectory
from tests.gpu_harness import (in_tie_set, make_gpu, needs_gpu, oracle_params, oracle_state_from, peak_err,
                                say, stored_belief)

pytestmark = [pytest.mark.gpu, needs_gpu]

SCAN_PEAK_TOL = 1e-5
# the log-normaliser: absolute plus relative part
LN_ABS, LN_REL = 1e-5, 1e-6


def _setup(occ, cell, n_dirs, max_range, n_theta, sxy=0.7, sth=0.7, flags=3, theta0=0.0):
    R = range_table(occ, cell, n_dirs, max_range)
    m, f = make_gpu(occ, cell, n_theta, sxy, sth, flags=flags, range_table=R, max_range_m=max_range,
                    theta0=theta0)
    return R, m, f


@pytest.mark.parametrize("f32_ops", [False, True])
def test_distance_is_exact_small(f32_ops):
    occ = bsp_rooms(40, 33, seed=31)
    theta0 = 0.377
    flags = 3 | (8 if f32_ops else 0)
    R, m, f = _setup(occ, 0.1, 64, 3.0, 12, flags=flags, theta0=theta0)
    rng = np.random.default_rng(32)
    z = rng.uniform(0.0, 3.2, 64).astype(np.float32)
    say(f"[scan] exact D small f32_ops={f32_ops}")
    d_gpu = f.scan_sqdist(z).cpu().numpy().astype(np.int64)
    Rq = O.quantize_ranges(R, 3.0)
    zq = O.quantize_ranges(z, 3.0)
    d_ref = O.scan_sqdist(Rq, zq, O.beam_offsets(theta0, 12, 64)).reshape(12, 33, 40)
    assert np.array_equal(d_gpu, d_ref)


@pytest.mark.parametrize("n_theta", [5, 72, 96, 120, 360])
def test_distance_is_exact_at_depth_384(n_theta):
    # 360 directions (depth 384), from a few channels to 360 (several passes
    # over channel blocks); the distance output streams the circulant operand
    occ = bsp_rooms(48, 37, seed=35)
    R, m, f = _setup(occ, 0.1, 360, 4.0, n_theta, theta0=0.9)
    rng = np.random.default_rng(36)
    z = rng.uniform(0.0, 4.2, 360).astype(np.float32)
    say(f"[scan] exact D depth 384 n_theta={n_theta}")
    d_gpu = f.scan_sqdist(z).cpu().numpy().astype(np.int64).reshape(n_theta, -1)
    Rq = O.quantize_ranges(R, 4.0)
    zq = O.quantize_ranges(z, 4.0)
    cells = rng.choice(48 * 37, 400, replace=False)
    d_ref = O.scan_sqdist(Rq, zq, O.beam_offsets(0.9, n_theta, 360), rows=cells)
    assert np.array_equal(d_gpu[:, cells], d_ref)


@pytest.mark.parametrize("n_theta,f32_ops", [(72, False), (120, False), (72, True), (120, True)])
def test_scan_update_at_depth_384_matches_oracle(n_theta, f32_ops):
    # the likelihood pass at depth 384: with BF16 operands up to 96 channels
    # stage the circulant operand in LDS and more stream it; FP32 operands
    # always stream it
    occ = bsp_rooms(40, 30, seed=37)
    R, m, f = _setup(occ, 0.1, 360, 4.0, n_theta, sxy=0.8, sth=0.8, flags=3 | (8 if f32_ops else 0))
    z = noisy_scan(occ, 0.1, (1.55, 1.45, 0.3), 360, 4.0, 0.1, seed=38)
    say(f"[scan] update depth 384 n_theta={n_theta} f32_ops={f32_ops}")
    f.apply_scan(z, 0.1)
    b_gpu, _, _, _ = f.read_belief()
    st = O.init_uniform(occ, n_theta)
    st = O.apply_scan(st, O.quantize_ranges(R, 4.0), O.quantize_ranges(z, 4.0), 0.1, 4.0)
    assert peak_err(b_gpu, st.B) <= SCAN_PEAK_TOL


def test_distance_is_exact_full_size_sampled():
    # 512x512 cells, 360 directions, 72 channels: the GEMM shape of the scan workload
    occ = rooms_and_corridors(512, 512, seed=3)
    R, m, f = _setup(occ, 0.05, 360, 10.0, 72, sxy=1.0, sth=1.0, theta0=1.234)
    rng = np.random.default_rng(33)
    poses, _ = smooth_trajectory(occ, 0.05, 1, seed=4)
    z = noisy_scan(occ, 0.05, poses[0], 360, 10.0, 0.1, seed=7)
    say("[scan] exact D full size")
    d_gpu = f.scan_sqdist(z).cpu().numpy().reshape(72, -1)
    Rq = O.quantize_ranges(R, 10.0)
    zq = O.quantize_ranges(z, 10.0)
    cells = rng.choice(512 * 512, 3000, replace=False)
    d_ref = O.scan_sqdist(Rq, zq, O.beam_offsets(1.234, 72, 360), rows=cells)
    assert np.array_equal(d_gpu[:, cells].astype(np.int64), d_ref)


_last_prior, _last_scan = [None], [None]  # the prior and scan of the latest step of _motion_and_scans


def _motion_and_scans(f32_ops, sigma_scan, seed_pose):
    """30 odometry steps on a 64 x 56 plan with a 90-beam scan every 10 steps;
    yields (t, GPU filter, oracle state, prior oracle state from the GPU's own
    stored prior, quantised table, quantised scan) after each scan."""
    occ = bsp_rooms(64, 56, seed=34)
    n_theta = 16
    flags = 3 | (8 if f32_ops else 0)
    R, m, f = _setup(occ, 0.1, 90, 4.0, n_theta, flags=flags)
    p = oracle_params(n_theta, 0.1, 0.7, 0.7, flags=3)
    Rq = O.quantize_ranges(R, 4.0)
    st = O.init_uniform(occ, n_theta)
    odo = random_odometry(30, seed=35)
    free = np.argwhere(occ == 0)
    rng = np.random.default_rng(seed_pose)
    for t, (u, v, w) in enumerate(odo):
        f.step_odometry(u, v, w)
        st = O.step(st, occ, p, u, v, w)
        if t % 10 == 9:
            j, i = free[rng.integers(len(free))]
            z = noisy_scan(occ, 0.1, ((i + 0.5) * 0.1, (j + 0.5) * 0.1, rng.uniform(-3, 3)), 90, 4.0, 0.1,
                           seed=t)
            _, _, th, ln_prior = f.read_belief(want_belief=False)
            prior_gpu = oracle_state_from(stored_belief(f), ln_prior, th)
            _last_prior[0], _last_scan[0] = prior_gpu, z
            zq = O.quantize_ranges(z, 4.0)
            f.apply_scan(z, sigma_scan)
            st = O.apply_scan(st, Rq, zq, sigma_scan, 4.0)
            yield t, f, st, O.apply_scan(prior_gpu, Rq, zq, sigma_scan, 4.0)


@pytest.mark.parametrize("f32_ops", [False, True])
def test_scan_update_matches_oracle_with_motion(f32_ops):
    # a broad likelihood (sigma 1.5 m): the posterior keeps hundreds of states
    # within 1e-3 of its peak, so the belief comparison is not one between two
    # delta functions
    for t, f, st, from_prior in _motion_and_scans(f32_ops, 1.5, 36):
        b, pose, _, ln = f.read_belief()
        err = peak_err(b, st.B)
        near_peak = int((st.B > 1e-3 * st.B.max()).sum())
        say(f"[scan] step {t} f32_ops={f32_ops} sigma 1.5: peak-normalised error {err:.3e}, {near_peak} states "
            f"above 1e-3 of the peak, log_norm {ln:.8f} vs {from_prior.log_norm:.8f} (oracle from the GPU prior) "
            f"and {st.log_norm:.8f} (oracle trajectory)")
        assert near_peak >= 100
        assert err <= SCAN_PEAK_TOL
        assert peak_err(b, from_prior.B) <= SCAN_PEAK_TOL
        assert in_tie_set(pose.as_tuple(), st.B, 1e-5)
        assert abs(ln - from_prior.log_norm) <= LN_ABS + LN_REL * abs(from_prior.log_norm)
        assert abs(ln - st.log_norm) <= LN_ABS + LN_REL * abs(st.log_norm)


@pytest.mark.parametrize("f32_ops", [False, True])
def test_sharp_scan_log_normaliser_from_the_gpu_prior(f32_ops):
    # sigma 0.1 m: the posterior collapses onto a few states whose prior may
    # be far below the prior's peak.  The log-normaliser is compared with the
    # oracle's scan of the exact FP32 prior the GPU holds (no extra term).
    for t, f, st, from_prior in _motion_and_scans(f32_ops, 0.1, 36):
        b, pose, _, ln = f.read_belief()
        say(f"[scan] step {t} f32_ops={f32_ops} sigma 0.1: log_norm {ln:.8f} vs {from_prior.log_norm:.8f} "
            f"(oracle from the GPU prior), peak-normalised error {peak_err(b, from_prior.B):.3e}")
        assert abs(ln - from_prior.log_norm) <= LN_ABS + LN_REL * abs(from_prior.log_norm)
        assert peak_err(b, from_prior.B) <= SCAN_PEAK_TOL
        assert in_tie_set(pose.as_tuple(), from_prior.B, 1e-5)


@pytest.mark.parametrize("sigma", [0.1, 0.3, 1.5])
def test_scan_posterior_against_the_continuous_range_model(sigma):
    # What the quantisation of ranges to h = max_range / 256 costs: the GPU
    # posterior (quantised model) against the oracle's per-beam Gaussian on
    # unquantised FP64 ranges, from the same FP32 prior.  Stated tolerance:
    # the same most probable state, and L1 <= 0.1 (the oracle's own quantised
    # and continuous posteriors differ by at most 0.045 on these scans).
    occ = bsp_rooms(64, 56, seed=34)
    R = range_table(occ, 0.1, 90, 4.0)
    for t, f, st, from_prior in _motion_and_scans(False, sigma, 36):
        b, pose, th, _ = f.read_belief()
        prior = _last_prior[0]
        cont = O.apply_scan_continuous(prior, R, _last_scan[0], sigma)
        l1 = float(np.abs(b.astype(np.float64) - cont.B).sum())
        best = np.unravel_index(int(np.argmax(cont.B)), cont.B.shape)
        say(f"[scan] step {t} sigma {sigma}: L1 to the continuous model {l1:.3e}, argmax {pose.as_tuple()} vs "
            f"{tuple(int(v) for v in best)}")
        assert l1 <= 0.1
        assert pose.as_tuple() == tuple(int(v) for v in best)


def test_noise_free_scan_peaks_at_the_true_state():
    occ = bsp_rooms(48, 40, seed=37)
    n_theta = 8
    R, m, f = _setup(occ, 0.1, 72, 3.0, n_theta)
    Rq = O.quantize_ranges(R, 3.0)
    s = O.beam_offsets(0.0, n_theta, 72)
    j, i, k = 17, 23, 5
    assert occ[j, i] == 0
    h = 3.0 / 256
    zq = np.array([Rq[j * 48 + i, (b + s[k]) % 72] for b in range(72)])
    z = ((zq + 128) * h).astype(np.float32)  # ranges that quantise back to zq exactly
    assert np.array_equal(O.quantize_ranges(z, 3.0), zq)
    f.apply_scan(z, 0.05)
    b, pose, _, _ = f.read_belief()
    D = O.scan_sqdist(Rq, zq, s).reshape(n_theta, 40, 48)
    assert D[pose.k, pose.j, pose.i] == 0
    assert b[k, j, i] == b.max()


def test_scan_errors():
    from paper_1910_00572_amd import mcl
    occ = bsp_rooms(32, 30, seed=38)
    _, f = make_gpu(occ, 0.1, 8, 0.5, 0.5)
    with pytest.raises(mcl.MclError) as ei:
        f.apply_scan(np.ones(16, np.float32), 0.1)
    assert ei.value.status == mcl.ESTATE
    R, m, g = _setup(occ, 0.1, 16, 2.0, 8)
    with pytest.raises(mcl.MclError) as ei:
        g.apply_scan(np.ones(15, np.float32), 0.1)
    assert ei.value.status == mcl.EINVAL
    with pytest.raises(mcl.MclError) as ei:
        g.apply_scan(np.ones(16, np.float32), 0.0)
    assert ei.value.status == mcl.EINVAL


def test_full_size_scan_ratios_match_oracle_distances():
    # 512x512x72 with 360 beams: the posterior ratio of any two states equals
    # the prior ratio times exp(-c (D_a - D_b)) with D from the oracle's direct
    # per-beam sum (sampled states, full-size launch shape).
    occ = rooms_and_corridors(512, 512, seed=3)
    poses, odo = smooth_trajectory(occ, 0.05, 10, seed=4)
    R, m, f = _setup(occ, 0.05, 360, 10.0, 72, sxy=1.0, sth=1.0)
    for u, v, w in odo:
        f.step_odometry(u, v, w)
    prior, _, th, _ = f.read_belief()
    z = noisy_scan(occ, 0.05, poses[-1], 360, 10.0, 0.1, seed=7)
    f.apply_scan(z, 0.1)
    post, pose, _, _ = f.read_belief()
    Rq = O.quantize_ranges(R, 10.0)
    zq = O.quantize_ranges(z, 10.0)
    s = O.beam_offsets(th, 72, 360)
    h = 10.0 / 256
    c = h * h / (2 * 0.1 ** 2)
    # reference state: the GPU posterior argmax; samples near it carry mass
    ref_cell = pose.j * 512 + pose.i
    rng = np.random.default_rng(39)
    flat_post = post.reshape(72, -1)
    flat_prior = prior.reshape(72, -1)
    cand = np.argwhere(flat_post > flat_post.max() * 1e-3)
    pick = cand[rng.choice(len(cand), min(300, len(cand)), replace=False)]
    cells = np.unique(np.concatenate([pick[:, 1], [ref_cell]]))
    D = O.scan_sqdist(Rq, zq, s, rows=cells)
    col = {cc: n for n, cc in enumerate(cells)}
    d_ref = D[pose.k, col[ref_cell]]
    for k, cell in pick:
        lhs = math.log(flat_post[k, cell]) - math.log(flat_post[pose.k, ref_cell])
        rhs = (math.log(flat_prior[k, cell]) - math.log(flat_prior[pose.k, ref_cell])
               - c * (D[k, col[cell]] - d_ref))
        assert lhs == pytest.approx(rhs, abs=2e-4)
