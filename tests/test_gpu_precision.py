"""Reduced-precision storage (BF16 / FP16) against the FP64 oracle (GPU only).

Bound: L1 = sum |B_gpu - B_oracle| <= 1e-2 on sum-normalised beliefs and the
GPU argmax inside the oracle's tie set {B >= max (1 - 2^-7)} (2^-7 is half a
BF16 unit in the last place).  Arithmetic is FP32 in every case; only the
stored belief is rounded (round to nearest even) after each step, with the
lazy max-scaling keeping the stored peak near one.
"""

import numpy as np
import pytest

import oracle as O
from gen import bsp_rooms, random_odometry, rooms_and_corridors, smooth_trajectory
from tests.gpu_harness import in_tie_set, l1_err, make_gpu, needs_gpu, oracle_params, peak_err, say, stored_belief

pytestmark = [pytest.mark.gpu, needs_gpu]

L1_TOL = 1e-2
TIE_TAU = 2.0 ** -7


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_reduced_precision_long_run(storage):
    occ = rooms_and_corridors(128, 128, seed=41)
    poses, odo = smooth_trajectory(occ, 0.05, 200, seed=42)
    n_theta = 32
    p = oracle_params(n_theta, 0.05, 1.0, 1.0)
    _, f = make_gpu(occ, 0.05, n_theta, 1.0, 1.0, storage=storage)
    st = O.init_uniform(occ, n_theta)
    M = O.free_mask(occ)
    worst = 0.0
    for t, (u, v, w) in enumerate(odo):
        f.step_odometry(u, v, w)
        st = O.step(st, occ, p, u, v, w, M=M)
        if t % 20 == 19:
            b, pose, _, ln = f.read_belief()
            l1 = l1_err(b, st.B)
            worst = max(worst, l1)
            assert l1 <= L1_TOL, f"{storage} step {t}: L1 {l1:.3e}"
            assert in_tie_set(pose.as_tuple(), st.B, TIE_TAU), f"{storage} step {t}: argmax {pose.as_tuple()}"
            assert abs(ln - st.log_norm) < 1e-2
    say(f"[precision] {storage} worst L1 over 200 steps {worst:.3e}")


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_reduced_precision_anisotropic(storage):
    # the anisotropic two-pass step stores the belief in 16 bits as well
    occ = bsp_rooms(72, 60, seed=45)
    odo = random_odometry(40, seed=46, max_step_m=0.12)
    n_theta = 24
    p = oracle_params(n_theta, 0.1, 1.1, 0.8, flags=3 | 32, sigma_lateral=0.5)
    _, f = make_gpu(occ, 0.1, n_theta, 1.1, 0.8, flags=3 | 32, sigma_lateral=0.5, storage=storage)
    st = O.init_uniform(occ, n_theta)
    M = O.free_mask(occ)
    worst = 0.0
    for t, (u, v, w) in enumerate(odo):
        f.step_odometry(u, v, w)
        st = O.step(st, occ, p, u, v, w, M=M)
        if t % 10 == 9:
            b, pose, _, ln = f.read_belief()
            l1 = l1_err(b, st.B)
            worst = max(worst, l1)
            assert l1 <= L1_TOL, f"{storage} step {t}: L1 {l1:.3e}"
            assert in_tie_set(pose.as_tuple(), st.B, TIE_TAU), f"{storage} step {t}: argmax {pose.as_tuple()}"
            assert abs(ln - st.log_norm) < 1e-2
    say(f"[precision] anisotropic {storage} worst L1 over 40 steps {worst:.3e}")


def test_fp16_normalize_keeps_range():
    # FP16 cannot hold a sum-one belief of 16k states; normalize peaks it at one
    occ = bsp_rooms(64, 64, seed=43)
    _, f = make_gpu(occ, 0.1, 16, 0.5, 0.5, storage="f16")
    for u, v, w in random_odometry(5, seed=44):
        f.step_odometry(u, v, w)
    before, _, _, ln0 = f.read_belief()
    ln = f.normalize()
    after, _, _, ln1 = f.read_belief()
    assert ln == pytest.approx(ln0, abs=1e-6) and ln1 == pytest.approx(ln0, abs=1e-6)
    assert np.abs(after.astype(np.float64) - before).sum() < 1e-3


def test_full_size_mixed_precision_one_step_and_argmax_agreement():
    # 1024x1024 map, 128 bins (134M states).  FP32 storage: one oracle step from
    # the GPU's own belief at the launch shape the benchmark uses.  BF16 vs FP32
    # on the GPU over 500 steps: argmax of BF16 inside the FP32 tie set.
    occ = rooms_and_corridors(1024, 1024, seed=5)
    _, odo = smooth_trajectory(occ, 0.05, 500, seed=6)
    p = oracle_params(128, 0.05, 1.0, 1.0)
    m, f32 = make_gpu(occ, 0.05, 128, 1.0, 1.0, storage="f32")
    from paper_1910_00572_amd import mcl
    bf = mcl.Filter(m, 128, 1.0, storage="bf16")
    agree = 0
    checks = 0
    for t in range(499):
        f32.step_odometry(*odo[t])
        bf.step_odometry(*odo[t])
        if t % 50 == 49:
            _, pa, _, _ = f32.read_belief(want_belief=False)
            b16, pb, _, _ = bf.read_belief()
            b32 = f32.export_belief().cpu().numpy().astype(np.float64)
            checks += 1
            agree += int(in_tie_set(pb.as_tuple(), b32, TIE_TAU))
            l1 = float(np.abs(b16 - b32).sum())
            say(f"[precision] full size step {t}: BF16 vs FP32 L1 {l1:.3e}")
            assert l1 <= L1_TOL
    assert agree == checks
    b, _, th, _ = f32.read_belief()
    st = O.FilterState(B=b.astype(np.float64) / b.sum(dtype=np.float64), theta=th)
    say("[precision] oracle step at 1024x1024x128")
    ref = O.step(st, occ, p, *odo[499])
    f32.step_odometry(*odo[499])
    b2, pose, _, _ = f32.read_belief()
    err = peak_err(b2, ref.B)
    say(f"[precision] full size FP32 one-step peak-normalised error {err:.3e}")
    assert err <= 1e-5
    assert in_tie_set(pose.as_tuple(), ref.B, 1e-6)


@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_reduced_precision_resume_of_a_sum_one_belief(storage):
    # 300 x 300 cells x 256 headings: a sum-one belief of 23 M states holds
    # values near 4e-8, below FP16's smallest subnormal (6e-8).  Resuming a
    # 16-bit filter from such an export must keep it (the upload stores the
    # belief max-scaled, as every step does), to the 16-bit storage's
    # precision: L1 <= 1e-2 and the argmax in the tie set.
    occ = bsp_rooms(300, 300, seed=47)
    odo = random_odometry(3, seed=48)
    _, f = make_gpu(occ, 0.1, 256, 0.7, 0.7)
    for u, v, w in odo:
        f.step_odometry(u, v, w)
    b, _, th, _ = f.read_belief()
    assert np.median(b[b > 0]) < 6e-8
    _, g = make_gpu(occ, 0.1, 256, 0.7, 0.7, storage=storage, init=b, theta0=th)
    b2, pose, th2, ln2 = g.read_belief()
    ref = b.astype(np.float64)
    l1 = float(np.abs(b2.astype(np.float64) - ref).sum())
    say(f"[precision] {storage} resume of a sum-one FP32 export: L1 {l1:.3e}")
    assert l1 <= L1_TOL
    assert in_tie_set(pose.as_tuple(), ref, TIE_TAU)
    assert th2 == th and ln2 == 0.0


def test_reduced_precision_at_the_large_map_shapes():
    # BF16 and FP16 storage through the launch shapes large maps use (16-row
    # strips, 8 waves, one slice buffer, 4-byte strip alignment; and 8-row
    # strips), 128 heading bins, 200 steps against the FP64 oracle: L1 <= 1e-2
    # and the argmax in the tie set at every 20th step.
    occ = rooms_and_corridors(128, 128, seed=49)
    _, odo = smooth_trajectory(occ, 0.05, 200, seed=50)
    n_theta = 128
    p = oracle_params(n_theta, 0.05, 1.0, 1.0)
    from paper_1910_00572_amd import mcl
    m = mcl.Map(occ, 0.05, 1.0)
    shapes = [(0, 16, 512, 1, 1, 0, 4), (0, 8, 512, 1, 1, 0, 4)]
    gpu = {(st, sh): mcl.Filter(m, n_theta, 1.0, storage=st, launch_shape=sh)
           for st in ("bf16", "f16") for sh in shapes}
    st_o = O.init_uniform(occ, n_theta)
    M = O.free_mask(occ)
    worst = {k: 0.0 for k in gpu}
    for t, (u, v, w) in enumerate(odo):
        for f in gpu.values():
            f.step_odometry(u, v, w)
        st_o = O.step(st_o, occ, p, u, v, w, M=M)
        if t % 20 == 19:
            for key, f in gpu.items():
                b, pose, _, ln = f.read_belief()
                l1 = l1_err(b, st_o.B)
                worst[key] = max(worst[key], l1)
                assert l1 <= L1_TOL, f"{key} step {t}: L1 {l1:.3e}"
                assert in_tie_set(pose.as_tuple(), st_o.B, TIE_TAU), f"{key} step {t}: argmax {pose.as_tuple()}"
                assert abs(ln - st_o.log_norm) < 1e-2
    for key, wv in worst.items():
        say(f"[precision] {key}: worst L1 over 200 steps {wv:.3e}")


@pytest.mark.parametrize("sigma", [0.3, 0.6, 1.3], ids=lambda s: f"sigma{s}")
@pytest.mark.parametrize("storage", ["bf16", "f16"])
def test_reduced_precision_large_map_shape_at_every_radius(storage, sigma):
    # the large-map launch shape (16-row strips, 8 waves, one slice buffer)
    # in 16-bit storage runs its blurs in forms of its own (x blur summed
    # towards the centre, centre taps scaled to one); kernel radii 1, 2 and
    # 4 in x, y and theta, 40 steps against the FP64 oracle; the batched
    # kernel of the same shape stores bitwise what the single one stores
    from paper_1910_00572_amd import mcl
    occ = bsp_rooms(96, 80, seed=61)
    odo = random_odometry(40, seed=62, max_step_m=0.25) - np.array([0.12, 0.12, 0.0])
    n_theta = 24
    shape = (0, 16, 512, 1, 1, 0, 4)
    p = oracle_params(n_theta, 0.1, sigma, sigma)
    m, f = make_gpu(occ, 0.1, n_theta, sigma, sigma, storage=storage, launch_shape=shape)
    fb = mcl.Filter(m, n_theta, sigma, storage=storage, launch_shape=shape)
    ws = mcl.BatchWorkspace(1)
    st = O.init_uniform(occ, n_theta)
    M = O.free_mask(occ)
    say(f"[precision] large-map shape, {storage}, sigma {sigma}")
    for t, (u, v, w) in enumerate(odo):
        f.step_odometry(u, v, w)
        mcl.step_batch([fb], np.array([[u, v, w]]), ws)
        st = O.step(st, occ, p, u, v, w, M=M)
        if t % 10 == 9:
            b, pose, _, ln = f.read_belief()
            l1 = l1_err(b, st.B)
            assert l1 <= L1_TOL, f"step {t}: L1 {l1:.3e}"
            assert in_tie_set(pose.as_tuple(), st.B, TIE_TAU), f"step {t}: argmax {pose.as_tuple()}"
            assert abs(ln - st.log_norm) < 1e-2
    assert np.array_equal(stored_belief(f), stored_belief(fb))
    assert f.info().log_norm == fb.info().log_norm
