"""The full-circle step schedule (GPU only; through the C ABI).

When one workgroup holds every heading of its strip (one heading chunk), the
streaming step warps each channel once and takes the wrap-around of the
theta blur from reserved ring slots (Alg. 1's theta convolution is circular).
These cases sit on either side of the heading count that enables it, at
heading counts that leave the last channel group partly empty, at kernel
radii 2 to 4, with whole-cell shifts of up to six cells (so strips both with
and without row checks run) and a last strip of two rows.  The chunked
schedule recomputes its halo channels with the same arithmetic and the
stored belief is max-scaled, so the two schedules must store bitwise the
same belief in every storage type.
"""

import numpy as np
import pytest

from gen import bsp_rooms, random_odometry
from tests.gpu_harness import make_gpu, needs_gpu, say, stored_belief
from tests.test_gpu_parity import _run_pair

pytestmark = [pytest.mark.gpu, needs_gpu]

CIRCLE = (0, 4, 256, 1, 2, 1)   # 4-row strips, 4 waves, two slice buffers, one heading chunk
CHUNKED = (0, 4, 256, 2, 2, 1)  # the same kernel with two heading chunks


def _odometry(seed):
    # up to 0.6 m per step at 0.1 m cells, both signs
    return random_odometry(12, seed=seed, max_step_m=0.6) - np.array([0.3, 0.3, 0.0])


# (headings, sigma in cells and bins): the schedule needs 2R + 8 headings
CASES = [(13, 1.0), (14, 1.0), (15, 1.0), (17, 0.4), (30, 1.3), (37, 0.6)]


@pytest.mark.parametrize("n_theta,sigma", CASES, ids=lambda v: str(v))
def test_circle_schedule_matches_the_oracle(n_theta, sigma):
    occ = bsp_rooms(80, 62, seed=21)
    _run_pair(occ, 0.1, n_theta, sigma, sigma, _odometry(22 + n_theta), check_every=3,
              tag=f"circle T={n_theta} sigma={sigma}", launch_shape=CIRCLE)


@pytest.mark.parametrize("storage", ["f32", "bf16", "f16"])
def test_circle_schedule_stores_what_the_chunked_one_stores(storage):
    occ = bsp_rooms(80, 62, seed=23)
    _, circle = make_gpu(occ, 0.1, 30, 1.0, 1.0, storage=storage, launch_shape=CIRCLE)
    _, chunked = make_gpu(occ, 0.1, 30, 1.0, 1.0, storage=storage, launch_shape=CHUNKED)
    assert circle.info().workgroups * 2 == chunked.info().workgroups
    say(f"[circle] {storage}: full circle against two chunks")
    for t, (u, v, w) in enumerate(_odometry(24)):
        circle.step_odometry(u, v, w)
        chunked.step_odometry(u, v, w)
        if t % 4 == 3:
            a, b = stored_belief(circle), stored_belief(chunked)
            assert np.array_equal(a, b), f"step {t}: stored beliefs differ"
            ln = chunked.info().log_norm
            assert circle.info().log_norm == pytest.approx(ln, abs=1e-5 + 1e-6 * abs(ln))


def test_circle_schedule_in_a_batch_equals_single_steps():
    # the batched step kernels take the schedule per job: filters of several
    # heading counts and storage types stepped in shared launches store
    # bitwise what they store stepped alone
    from paper_1910_00572_amd import mcl
    occ = bsp_rooms(72, 58, seed=25)
    m = mcl.Map(occ, 0.1, 1.0)
    specs = [(14, "f32"), (30, "bf16"), (37, "f16"), (30, "f32")]
    solo = [mcl.Filter(m, t, 1.0, storage=st, launch_shape=CIRCLE) for t, st in specs]
    batch = [mcl.Filter(m, t, 1.0, storage=st, launch_shape=CIRCLE) for t, st in specs]
    ws = mcl.BatchWorkspace(len(specs))
    odo = [_odometry(26 + i) for i in range(len(specs))]
    say("[circle] batch against single steps")
    for t in range(12):
        for i, f in enumerate(solo):
            f.step_odometry(*odo[i][t])
        mcl.step_batch(batch, np.stack([o[t] for o in odo]), ws)
    for a, b in zip(solo, batch):
        assert np.array_equal(stored_belief(a), stored_belief(b))
        assert a.info().log_norm == b.info().log_norm


def test_circle_schedule_with_jumps_past_the_halo():
    # 30-cell jumps up and down the map: slices whose first source row lies
    # past the last grid row (an empty descriptor in the unchecked loop) and
    # far above the first (the checked loop), against the oracle
    occ = bsp_rooms(80, 62, seed=27)
    odo = np.array([[0.0, 3.0, 0.1], [0.2, -3.0, -0.2], [-3.0, 0.4, 0.3], [3.1, 0.0, 0.0],
                    [0.0, 2.6, 0.5], [0.1, -2.9, 0.0]])
    _run_pair(occ, 0.1, 30, 1.0, 1.0, odo, tag="circle jumps", launch_shape=CIRCLE)
