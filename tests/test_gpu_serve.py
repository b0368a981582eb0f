"""Batched stepping and the continuous-batching server (GPU only; through the C ABI).

Every filter stepped in a batch, or served in a mix of requests that arrive
while others run, must give bitwise the same belief as the same filter run
alone; the server must respect its HBM budget.
"""

import numpy as np
import pytest

from gen import bsp_rooms, noisy_scan, random_odometry, range_table
from tests.gpu_harness import needs_gpu, say

pytestmark = [pytest.mark.gpu, needs_gpu]


def _maps(with_scan=True):
    from paper_1910_00572_amd import mcl
    maps = {}
    for n, size in enumerate((48, 64, 80)):
        occ = bsp_rooms(size, size, seed=50 + n)
        R = range_table(occ, 0.1, 60, 3.0) if with_scan else None
        maps[size] = (occ, mcl.Map(occ, 0.1, 0.8, range_table=R, max_range_m=3.0))
    return maps


def test_step_batch_is_bitwise_identical_to_single_steps():
    from paper_1910_00572_amd import mcl
    maps = _maps(with_scan=False)
    specs = [(48, 8, "f32"), (64, 12, "bf16"), (80, 6, "f32"), (64, 16, "f16"), (48, 10, "bf16")]
    solo = [mcl.Filter(maps[g][1], t, 0.7, storage=s) for g, t, s in specs]
    batch = [mcl.Filter(maps[g][1], t, 0.7, storage=s) for g, t, s in specs]
    ws = mcl.BatchWorkspace(len(specs))
    odo = [random_odometry(12, seed=60 + i) for i in range(len(specs))]
    say("[serve] step_batch vs single")
    for t in range(12):
        for i, f in enumerate(solo):
            f.step_odometry(*odo[i][t])
        mcl.step_batch(batch, np.stack([o[t] for o in odo]), ws)
    for a, b in zip(solo, batch):
        ea = a.export_belief().cpu().numpy()
        eb = b.export_belief().cpu().numpy()
        assert np.array_equal(ea, eb)
        assert a.info().log_norm == b.info().log_norm


def test_step_batch_with_gate_and_whole_cell_warp():
    # filters whose maps use the sub-cell gate and the whole-cell warp with a
    # carried remainder: the batch keeps each filter's host state, so the
    # result is bitwise that of stepping alone (some filters skip launches)
    from paper_1910_00572_amd import mcl
    occs = [bsp_rooms(size, size, seed=70 + n) for n, size in enumerate((40, 56))]
    flags = [mcl.DEFAULT_FLAGS | mcl.INTEGER_SHIFT, mcl.DEFAULT_FLAGS | mcl.INTEGER_SHIFT | mcl.SUBCELL_GATE]
    maps = [mcl.Map(o, 0.1, 0.7, flags=fl) for o in occs for fl in flags]
    solo = [mcl.Filter(m, 8 + 2 * i, 0.7, storage="f32") for i, m in enumerate(maps)]
    batch = [mcl.Filter(m, 8 + 2 * i, 0.7, storage="f32") for i, m in enumerate(maps)]
    ws = mcl.BatchWorkspace(len(maps))
    odo = [random_odometry(15, seed=80 + i, max_step_m=0.06) for i in range(len(maps))]
    say("[serve] step_batch vs single, whole-cell warp")
    for t in range(15):
        for i, f in enumerate(solo):
            f.step_odometry(*odo[i][t])
        mcl.step_batch(batch, np.stack([o[t] for o in odo]), ws)
    for a, b in zip(solo, batch):
        assert np.array_equal(a.export_belief().cpu().numpy(), b.export_belief().cpu().numpy())
        assert a.info().log_norm == b.info().log_norm


def test_server_mix_equals_alone_and_respects_budget():
    from paper_1910_00572_amd import mcl
    from paper_1910_00572_amd.serve import Request, Server, run_alone
    maps = _maps()
    mp = {k: v[1] for k, v in maps.items()}
    rng = np.random.default_rng(70)
    reqs = []
    for rid in range(10):
        g = int(rng.choice([48, 64, 80]))
        n_theta = int(rng.choice([8, 12]))
        storage = str(rng.choice(["f32", "bf16"]))
        steps = int(rng.integers(15, 31))
        odo = random_odometry(steps, seed=100 + rid)
        scans = {}
        if rid % 2 == 0:
            occ = maps[g][0]
            free = np.argwhere(occ == 0)
            for t in range(9, steps, 10):
                j, i = free[rng.integers(len(free))]
                scans[t] = noisy_scan(occ, 0.1, ((i + 0.5) * 0.1, (j + 0.5) * 0.1, 0.3), 60, 3.0, 0.1, seed=rid * 100 + t)
        if rid == 3:
            odo[steps // 2] = (100.0 * 0.1, 0.0, 0.0)  # a 100-cell jump: all mass leaves the grid
        reqs.append(Request(rid, float(rng.uniform(0, 0.05)), g, n_theta, storage, odo, scans, sigma_theta=0.7))
    # budget: about three of the largest filters at once
    probe = Server(mp, 1 << 40)
    need = max(probe._workspace_bytes(r) for r in reqs)
    server = Server(mp, 3 * need, max_active=8, keep_beliefs=True)
    say("[serve] server mix")
    results, stats = server.run(reqs)
    assert stats["peak_bytes"] <= 3 * need
    assert stats["peak_active"] >= 2  # work overlapped
    assert len(results) == len(reqs)
    assert stats["degenerate_requests"] == 1 and results[3].degenerate
    for r in reqs:
        b, pose, ln, degen = run_alone(mp, r)
        got = results[r.rid]
        assert np.array_equal(got.belief, b), f"request {r.rid}"
        assert got.pose == pose and got.log_norm == ln and got.degenerate == degen
