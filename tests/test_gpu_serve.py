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
        # the server takes the pose from the exported belief (lowest flat index wins ties)
        assert got.pose == tuple(int(v) for v in np.unravel_index(int(np.argmax(b)), b.shape))
        assert got.log_norm == ln and got.degenerate == degen
    assert stats["graph_replays"] >= stats["iterations"] and stats["graph_captures"] < stats["iterations"]


def test_graph_batch_is_bitwise_identical_to_single_steps():
    # the graph-replayed batch: the same filters stepped alone and through
    # mcl_batch_step, with a filter leaving and one joining half way (a new
    # launch structure, captured once and then replayed)
    import torch
    from paper_1910_00572_amd import mcl
    maps = _maps(with_scan=False)
    specs = [(48, 8, "f32"), (64, 12, "bf16"), (80, 6, "f32"), (64, 16, "f16"), (48, 10, "bf16"), (80, 9, "f32")]
    solo = [mcl.Filter(maps[g][1], t, 0.7, storage=s) for g, t, s in specs]
    stream = torch.cuda.Stream()  # graphs are not captured on the default stream
    with pytest.raises(mcl.MclError):
        mcl.BatchRunner(len(specs), stream=torch.cuda.default_stream())
    batch = [mcl.Filter(maps[g][1], t, 0.7, storage=s, stream=stream) for g, t, s in specs]
    runner = mcl.BatchRunner(len(specs), stream=stream)
    odo = [random_odometry(16, seed=90 + i) for i in range(len(specs))]
    say("[serve] graph batch vs single")
    for t in range(16):
        members = list(range(5)) if t < 8 else [0, 2, 3, 4, 5]  # filter 1 leaves, filter 5 joins
        for i in members:
            solo[i].step_odometry(*odo[i][t])
        runner.step([batch[i] for i in members], np.stack([odo[i][t] for i in members]))
    torch.cuda.synchronize()
    for a, b in zip(solo, batch):
        assert np.array_equal(a.export_belief().cpu().numpy(), b.export_belief().cpu().numpy())
        assert a.info().log_norm == b.info().log_norm
    captures, replays = runner.counts()
    say(f"[serve] graph captures {captures}, replays {replays}")
    assert replays == 16 and captures <= 4


def test_scan_batch_is_bitwise_identical_to_single_scans():
    # the scans of several filters of one map in shared launches: each filter
    # ends bitwise where mcl_apply_scan leaves it, for BF16 and FP32 matrix
    # operands, mixed storage types and heading counts
    from paper_1910_00572_amd import mcl
    for f32_ops in (False, True):
        occ = bsp_rooms(64, 56, seed=95)
        R = range_table(occ, 0.1, 90, 4.0)
        flags = mcl.DEFAULT_FLAGS | (mcl.SCAN_F32 if f32_ops else 0)
        m = mcl.Map(occ, 0.1, 0.7, range_table=R, max_range_m=4.0, flags=flags)
        specs = [(16, "f32"), (16, "f32"), (24, "bf16"), (16, "f16"), (24, "bf16"), (40, "f32")]
        solo = [mcl.Filter(m, t, 0.7, storage=s) for t, s in specs]
        batch = [mcl.Filter(m, t, 0.7, storage=s) for t, s in specs]
        free = np.argwhere(occ == 0)
        rng = np.random.default_rng(96)
        for step in range(12):
            uvw = np.stack([random_odometry(12, seed=97 + i)[step] for i in range(len(specs))])
            for f, o in zip(solo + batch, np.concatenate([uvw, uvw])):
                f.step_odometry(*o)
            if step % 4 == 3:
                zs = []
                for i in range(len(specs)):
                    j, x = free[rng.integers(len(free))]
                    zs.append(noisy_scan(occ, 0.1, ((x + 0.5) * 0.1, (j + 0.5) * 0.1, 0.5), 90, 4.0, 0.1,
                                         seed=step * 10 + i))
                sig = [0.1, 0.2, 0.1, 0.3, 0.15, 0.1]
                for f, z, sg in zip(solo, zs, sig):
                    f.apply_scan(z, sg)
                mcl.apply_scan_batch(batch, np.stack(zs), sig)
        say(f"[serve] scan batch vs single, f32_ops={f32_ops}")
        for a, b in zip(solo, batch):
            assert np.array_equal(a.export_belief().cpu().numpy(), b.export_belief().cpu().numpy())
            assert a.info().log_norm == b.info().log_norm


def test_scan_batch_rejects_mixed_maps():
    from paper_1910_00572_amd import mcl
    maps = _maps()
    a = mcl.Filter(maps[48][1], 8, 0.7)
    b = mcl.Filter(maps[64][1], 8, 0.7)
    with pytest.raises(mcl.MclError) as ei:
        mcl.apply_scan_batch([a, b], np.ones((2, 60), np.float32), 0.1)
    assert ei.value.status == mcl.EINVAL
