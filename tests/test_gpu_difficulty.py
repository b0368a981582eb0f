"""Map difficulty on the GPU vs the FP64 oracle (GPU only; through the C ABI).

The best match of a query scan is an exact integer search (squared distances
of quantised ranges, exact MFMA sums, lowest flat index k * H * W + q on
ties), so cell, heading and distance are compared bit for bit, for BF16 and
FP32 matrix operands and for every table depth the kernel is built for.  At
the full shape (128 x 128 cells, 360 directions, 72 channels) the oracle's
whole search runs for a sample of the queries; every other query is checked
by properties that fix a best match: its distance is the exact distance of
the state returned, the state is free, and no cheaper state is known (the
query's own cell at heading 0).
"""

import numpy as np
import pytest

import oracle as O
from gen import bsp_rooms, cell_scans, range_table, rooms_and_corridors
from tests.gpu_harness import make_gpu, needs_gpu, say

pytestmark = [pytest.mark.gpu, needs_gpu]


def _map(occ, cell, n_dirs, max_range, flags=3):
    from paper_1910_00572_amd import mcl
    R = range_table(occ, cell, n_dirs, max_range)
    m = mcl.Map(occ, cell, 0.7, flags=flags, range_table=R, max_range_m=max_range)
    return R, m


def _queries(occ, R, max_range, rng, n_noisy, n_clean, n_wall, n_random, seed):
    free = np.flatnonzero(occ.reshape(-1) == 0)
    wall = np.flatnonzero(occ.reshape(-1) != 0)
    cells = list(rng.choice(free, n_noisy + n_clean, replace=False))
    z = [cell_scans(R, cells[:n_noisy], 0.05, max_range, seed),
         cell_scans(R, cells[n_noisy:], 0.0, max_range, seed + 1),
         cell_scans(R, rng.choice(wall, n_wall, replace=False), 0.0, max_range, seed + 2),
         rng.uniform(0.0, max_range * 1.05, (n_random, R.shape[1])).astype(np.float32)]
    return np.concatenate(z)


@pytest.mark.parametrize("f32_ops", [False, True])
def test_best_match_is_exact_small(f32_ops):
    from paper_1910_00572_amd import mcl
    occ = bsp_rooms(40, 33, seed=41)
    R, m = _map(occ, 0.1, 64, 3.0, flags=3 | (8 if f32_ops else 0))
    rng = np.random.default_rng(42)
    z = _queries(occ, R, 3.0, rng, 10, 3, 2, 2, seed=43)  # 17 queries, batches of 4: ragged last batch
    say(f"[difficulty] exact small f32_ops={f32_ops}")
    cell, head, dist = mcl.best_match(m, 12, z, batch=4)
    Rq = O.quantize_ranges(R, 3.0)
    free = occ.reshape(-1) == 0
    for p in range(len(z)):
        ref = O.best_match(Rq, O.quantize_ranges(z[p], 3.0), 12, free)
        assert (int(cell[p]), int(head[p]), int(dist[p])) == ref, p


@pytest.mark.parametrize("n_dirs,n_theta", [(100, 7), (200, 5), (300, 3), (360, 9)])
def test_best_match_every_table_depth(n_dirs, n_theta):
    # depths 128, 256, 320 and 384; an odd channel count leaves part of a 32-column block empty
    from paper_1910_00572_amd import mcl
    occ = bsp_rooms(24, 20, seed=44)
    R, m = _map(occ, 0.15, n_dirs, 4.0)
    rng = np.random.default_rng(45)
    z = _queries(occ, R, 4.0, rng, 4, 1, 1, 1, seed=46)
    say(f"[difficulty] depth n_dirs={n_dirs} n_theta={n_theta}")
    cell, head, dist = mcl.best_match(m, n_theta, z, batch=3)
    Rq = O.quantize_ranges(R, 4.0)
    free = occ.reshape(-1) == 0
    for p in range(len(z)):
        ref = O.best_match(Rq, O.quantize_ranges(z[p], 4.0), n_theta, free)
        assert (int(cell[p]), int(head[p]), int(dist[p])) == ref, p


def test_best_match_full_shape():
    # 128 x 128 cells, 360 directions, 72 channels, one batch of 64 queries (4608 columns)
    from paper_1910_00572_amd import mcl
    occ = rooms_and_corridors(128, 128, seed=47)
    R, m = _map(occ, 0.05, 360, 10.0)
    free = occ.reshape(-1) == 0
    rng = np.random.default_rng(48)
    qcells = rng.choice(np.flatnonzero(free), 64, replace=False)
    z = cell_scans(R, qcells, 0.1, 10.0, seed=49)
    say("[difficulty] full shape")
    cell, head, dist = mcl.best_match(m, 72, z, batch=64)
    Rq = O.quantize_ranges(R, 10.0)
    zq = O.quantize_ranges(z, 10.0)
    s = O.beam_offsets(0.0, 72, 360)
    for p in range(64):
        assert free[cell[p]] and 0 <= head[p] < 72
        d_ret = O.scan_sqdist(Rq, zq[p], s[head[p]:head[p] + 1], rows=[cell[p]])[0, 0]
        d_own = O.scan_sqdist(Rq, zq[p], s[:1], rows=[qcells[p]])[0, 0]
        assert dist[p] == d_ret and dist[p] <= d_own, p
    for p in rng.choice(64, 3, replace=False):
        assert (int(cell[p]), int(head[p]), int(dist[p])) == O.best_match(Rq, zq[p], 72, free), p


def test_difficulty_matches_oracle():
    from paper_1910_00572_amd import mcl
    occ = bsp_rooms(40, 33, seed=50)
    R, m = _map(occ, 0.1, 64, 3.0)
    free = np.flatnonzero(occ.reshape(-1) == 0)
    qcells = free[::5]
    z = cell_scans(R, qcells, 0.15, 3.0, seed=51)
    say("[difficulty] D_M")
    cell, _, _ = mcl.best_match(m, 8, z)
    for thr in (0.0, 0.1, 0.25, 1.0):
        assert mcl.difficulty(m, qcells, cell, thr) == O.difficulty(cell, qcells, 40, 0.1, thr)
    assert mcl.difficulty(m, [], [], 1.0) == 0.0
    assert mcl.difficulty(m, [qcells[0]], [-1], 1.0) == 1.0


def test_best_match_edge_cases():
    from paper_1910_00572_amd import mcl
    occ = bsp_rooms(24, 20, seed=52)
    R, m = _map(occ, 0.15, 64, 4.0)
    say("[difficulty] edge cases")
    cell, head, dist = mcl.best_match(m, 4, np.zeros((0, 64), np.float32))
    assert len(cell) == len(head) == len(dist) == 0
    z = cell_scans(R, [int(np.flatnonzero(occ.reshape(-1) == 0)[0])], 0.0, 4.0, seed=53)
    for bad in (0, 361):
        with pytest.raises(mcl.MclError) as e:
            mcl.best_match(m, bad, z)
        assert e.value.status == mcl.EINVAL
    with pytest.raises(mcl.MclError) as e:
        mcl.best_match(m, 4, z[:, :63])  # one direction short of the table
    assert e.value.status == mcl.EINVAL
    zn = z.copy()
    zn[0, 5] = np.nan
    with pytest.raises(mcl.MclError) as e:
        mcl.best_match(m, 4, zn)
    assert e.value.status == mcl.EINVAL
    lib = mcl.load_library()
    need = lib.mcl_match_workspace_bytes(m.handle, 4, 8)
    assert need > 0
    import torch
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    out = np.empty(1, np.int32)
    st = lib.mcl_best_match(m.handle, 4, z.ctypes.data, 1, 8, out.ctypes.data, None, None, ws.data_ptr(),
                            need - 1, None)
    assert st == mcl.ENOMEM
    st = lib.mcl_best_match(m.handle, 4, z.ctypes.data, 1, 8, out.ctypes.data, None, None, ws.data_ptr(),
                            need, None)
    assert st == mcl.OK and out[0] == mcl.best_match(m, 4, z)[0][0]
    # no range table
    m2, _ = make_gpu(occ, 0.15, 4, 0.7, 0.7)
    assert lib.mcl_match_workspace_bytes(m2.handle, 4, 8) == 0
    st = lib.mcl_best_match(m2.handle, 4, z.ctypes.data, 1, 8, out.ctypes.data, None, None, ws.data_ptr(),
                            need, None)
    assert st == mcl.ESTATE
    # the batch size changes nothing: one query per batch, or every query in one batch
    rng = np.random.default_rng(54)
    zz = _queries(occ, R, 4.0, rng, 3, 1, 1, 0, seed=55)
    one = mcl.best_match(m, 6, zz, batch=1)
    allq = mcl.best_match(m, 6, zz, batch=64)
    for x, y in zip(one, allq):
        assert np.array_equal(x, y)
    # a map with no free cell: no candidate at all
    full = np.ones((20, 24), np.uint8)
    _, m3 = _map(full, 0.15, 64, 4.0)
    cell, head, dist = mcl.best_match(m3, 4, z)
    assert cell[0] == -1 and head[0] == -1 and dist[0] == -1
