"""The allocation-free batched step against mcl_step_batch (GPU only; through the C ABI).

mcl_step_batch_noalloc keeps its job table in the library's static device
array instead of a caller workspace.  Two calls in a row, the second with
fewer filters (the array keeps the first call's contents): every filter must
end bitwise where the same filter stepped by mcl_step_batch ends.
"""

import numpy as np
import pytest

from gen import bsp_rooms, random_odometry
from tests.gpu_harness import needs_gpu, say

pytestmark = [pytest.mark.gpu, needs_gpu]


def test_noalloc_batch_equals_the_workspace_batch():
    from paper_1910_00572_amd import mcl
    maps = {s: mcl.Map(bsp_rooms(s, s, seed=120 + s), 0.1, 0.8) for s in (48, 64, 80)}
    specs = [(48, 8, "f32"), (64, 12, "bf16"), (80, 6, "f32"), (64, 16, "f16"), (48, 10, "bf16"), (80, 72, "f32")]
    ref = [mcl.Filter(maps[g], t, 0.7, storage=s) for g, t, s in specs]
    got = [mcl.Filter(maps[g], t, 0.7, storage=s) for g, t, s in specs]
    ws = mcl.BatchWorkspace(len(specs))
    odo = np.stack([random_odometry(2, seed=130 + i) for i in range(len(specs))])  # (filters, steps, 3)
    for call, members in enumerate((list(range(6)), [1, 3, 5])):  # the second call: fewer filters
        say(f"[noalloc] call {call}: {len(members)} filters")
        uvw = odo[members, call]
        mcl.step_batch([ref[i] for i in members], uvw, ws)
        mcl.step_batch_noalloc([got[i] for i in members], uvw)
        for i in members:
            a = ref[i].export_belief().cpu().numpy()
            b = got[i].export_belief().cpu().numpy()
            assert np.array_equal(a, b), f"call {call}, filter {i}"
            assert ref[i].info().log_norm == got[i].info().log_norm


def test_noalloc_batch_rejects_more_filters_than_its_table_holds():
    from paper_1910_00572_amd import mcl
    m = mcl.Map(bsp_rooms(32, 32, seed=140), 0.1, 0.8)
    fs = [mcl.Filter(m, 4, 0.7) for _ in range(257)]
    with pytest.raises(mcl.MclError) as ei:
        mcl.step_batch_noalloc(fs, np.zeros((257, 3)))
    assert ei.value.status == mcl.EINVAL
    assert "at most 256" in str(ei.value)
