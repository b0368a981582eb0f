"""MI355X-native dense belief-tensor localization filter (arXiv 1910.00572).

The hot path lives in libmcl.so (HIP for gfx950, C ABI in include/mcl.h);
`paper_1910_00572_amd.mcl` is its Python binding.
"""

from .mcl import (  # noqa: F401
    Map, Filter, MclError, init_belief, step_odometry, apply_scan, normalize, read_belief, step_batch,
    load_library, ABI_SYMBOLS, BatchWorkspace,
)
