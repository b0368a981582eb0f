"""FP64 CPU oracle of the belief-tensor localization filter.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute anything in this package: only the test suite, the smoke check and
the benchmark's CPU-baseline leg use it.  It shares no code with the HIP
library (no kernels, headers, helpers or tables); both sides only consume the
same seeded inputs from `gen`.

Plain, slow and written to be checked against the paper by eye: separate
passes in the order of Alg. 1, float64 throughout, no fusion or blocking.
"""

from .filter import (
    FilterState,
    OracleParams,
    gaussian_taps,
    rotated_taps,
    conv2d,
    default_radius,
    free_mask,
    kernel_activation,
    wall_weights,
    init_uniform,
    slice_displacements,
    integer_shifts,
    shift_bilinear,
    blur_x,
    blur_y,
    blur_theta,
    step,
    run,
    belief_map,
    argmax_pose,
)
from .scan import quantize_ranges, beam_offsets, scan_sqdist, apply_scan, scan_sqdist_continuous, apply_scan_continuous
from .difficulty import best_match, difficulty
from .sample import dither_intensity, floyd_steinberg, floyd_steinberg_c, sample_mask, apply_scan_sampled

__all__ = [
    "FilterState",
    "OracleParams",
    "gaussian_taps",
    "rotated_taps",
    "conv2d",
    "default_radius",
    "free_mask",
    "kernel_activation",
    "wall_weights",
    "init_uniform",
    "slice_displacements",
    "integer_shifts",
    "shift_bilinear",
    "blur_x",
    "blur_y",
    "blur_theta",
    "step",
    "run",
    "belief_map",
    "argmax_pose",
    "quantize_ranges",
    "beam_offsets",
    "scan_sqdist",
    "apply_scan",
    "scan_sqdist_continuous",
    "apply_scan_continuous",
    "dither_intensity",
    "floyd_steinberg",
    "floyd_steinberg_c",
    "sample_mask",
    "apply_scan_sampled",
    "best_match",
    "difficulty",
]
