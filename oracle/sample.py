"""Oracle of the sampled observation update (Sec. III-B, Floyd-Steinberg dithering).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Instead of comparing a scan against every state, the paper selects a subset
of states that follows the belief map with Floyd-Steinberg error diffusion and
applies eq. (sensor update) to that subset.  The paper gives no further
detail; the readings taken here:

  * Intensity.  I(i, j) = min(1, N_s * m(i, j) / sum m), with m the belief map
    (max over headings, Sec. III-A last paragraph) and N_s the requested number
    of samples, so that about N_s cells come out selected (the sum is taken in
    FP64 and rounded to FP32; product and quotient are FP32).  The dithering
    decision is taken in FP32, the precision the GPU kernel uses.
  * Dithering.  Floyd-Steinberg in raster order (rows top to bottom, columns
    left to right), threshold 1/2, error weights 7/16 to the right, 3/16 below
    left, 5/16 below and 1/16 below right; error that would leave the grid is
    dropped.  The error a cell receives is summed in the order its sources are
    visited, then added to its intensity; every product and sum is an FP32
    operation rounded to nearest (no fused multiply-add).
  * Update.  A selected cell is a sample for all of its headings.  A state
    that is not sampled takes the likelihood of the best-matching sample
    (the scan neither supports nor contradicts it), so samples can only lose
    mass relative to unsampled states; then the belief is renormalised (eta).
    With every cell selected this is exactly the dense update of `oracle.scan`.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

from .filter import FilterState, belief_map
from .scan import beam_offsets, scan_sqdist

_F = np.float32
_W_RIGHT, _W_BELOW_LEFT, _W_BELOW, _W_BELOW_RIGHT = _F(7.0 / 16), _F(3.0 / 16), _F(5.0 / 16), _F(1.0 / 16)


def dither_intensity(m: np.ndarray, n_samples: int) -> np.ndarray:
    """I = min(1, N_s * m / sum m): the sum in FP64 rounded to FP32, then FP32 product and quotient."""
    m32 = np.asarray(m, dtype=np.float32)
    total = _F(m32.astype(np.float64).sum())
    if not total > 0:
        return np.zeros_like(m32)
    return np.minimum(_F(1.0), (_F(n_samples) * m32) / total).astype(np.float32)


def floyd_steinberg(intensity: np.ndarray) -> np.ndarray:
    """Binary selection mask (uint8) of Floyd-Steinberg error diffusion, raster order, FP32."""
    img = np.asarray(intensity, dtype=np.float32)
    H, W = img.shape
    err = np.zeros((H, W), np.float32)  # error received so far, summed in arrival order
    out = np.zeros((H, W), np.uint8)
    for j in range(H):
        for i in range(W):
            v = _F(img[j, i] + err[j, i])
            sel = v >= _F(0.5)
            out[j, i] = 1 if sel else 0
            e = _F(v - (_F(1.0) if sel else _F(0.0)))
            if i + 1 < W:
                err[j, i + 1] = _F(err[j, i + 1] + _F(_W_RIGHT * e))
            if j + 1 < H:
                if i - 1 >= 0:
                    err[j + 1, i - 1] = _F(err[j + 1, i - 1] + _F(_W_BELOW_LEFT * e))
                err[j + 1, i] = _F(err[j + 1, i] + _F(_W_BELOW * e))
                if i + 1 < W:
                    err[j + 1, i + 1] = _F(err[j + 1, i + 1] + _F(_W_BELOW_RIGHT * e))
    return out


_HERE = os.path.dirname(os.path.abspath(__file__))
_FS_SRC = os.path.join(_HERE, "fs_dither.c")
_FS_LIB = os.path.join(_HERE, "_fs_dither.so")
_fs = None


def build_c(force: bool = True) -> str:
    """Compile fs_dither.c (gcc, no contraction of products into sums)."""
    if force or not os.path.exists(_FS_LIB):
        tmp = _FS_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
                               _FS_SRC, "-o", tmp])
        os.replace(tmp, _FS_LIB)
    return _FS_LIB


def floyd_steinberg_c(intensity: np.ndarray) -> np.ndarray:
    """`floyd_steinberg` in C (same operations in the same order), for large images."""
    global _fs
    if _fs is None:
        if not os.path.exists(_FS_LIB):
            build_c(force=False)
        lib = ctypes.CDLL(_FS_LIB)
        lib.oracle_fs_dither.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_void_p]
        lib.oracle_fs_dither.restype = ctypes.c_int
        _fs = lib
    img = np.ascontiguousarray(intensity, dtype=np.float32)
    H, W = img.shape
    out = np.zeros((H, W), np.uint8)
    if H and W:
        if _fs.oracle_fs_dither(img.ctypes.data, W, H, out.ctypes.data) != 0:
            raise MemoryError("fs_dither: out of memory")
    return out


def sample_mask(B: np.ndarray, n_samples: int) -> np.ndarray:
    """Cells selected from the belief map of B (n_theta, H, W)."""
    return floyd_steinberg(dither_intensity(belief_map(B), n_samples))


def apply_scan_sampled(state: FilterState, Rq: np.ndarray, zq: np.ndarray, sigma_m: float,
                       max_range_m: float, mask: np.ndarray) -> FilterState:
    """Eq. (sensor update) on the states of the selected cells (FP64).

    D is the exact integer squared distance of the quantised scan (as in
    `oracle.scan`); D* its minimum over all sampled states.  Sampled states are
    multiplied by exp(-c (D - D*)), the others keep their value; the belief is
    renormalised and the log-normaliser grows by ln sum B' - c D*.  No sample:
    no update.
    """
    n_theta, H, W = state.B.shape
    cells = np.flatnonzero(np.asarray(mask).reshape(-1))
    ns = state.copy()
    if len(cells) == 0:
        return ns
    s = beam_offsets(state.theta, n_theta, Rq.shape[1])
    D = scan_sqdist(Rq, zq, s, rows=cells)  # (n_theta, n_cells)
    h = max_range_m / 256.0
    c = h * h / (2.0 * sigma_m * sigma_m)
    dstar = int(D.min())
    flat = state.B.reshape(n_theta, H * W).copy()
    flat[:, cells] = flat[:, cells] * np.exp(-c * (D - dstar))
    total = float(flat.sum())
    if not (total > 0.0):
        ns.degenerate = True
        return ns
    ns.B = (flat / total).reshape(n_theta, H, W)
    ns.log_norm = state.log_norm + math.log(total) - c * dstar - math.log(float(state.B.sum()))
    return ns
