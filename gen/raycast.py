"""ctypes front end of raycast.c (built in place by `build()`)."""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "raycast.c")
_LIB = os.path.join(_HERE, "_raycast.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile raycast.c into gen/_raycast.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.gen_range_table.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                        ctypes.c_int, ctypes.c_double, ctypes.c_void_p]
        lib.gen_range_table.restype = None
        lib.gen_scan.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_void_p]
        lib.gen_scan.restype = None
        _lib = lib
    return _lib


def range_table(occ: np.ndarray, cell_m: float, n_dirs: int, max_range_m: float) -> np.ndarray:
    """(H*W, n_dirs) float32 expected ranges from every cell centre."""
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    h, w = occ.shape
    out = np.empty((h * w, n_dirs), np.float32)
    _load().gen_range_table(occ.ctypes.data, w, h, float(cell_m), int(n_dirs), float(max_range_m),
                            out.ctypes.data)
    return out


def scan_at(occ: np.ndarray, cell_m: float, x: float, y: float, heading: float, n_beams: int,
            max_range_m: float) -> np.ndarray:
    """(n_beams,) float32 noise-free ranges from world pose (x, y, heading)."""
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    h, w = occ.shape
    out = np.empty(n_beams, np.float32)
    _load().gen_scan(occ.ctypes.data, w, h, float(cell_m), float(x), float(y), float(heading),
                     int(n_beams), float(max_range_m), out.ctypes.data)
    return out


def noisy_scan(occ, cell_m, pose, n_beams, max_range_m, sigma_m, seed) -> np.ndarray:
    """Scan from `pose` plus N(0, sigma_m) per beam, clamped to [0, max_range]."""
    rng = np.random.default_rng(seed)
    z = scan_at(occ, cell_m, pose[0], pose[1], pose[2], n_beams, max_range_m).astype(np.float64)
    z = z + rng.normal(0.0, sigma_m, n_beams)
    return np.clip(z, 0.0, max_range_m).astype(np.float32)


def cell_scans(R: np.ndarray, cells, sigma_m: float, max_range_m: float, seed: int) -> np.ndarray:
    """(len(cells), n_dirs) float32 scans taken at cell centres, heading 0: the
    expected ranges R[cells] plus N(0, sigma_m) per beam, clamped to [0, max_range]."""
    rng = np.random.default_rng(seed)
    z = np.asarray(R, np.float64)[np.asarray(cells)]
    if sigma_m > 0:
        z = z + rng.normal(0.0, sigma_m, z.shape)
    return np.clip(z, 0.0, max_range_m).astype(np.float32)
