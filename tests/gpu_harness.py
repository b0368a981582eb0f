"""Shared helpers of the GPU parity tests: run the HIP path and the oracle side by side."""

from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle as O

try:
    import torch
    HAVE_GPU = torch.cuda.is_available()
except Exception:  # pragma: no cover
    HAVE_GPU = False

needs_gpu = pytest.mark.skipif(not HAVE_GPU, reason="needs a GPU")

# FP32 bound on the peak-normalised max-abs error against the FP64 oracle.
FP32_PEAK_TOL = 1e-5
# argmax agreement: the GPU argmax lies in the oracle's tie set {B >= max (1 - tau)}
FP32_TIE_TAU = 1e-6


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def oracle_params(n_theta, cell, sxy, sth, rxy=-1, rth=-1, flags=3, sigma_lateral=-1.0):
    return O.OracleParams(n_theta=n_theta, cell_m=cell, sigma_xy=sxy, sigma_theta=sth, radius_xy=rxy,
                          sigma_lateral=sigma_lateral if flags & 32 else -1.0,
                          radius_theta=rth, mask_before_blur=bool(flags & 1),
                          wall_normalize=bool(flags & 2), subcell_gate=bool(flags & 4),
                          integer_shift=bool(flags & 16))


def make_gpu(occ, cell, n_theta, sxy, sth, rxy=-1, rth=-1, storage="f32", flags=3, init=None, theta0=0.0,
             range_table=None, max_range_m=0.0, sigma_lateral=0.0, launch_shape=None):
    from paper_1910_00572_amd import mcl
    m = mcl.Map(occ, cell, sxy, radius_xy=rxy, flags=flags, range_table=range_table, max_range_m=max_range_m)
    f = mcl.Filter(m, n_theta, sth, radius_theta=rth, storage=storage, init=init, theta0=theta0,
                   sigma_lateral=sigma_lateral, launch_shape=launch_shape)
    return m, f


def peak_err(gpu_b, ref_b):
    return float(np.abs(gpu_b.astype(np.float64) - ref_b).max() / ref_b.max())


def l1_err(gpu_b, ref_b):
    return float(np.abs(gpu_b.astype(np.float64) - ref_b).sum())


def in_tie_set(pose_kji, ref_b, tau):
    k, j, i = pose_kji
    return bool(ref_b[k, j, i] >= ref_b.max() * (1.0 - tau))


def stored_belief(f):
    """The filter's stored belief as the kernels hold it (pitch layout,
    storage type, scaled), widened to float64 and cut to (T, H, W).

    Read with a plain device-to-host copy of mcl_info.belief_device, so a
    test can start the oracle from exactly the values the GPU holds.
    """
    import ctypes
    inf = f.info(sync=True)
    eb = 4 if inf.storage == 0 else 2
    n = inf.n_theta * inf.height * inf.pitch
    raw = np.empty(n * eb, np.uint8)
    hip = ctypes.CDLL("libamdhip64.so.7")
    hip.hipMemcpy.restype = ctypes.c_int
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    rc = hip.hipMemcpy(raw.ctypes.data, inf.belief_device, n * eb, 2)  # device to host
    assert rc == 0, f"hipMemcpy failed ({rc})"
    if inf.storage == 0:
        vals = raw.view(np.float32).astype(np.float64)
    elif inf.storage == 1:
        vals = (raw.view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    else:
        vals = raw.view(np.float16).astype(np.float64)
    return vals.reshape(inf.n_theta, inf.height, inf.pitch)[:, :, :inf.width].copy()


def oracle_state_from(stored, log_norm, theta):
    """An oracle state holding the GPU's stored belief, renormalised in FP64."""
    return O.FilterState(B=stored / stored.sum(), theta=theta, log_norm=log_norm)
