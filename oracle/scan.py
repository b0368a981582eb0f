"""FP64 oracle of the dense range-scan observation update.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper's observation update is eq. (sensor update): P(x | u, z) =
eta P(z | x) P(x | u), normalised to sum one (Sec. III-B).  The paper applies
it on a sampled subset; here it is applied to every state with a per-beam
Gaussian range model:

    P(z | i, j, k) ~ exp(-sum_b (z_b - r(i, j, psi_k + b 2pi/N))^2 / (2 sigma^2)),

r being the expected range from the cell along a world direction, read from a
table of N directions.  Ranges are quantised to h = max_range / 256 on both
sides, so the squared distance is an exact integer (the reading that keeps
the dense form well conditioned).  The distance here is
computed directly per beam, not through the expanded product form.
"""

from __future__ import annotations

import math

import numpy as np

from .filter import FilterState


def quantize_ranges(r, max_range_m: float) -> np.ndarray:
    """Centred range counts: clamp(floor(r / h + 1/2), 0, 256) - 128, h = max_range / 256."""
    h = max_range_m / 256.0
    q = np.floor(np.asarray(r, dtype=np.float64) / h + 0.5)
    return np.clip(q, 0, 256).astype(np.int64) - 128


def beam_offsets(theta: float, n_theta: int, n_beams: int) -> np.ndarray:
    """s_k: table column of beam 0 for channel k, the nearest direction to psi_k."""
    dth = 2.0 * math.pi / n_theta
    step = 2.0 * math.pi / n_beams
    s = np.empty(n_theta, np.int64)
    for k in range(n_theta):
        s[k] = int(math.floor((theta + k * dth) / step + 0.5)) % n_beams
    return s


def scan_sqdist(Rq: np.ndarray, zq: np.ndarray, s: np.ndarray, rows=None,
                chunk: int = 4096) -> np.ndarray:
    """D[k, c] = sum_b (zq[b] - Rq[c, (b + s_k) mod N])^2, exact in int64.

    Rq: (n_cells, N) quantised table; rows: optional subset of cell indices.
    Returns (len(s), n_selected) int64.
    """
    Rq = np.asarray(Rq, dtype=np.int64)
    zq = np.asarray(zq, dtype=np.int64)
    n = Rq.shape[1]
    sel = np.arange(Rq.shape[0]) if rows is None else np.asarray(rows)
    out = np.empty((len(s), len(sel)), np.int64)
    b = np.arange(n)
    for k, sk in enumerate(s):
        cols = (b + int(sk)) % n
        for a in range(0, len(sel), chunk):
            blk = Rq[sel[a:a + chunk]][:, cols]
            diff = zq[None, :] - blk
            out[k, a:a + chunk] = (diff * diff).sum(axis=1)
    return out


def apply_scan(state: FilterState, Rq: np.ndarray, zq: np.ndarray, sigma_m: float,
               max_range_m: float) -> FilterState:
    """Dense observation update in the log domain, then renormalisation.

    L = ln B - c D with c = h^2 / (2 sigma^2); B' = exp(L - max L); B'' = B' / sum B';
    the log-normaliser grows by ln sum_q B_q P(z | q) = max L + ln sum B'.
    A belief with no mass left is reported as degenerate and left unchanged.
    """
    n_theta, H, W = state.B.shape
    s = beam_offsets(state.theta, n_theta, Rq.shape[1])
    D = scan_sqdist(Rq, zq, s).reshape(n_theta, H, W)
    h = max_range_m / 256.0
    c = h * h / (2.0 * sigma_m * sigma_m)
    ns = state.copy()
    with np.errstate(divide="ignore"):
        L = np.log(state.B) - c * D
    mstar = float(L.max())
    if not math.isfinite(mstar):
        ns.degenerate = True
        return ns
    Bp = np.exp(L - mstar)
    total = float(Bp.sum())
    ns.B = Bp / total
    ns.log_norm = state.log_norm + mstar + math.log(total)
    return ns


def scan_sqdist_continuous(R: np.ndarray, z: np.ndarray, s: np.ndarray, chunk: int = 4096) -> np.ndarray:
    """sum_b (z[b] - R[c, (b + s_k) mod N])^2 in FP64 metres^2, on unquantised ranges: (len(s), n_cells)."""
    R = np.asarray(R, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    n = R.shape[1]
    out = np.empty((len(s), R.shape[0]), np.float64)
    b = np.arange(n)
    for k, sk in enumerate(s):
        cols = (b + int(sk)) % n
        for a in range(0, R.shape[0], chunk):
            diff = z[None, :] - R[a:a + chunk][:, cols]
            out[k, a:a + chunk] = (diff * diff).sum(axis=1)
    return out


def apply_scan_continuous(state: FilterState, R: np.ndarray, z: np.ndarray, sigma_m: float) -> FilterState:
    """The per-beam Gaussian of the scan model on unquantised FP64 ranges:
    L = ln B - sum_b (z_b - r)^2 / (2 sigma^2), then as apply_scan.

    This is the model before the quantisation reading (ranges in multiples of
    max_range / 256); it measures what that reading costs the posterior and is
    not the parity reference of the quantised kernels.  With ranges that are
    already multiples of h it equals apply_scan.
    """
    n_theta, H, W = state.B.shape
    s = beam_offsets(state.theta, n_theta, R.shape[1])
    D = scan_sqdist_continuous(R, z, s).reshape(n_theta, H, W)
    ns = state.copy()
    with np.errstate(divide="ignore"):
        L = np.log(state.B) - D / (2.0 * sigma_m * sigma_m)
    mstar = float(L.max())
    if not math.isfinite(mstar):
        ns.degenerate = True
        return ns
    Bp = np.exp(L - mstar)
    total = float(Bp.sum())
    ns.B = Bp / total
    ns.log_norm = state.log_norm + mstar + math.log(total)
    return ns
