"""FP64 oracle of one odometry step of the belief-tensor filter.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function cites
the passage of the paper it follows:

* Sec. III-A (belief tensor): B has shape (Theta, H, W); entry [k, j, i] is the
  state x = (i*delta, j*delta, k*delta_Theta + theta_t), with theta_t a running
  heading offset updated by theta_t = theta_{t-1} + w.
* Sec. III-A-1 (motion update): channel k moves by R(psi_k) [u, v]^T, with
  psi_k the heading of that channel, through a translation-only affine warp.
* Sec. III-A-2 (motion uncertainty): a 3-D Gaussian convolution.
* Sec. III-A-3 and Alg. 1 (map sensor update): multiply by the traversability
  map before and after the blur, then divide by the kernel activation of the
  free-space tensor.
* Eq. (sensor update): renormalise so the belief sums to one.

Readings where the paper is silent or ambiguous:
isotropic xy noise (so the heading rotation of the covariance is a no-op and
the kernel separates), sampled taps normalised to sum one with radius
ceil(3 sigma), bilinear warp with zero outside the grid, the pre-step heading
rotating (u, v), renormalisation after every step with the log of the kept
mass accumulated, and the sub-cell gate as an option that accumulates motion.
The integer-shift option reads the warp of Alg. 1 as a whole-cell translation:
each channel moves by its displacement plus the remainder it carries, rounded
to whole cells (half up), and carries the new remainder.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class OracleParams:
    n_theta: int
    cell_m: float
    sigma_xy: float            # motion-noise std-dev in cells (Sec. III-A-2, diag entries)
    sigma_theta: float         # motion-noise std-dev in theta bins
    radius_xy: int = -1        # -1 => ceil(3 sigma)
    radius_theta: int = -1
    mask_before_blur: bool = True   # Alg. 1, statement after the warp
    wall_normalize: bool = True     # Alg. 1, division by the kernel activation
    subcell_gate: bool = False      # Alg. 1, "IF |u_{t,k}| >= 1"
    integer_shift: bool = False     # whole-cell warp with a per-channel remainder carry
    sigma_lateral: float = -1.0     # >= 0: anisotropic noise, sigma_xy along the heading, this across

    def rxy(self) -> int:
        if self.radius_xy >= 0:
            return self.radius_xy
        if self.sigma_lateral >= 0:
            return default_radius(max(self.sigma_xy, self.sigma_lateral))
        return default_radius(self.sigma_xy)

    def rth(self) -> int:
        return default_radius(self.sigma_theta) if self.radius_theta < 0 else self.radius_theta


@dataclasses.dataclass
class FilterState:
    B: np.ndarray              # (Theta, H, W) float64, sums to 1
    theta: float = 0.0         # running heading offset theta_t (rad)
    log_norm: float = 0.0      # sum over steps of ln(kept mass)
    steps: int = 0
    acc: tuple = (0.0, 0.0)    # accumulated world displacement (sub-cell gate only)
    degenerate: bool = False
    rem: np.ndarray | None = None  # (Theta, 2) carried remainder in cells (integer shift only)

    def copy(self) -> "FilterState":
        return dataclasses.replace(self, B=self.B.copy(), rem=None if self.rem is None else self.rem.copy())


# --------------------------------------------------------------------------
# kernel and map precomputation
# --------------------------------------------------------------------------

def default_radius(sigma: float) -> int:
    return int(math.ceil(3.0 * sigma))


def gaussian_taps(sigma: float, radius: int) -> np.ndarray:
    """Sampled 1-D Gaussian exp(-m^2 / (2 sigma^2)), |m| <= radius, summing to 1.

    Eq. (Gaussian kernel) with a diagonal covariance restricted to one axis; the
    paper prints no normalising constant, and any constant cancels in the
    wall normalisation and the renormalisation.  sigma = 0 is a unit impulse.
    """
    m = np.arange(-radius, radius + 1, dtype=np.float64)
    if sigma == 0.0:
        g = (m == 0).astype(np.float64)
    else:
        g = np.exp(-(m * m) / (2.0 * sigma * sigma))
    return g / g.sum()


def free_mask(occupancy: np.ndarray) -> np.ndarray:
    """Traversability M (1 free, 0 occupied) as float64 (Sec. III-A-3)."""
    return (np.asarray(occupancy) == 0).astype(np.float64)


def _translate(a: np.ndarray, d: int, axis: int) -> np.ndarray:
    """out[.., p, ..] = a[.., p - d, ..] along `axis`; zero where p - d is outside."""
    out = np.zeros_like(a)
    n = a.shape[axis]
    if abs(d) >= n:
        return out
    src = [slice(None)] * a.ndim
    dst = [slice(None)] * a.ndim
    if d >= 0:
        dst[axis] = slice(d, n)
        src[axis] = slice(0, n - d)
    else:
        dst[axis] = slice(0, n + d)
        src[axis] = slice(-d, n)
    out[tuple(dst)] = a[tuple(src)]
    return out


def blur_x(s: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Convolution along x (last axis) with taps g, zero outside the grid (Sec. III-A-2)."""
    r = (len(g) - 1) // 2
    out = np.zeros_like(s)
    for m in range(-r, r + 1):
        out += g[m + r] * _translate(s, m, axis=-1)
    return out


def blur_y(s: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Convolution along y (second-to-last axis), zero outside the grid."""
    r = (len(g) - 1) // 2
    out = np.zeros_like(s)
    for m in range(-r, r + 1):
        out += g[m + r] * _translate(s, m, axis=-2)
    return out


def blur_theta(s: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Convolution along theta (axis 0), circular because heading wraps."""
    r = (len(g) - 1) // 2
    out = np.zeros_like(s)
    for m in range(-r, r + 1):
        out += g[m + r] * np.roll(s, m, axis=0)
    return out


def rotated_taps(sigma_f: float, sigma_l: float, radius: int, psi: float) -> np.ndarray:
    """2-D taps of the heading-rotated Gaussian (eq. Gaussian kernel and its covariance), summing to 1.

    Covariance R(psi) diag(sigma_f^2, sigma_l^2) R(psi)^T: sigma_f along the
    heading (cos psi, sin psi), sigma_l across it.  Tap [n + r, m + r] is the
    weight of the displacement (m, n) = (dx, dy) in cells, |m|, |n| <= radius.
    """
    c, s = math.cos(psi), math.sin(psi)
    g = np.zeros((2 * radius + 1, 2 * radius + 1))
    for n in range(-radius, radius + 1):
        for m in range(-radius, radius + 1):
            a = c * m + s * n     # along the heading
            b = -s * m + c * n    # across it
            q = a * a / (sigma_f * sigma_f) + b * b / (sigma_l * sigma_l)
            g[n + radius, m + radius] = math.exp(-0.5 * q)
    return g / g.sum()


def conv2d(s: np.ndarray, g: np.ndarray) -> np.ndarray:
    """out(i, j) = sum_{m, n} g[n + r, m + r] s(i - m, j - n) on an (H, W) plane, zero outside."""
    r = (g.shape[0] - 1) // 2
    out = np.zeros_like(s)
    for n in range(-r, r + 1):
        for m in range(-r, r + 1):
            out += g[n + r, m + r] * _translate(_translate(s, m, axis=-1), n, axis=-2)
    return out


def kernel_activation(M: np.ndarray, g_xy: np.ndarray, g_th: np.ndarray) -> np.ndarray:
    """G(B_0, k): the blur of the binary free-space tensor (Alg. 1, last statement).

    B_0 is M broadcast over theta, so the theta blur only contributes the sum
    of its taps and the result is the same for every channel k.
    """
    return blur_y(blur_x(M, g_xy), g_xy) * g_th.sum()


def wall_weights(M: np.ndarray, A: np.ndarray, wall_normalize: bool = True) -> np.ndarray:
    """Post-blur multiplier: M / G(B_0) on free cells, 0 on occupied ones.

    Alg. 1 multiplies by M and then by the pixel-wise inverse of the kernel
    activation (Sec. III-A-3, the "cliff" argument).  A > 0 on every free cell
    because the activation includes the cell itself.
    """
    if not wall_normalize:
        return M.copy()
    out = np.zeros_like(M)
    free = M > 0
    out[free] = M[free] / A[free]
    return out


def init_uniform(occupancy: np.ndarray, n_theta: int) -> FilterState:
    """B_0 uniform over free cells and all headings (Sec. III-A, belief tensor)."""
    M = free_mask(occupancy)
    total = M.sum() * n_theta
    if total == 0:
        raise ValueError("map has no free cell")
    B = np.broadcast_to(M / total, (n_theta,) + M.shape).copy()
    return FilterState(B=B)


# --------------------------------------------------------------------------
# motion update
# --------------------------------------------------------------------------

def slice_displacements(u: float, v: float, theta: float, n_theta: int, cell_m: float):
    """Per-channel displacement in cells: R(theta + k delta_Theta) [u, v]^T / cell.

    Sec. III-A-1: channel k has heading psi_k = theta + k delta_Theta; its
    motion is the robot-frame increment rotated into the world frame.
    """
    dth = 2.0 * math.pi / n_theta
    dx = np.empty(n_theta)
    dy = np.empty(n_theta)
    for k in range(n_theta):
        psi = theta + k * dth
        c, s = math.cos(psi), math.sin(psi)
        dx[k] = (u * c - v * s) / cell_m
        dy[k] = (u * s + v * c) / cell_m
    return dx, dy


def shift_bilinear(b: np.ndarray, dx: float, dy: float) -> np.ndarray:
    """Translate one (H, W) channel by (dx, dy) cells with bilinear weights.

    The affine warp of Sec. III-A-1 with matrix [[1, 0, dx], [0, 1, dy]], read
    as a mass-conserving bilinear resampling: with n = floor(d), f = d - n,
    out(i, j) = sum_{a, b in {0,1}} wx_a wy_b B(i - nx - a, j - ny - b),
    wx_0 = 1 - fx, wx_1 = fx (likewise in y); zero outside the grid.
    """
    nx = math.floor(dx)
    ny = math.floor(dy)
    fx = dx - nx
    fy = dy - ny
    out = np.zeros_like(b)
    for a, wa in ((0, 1.0 - fx), (1, fx)):
        for bb, wb in ((0, 1.0 - fy), (1, fy)):
            if wa == 0.0 or wb == 0.0:
                continue
            out += (wa * wb) * _translate(_translate(b, nx + a, axis=1), ny + bb, axis=0)
    return out


def integer_shifts(dx, dy, rem):
    """Whole-cell displacements with a carried remainder (integer-shift option).

    Channel k moves by n = floor(d + 1/2) cells, d = its displacement plus the
    remainder it carries, and keeps d - n (so |remainder| <= 1/2 and the sum of
    the whole-cell moves tracks the summed displacement).  Returns (nx, ny,
    new remainder).
    """
    r = np.zeros((len(dx), 2)) if rem is None else rem
    d = np.stack([np.asarray(dx, float) + r[:, 0], np.asarray(dy, float) + r[:, 1]], axis=1)
    n = np.floor(d + 0.5)
    return n[:, 0], n[:, 1], d - n


def step(state: FilterState, occupancy: np.ndarray, p: OracleParams, u: float, v: float,
         w: float, *, M=None, Wt=None) -> FilterState:
    """One odometry step, Alg. 1 followed by renormalisation.

    Order of passes: warp every channel (AF), multiply by M, 3-D Gaussian blur
    (x, then y, then circular theta), multiply by M / G(B_0), renormalise.
    A degenerate step (no mass survives) leaves the belief unchanged and sets
    the flag.  Returns a new state.
    """
    if M is None:
        M = free_mask(occupancy)
    g_xy = gaussian_taps(p.sigma_xy, p.rxy())
    g_th = gaussian_taps(p.sigma_theta, p.rth())
    if Wt is None:
        Wt = wall_weights(M, kernel_activation(M, g_xy, g_th), p.wall_normalize)
    ns = state.copy()
    ns.steps += 1
    if p.subcell_gate:
        c, s = math.cos(state.theta), math.sin(state.theta)
        ax = state.acc[0] + u * c - v * s
        ay = state.acc[1] + u * s + v * c
        ns.theta = state.theta + w
        if math.hypot(ax, ay) < p.cell_m:
            ns.acc = (ax, ay)
            return ns
        ns.acc = (0.0, 0.0)
        dx, dy = slice_displacements(ax, ay, 0.0, p.n_theta, p.cell_m)
    else:
        dx, dy = slice_displacements(u, v, state.theta, p.n_theta, p.cell_m)
        ns.theta = state.theta + w
    if p.integer_shift:
        dx, dy, ns.rem = integer_shifts(dx, dy, state.rem)
    S = np.empty_like(state.B)
    for k in range(p.n_theta):
        S[k] = shift_bilinear(state.B[k], dx[k], dy[k])
    if p.mask_before_blur:
        S = S * M
    if p.sigma_lateral >= 0:
        U = _anisotropic_blur(S, M, p, g_th, state.theta)
    else:
        T = blur_theta(blur_y(blur_x(S, g_xy), g_xy), g_th)
        U = T * Wt
    total = float(U.sum())
    if not (total > 0.0) or not math.isfinite(total):
        ns.B = state.B.copy()
        ns.degenerate = True
        return ns
    ns.B = U / total
    ns.log_norm = state.log_norm + math.log(total)
    return ns


def _anisotropic_blur(S, M, p, g_th, theta):
    """Anisotropic, heading-rotated motion noise (eq. Gaussian kernel with its rotated covariance).

    The kernel of output channel k is the 2-D Gaussian rotated to that
    channel's heading psi_k = theta + k delta_Theta (the heading its motion
    was rotated by) times the theta Gaussian, so the theta blur runs first and
    each channel then gets its own 2-D blur.  The kernel activation G(B_0, k)
    depends on k: the channel's 2-D blur of M times the sum of the theta taps.
    Then the post-blur mask and M / G(B_0, k) as in Alg. 1.
    """
    r = p.rxy()
    dth = 2.0 * math.pi / p.n_theta
    T = blur_theta(S, g_th)
    U = np.empty_like(S)
    for k in range(p.n_theta):
        g = rotated_taps(p.sigma_xy, p.sigma_lateral, r, theta + k * dth)
        Tk = conv2d(T[k], g)
        Ak = conv2d(M, g) * g_th.sum()
        U[k] = Tk * wall_weights(M, Ak, p.wall_normalize)
    return U


def run(occupancy: np.ndarray, p: OracleParams, odometry, state: FilterState | None = None,
        callback=None) -> FilterState:
    """Apply `step` for every (u, v, w) row of `odometry`; callback(t, state) after each."""
    M = free_mask(occupancy)
    g_xy = gaussian_taps(p.sigma_xy, p.rxy())
    g_th = gaussian_taps(p.sigma_theta, p.rth())
    Wt = wall_weights(M, kernel_activation(M, g_xy, g_th), p.wall_normalize)
    st = init_uniform(occupancy, p.n_theta) if state is None else state
    for t, (u, v, w) in enumerate(odometry):
        st = step(st, occupancy, p, float(u), float(v), float(w), M=M, Wt=Wt)
        if callback is not None:
            callback(t, st)
    return st


# --------------------------------------------------------------------------
# readout
# --------------------------------------------------------------------------

def belief_map(B: np.ndarray) -> np.ndarray:
    """Max over the theta channels (Sec. III-A, last paragraph)."""
    return B.max(axis=0)


def argmax_pose(B: np.ndarray):
    """(k, j, i) of the largest entry; the lowest flat index wins ties."""
    flat = int(np.argmax(B.reshape(-1)))
    k, rem = divmod(flat, B.shape[1] * B.shape[2])
    j, i = divmod(rem, B.shape[2])
    return k, j, i
