"""Dense brute-force model of one filter step, independent of `oracle/`.

Used only to pin the oracle on tiny grids.  It is written from the paper in
a different form than the oracle, so a slip in either shows up as a mismatch:

* the affine warp is a *push*: every source state scatters its mass to the
  four cells around its continuous target position (the oracle pulls);
* the motion-noise kernel is the unseparated 3-D Gaussian
  exp(-1/2 d^T Sigma^-1 d) with Sigma = R_z^T diag(sx^2, sy^2, st^2) R_z
  (eq. Gaussian kernel and its covariance), evaluated on the box
  |dx|, |dy| <= r_xy, |dtheta| <= r_theta, normalised over the box, and stored
  as an explicit n x n matrix (the oracle runs separable shifted sums);
* the kernel activation is that matrix applied to the free-space vector.
"""

from __future__ import annotations

import math

import numpy as np


def _rot(psi):
    c, s = math.cos(psi), math.sin(psi)
    return np.array([[c, -s], [s, c]])


def _quad_form(d, psi, sx, sy, st):
    """d^T Sigma^-1 d for the rotated diagonal covariance; zero sigmas are impulses."""
    Rz = np.eye(3)
    Rz[:2, :2] = _rot(psi)
    sig = np.array([sx, sy, st], dtype=np.float64)
    live = sig > 0
    if np.any(np.abs(np.asarray(d)[~live]) > 0):
        return math.inf
    if not live.any():
        return 0.0
    Sigma = Rz.T @ np.diag(np.where(live, sig, 1.0) ** 2) @ Rz
    idx = np.where(live)[0]
    sub = Sigma[np.ix_(idx, idx)]
    dv = np.asarray(d, dtype=np.float64)[idx]
    return float(dv @ np.linalg.solve(sub, dv))


class DenseModel:
    """Explicit matrices for one map and one set of noise parameters."""

    def __init__(self, occ, n_theta, sigma_xy, r_xy, sigma_th, r_th, wall_normalize=True,
                 mask_before_blur=True, sigma_lateral=None, theta=0.0):
        self.occ = np.asarray(occ)
        self.H, self.W = self.occ.shape
        self.T = n_theta
        self.n = n_theta * self.H * self.W
        self.mask = np.tile((self.occ == 0).astype(np.float64).reshape(-1), n_theta)
        self.wall_normalize = wall_normalize
        self.mask_before_blur = mask_before_blur
        self.sigma_lateral = sigma_lateral
        self.theta = theta
        self.K = self._kernel_matrix(sigma_xy, r_xy, sigma_th, r_th)
        A = self.K @ self.mask
        self.post = np.where(self.mask > 0, self.mask / np.where(A > 0, A, 1.0), 0.0) \
            if wall_normalize else self.mask.copy()

    def idx(self, k, j, i):
        return (k * self.H + j) * self.W + i

    def _box(self, psi, sx, sy, sth, rxy, rth):
        box = []
        for dk in range(-rth, rth + 1):
            for dy in range(-rxy, rxy + 1):
                for dx in range(-rxy, rxy + 1):
                    q = _quad_form((dx, dy, dk), psi, sx, sy, sth)
                    box.append((dx, dy, dk, 0.0 if math.isinf(q) else math.exp(-0.5 * q)))
        z = sum(b[3] for b in box)
        return [(dx, dy, dk, w / z) for dx, dy, dk, w in box]

    def _kernel_matrix(self, sxy, rxy, sth, rth):
        # isotropic: one box (its rotation is immaterial); anisotropic: the box of
        # each *target* channel, with the covariance R(psi) diag(s^2) R(psi)^T of
        # that channel's heading psi (passed as -psi to the R_z^T D R_z form)
        dth = 2.0 * math.pi / self.T
        if self.sigma_lateral is None:
            boxes = [self._box(0.37, sxy, sxy, sth, rxy, rth)] * self.T
        else:
            boxes = [self._box(-(self.theta + tk * dth), sxy, self.sigma_lateral, sth, rxy, rth)
                     for tk in range(self.T)]
        K = np.zeros((self.n, self.n))
        for k in range(self.T):
            for j in range(self.H):
                for i in range(self.W):
                    src = self.idx(k, j, i)
                    for dk in range(-rth, rth + 1):
                        tk = (k + dk) % self.T
                        for dx, dy, ddk, wgt in boxes[tk]:
                            if ddk != dk or wgt == 0.0:
                                continue
                            ti, tj = i + dx, j + dy
                            if 0 <= ti < self.W and 0 <= tj < self.H:
                                K[self.idx(tk, tj, ti), src] += wgt
        return K

    def push_matrix(self, u, v, theta, cell):
        P = np.zeros((self.n, self.n))
        for k in range(self.T):
            d = _rot(theta + k * 2.0 * math.pi / self.T) @ np.array([u, v]) / cell
            for j in range(self.H):
                for i in range(self.W):
                    tx, ty = i + d[0], j + d[1]
                    i0, j0 = math.floor(tx), math.floor(ty)
                    fx, fy = tx - i0, ty - j0
                    for ii, wx in ((i0, 1.0 - fx), (i0 + 1, fx)):
                        for jj, wy in ((j0, 1.0 - fy), (j0 + 1, fy)):
                            if 0 <= ii < self.W and 0 <= jj < self.H:
                                P[self.idx(k, jj, ii), self.idx(k, j, i)] += wx * wy
        return P

    def step(self, b, u, v, theta, cell):
        """Returns (unnormalised next belief as (T, H, W), kept mass)."""
        x = self.push_matrix(u, v, theta, cell) @ b.reshape(-1)
        if self.mask_before_blur:
            x = self.mask * x
        x = self.post * (self.K @ x)
        return x.reshape(self.T, self.H, self.W), float(x.sum())
