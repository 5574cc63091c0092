"""Sampling grids of the problem statement (Section 1, "Description of the problem").

A slice's sinogram y(t, theta) is sampled at n detector bins and V angles in
[0, pi); the reconstructed slice x(u1, u2) at N x N pixels.
Readings (the paper fixes none of these):
  t_i = (i - n/2) dt, dt = 2/n           (bin n/2 is t = 0; +1 is not sampled)
  u   = ((q - N/2) d, (p - N/2) d), d = 2/N, row p <-> u2, column q <-> u1
  theta_j = j pi / V, weight w_j = pi / V; for non-uniform angles w_j is half the
  gap between the neighbours, taken with period pi.
"""
from __future__ import annotations

import numpy as np


class Geometry:
    def __init__(self, n_det: int, n_angles: int, n_out: int, angles=None):
        self.n = int(n_det)
        self.V = int(n_angles)
        self.N = int(n_out)
        self.dt = 2.0 / self.n
        self.d = 2.0 / self.N
        if angles is None:
            self.theta = np.arange(self.V, dtype=np.float64) * (np.pi / self.V)
            self.uniform = True
        else:
            self.theta = np.asarray(angles, dtype=np.float64).copy()
            assert self.theta.shape == (self.V,)
            self.uniform = False
        self.w = self._weights()

    def _weights(self) -> np.ndarray:
        if self.uniform:
            return np.full(self.V, np.pi / self.V)
        th = self.theta
        prev = np.concatenate([[th[-1] - np.pi], th[:-1]])
        nxt = np.concatenate([th[1:], [th[0] + np.pi]])
        return 0.5 * (nxt - prev)

    def t(self) -> np.ndarray:
        return (np.arange(self.n) - self.n // 2) * self.dt

    def u(self) -> np.ndarray:
        return (np.arange(self.N) - self.N // 2) * self.d
