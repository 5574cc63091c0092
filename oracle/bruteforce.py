"""Pixel-driven brute-force backprojection and its transpose (FP64).

B_d discretises Eq. 2 (Section 1): the integral over theta becomes the sum over
the V angles with weights w_j, and y(u . xi_theta, theta) is read from the
detector samples by linear interpolation (the hat function Lambda), with zero
outside the sampled bins. This is the "slant-stack" direct summation the paper
compares against (Section 2, last paragraph), O(N^2 V) per slice:

    B_d y[p][q] = sum_j w_j sum_i y[j][i] Lambda(s_pqj - i),
    s_pqj = (u_pq . xi_j) / dt + n/2.

R_d discretises Eq. 1 as the exact transpose of B_d under the weighted inner
products <f, f'> = d^2 sum f f' and <g, g'> = dt sum_j w_j sum_i g g':

    R_d f[j][i] = (d^2 / dt) sum_pq f[p][q] Lambda(s_pqj - i),

so <R_d f, g> = <f, B_d g> holds to rounding (the adjoint relation B = R* of
Section 1).
"""
from __future__ import annotations

import numpy as np

from .geometry import Geometry


def _positions(geom: Geometry, j: int, rows=None, cols=None) -> np.ndarray:
    """s_pqj for the requested rows/columns (all by default)."""
    u = geom.u()
    u1 = u[None, :] if cols is None else u[cols][None, :]
    u2 = u[:, None] if rows is None else u[rows][:, None]
    c, s = np.cos(geom.theta[j]), np.sin(geom.theta[j])
    return (u1 * c + u2 * s) / geom.dt + geom.n / 2


def _lerp(row: np.ndarray, s: np.ndarray) -> np.ndarray:
    """sum_i row[i] Lambda(s - i) with row[i] = 0 outside [0, n)."""
    n = row.shape[0]
    ext = np.concatenate([[0.0], row, [0.0]])  # ext[k] = row[k-1]
    i0 = np.floor(s)
    f = s - i0
    i0 = i0.astype(np.int64)
    a = np.clip(i0 + 1, 0, n + 1)
    b = np.clip(i0 + 2, 0, n + 1)
    va = np.where((i0 >= 0) & (i0 < n), ext[a], 0.0)
    vb = np.where((i0 + 1 >= 0) & (i0 + 1 < n), ext[b], 0.0)
    return (1.0 - f) * va + f * vb


def backproject(sino: np.ndarray, geom: Geometry) -> np.ndarray:
    """B_d of one sinogram [V][n] -> image [N][N], FP64."""
    y = np.asarray(sino, dtype=np.float64)
    assert y.shape == (geom.V, geom.n)
    out = np.zeros((geom.N, geom.N))
    for j in range(geom.V):
        out += geom.w[j] * _lerp(y[j], _positions(geom, j))
    return out


def backproject_pixels(sino: np.ndarray, geom: Geometry, rows, cols) -> np.ndarray:
    """B_d evaluated only at the listed pixels (rows[k], cols[k]) -> [K]."""
    y = np.asarray(sino, dtype=np.float64)
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    u = geom.u()
    u1, u2 = u[cols], u[rows]
    out = np.zeros(rows.shape[0])
    for j in range(geom.V):
        c, s = np.cos(geom.theta[j]), np.sin(geom.theta[j])
        out += geom.w[j] * _lerp(y[j], (u1 * c + u2 * s) / geom.dt + geom.n / 2)
    return out


def project(img: np.ndarray, geom: Geometry) -> np.ndarray:
    """R_d of one image [N][N] -> sinogram [V][n], FP64 (transpose of B_d)."""
    f = np.asarray(img, dtype=np.float64)
    assert f.shape == (geom.N, geom.N)
    n = geom.n
    out = np.zeros((geom.V, n))
    scale = geom.d ** 2 / geom.dt
    fv = f.ravel()
    for j in range(geom.V):
        s = _positions(geom, j).ravel()
        i0 = np.floor(s)
        fr = s - i0
        i0 = i0.astype(np.int64)
        acc = np.zeros(n + 2)  # acc[k] collects bin k-1
        ia = np.clip(i0 + 1, 0, n + 1)
        ib = np.clip(i0 + 2, 0, n + 1)
        ma = (i0 >= 0) & (i0 < n)
        mb = (i0 + 1 >= 0) & (i0 + 1 < n)
        acc += np.bincount(ia[ma], weights=(fv * (1.0 - fr))[ma], minlength=n + 2)
        acc += np.bincount(ib[mb], weights=(fv * fr)[mb], minlength=n + 2)
        out[j] = scale * acc[1:n + 1]
    return out


def inner_image(f: np.ndarray, g: np.ndarray, geom: Geometry) -> float:
    return float(geom.d ** 2 * np.sum(f * g))


def inner_sino(a: np.ndarray, b: np.ndarray, geom: Geometry) -> float:
    return float(geom.dt * np.sum(geom.w[:, None] * a * b))
