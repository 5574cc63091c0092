"""The BST steps of Section 2 written with literal sums and per-point loops.

For tiny sizes only (N <= 32). It follows the same readings as `bst.py`, but
computes the 1D transform of P3 and the 2D inverse of P6 as explicit DFT sums
(no FFT library) and evaluates P5 point by point with scalar branching, so that
indexing, sign, scaling and Hermitian-convention slips in the vectorised oracle
show up as a mismatch. The 2D inverse over the half plane uses the real-linear
form of the C2R convention:
    b[y][x] = dk^2 sum_{a=0}^{G/2} c_a sum_b Re(C[b][a] e^{2 pi i (a x + b y)/G}),
with c_0 = c_{G/2} = 1 and c_a = 2 otherwise.
"""
from __future__ import annotations

import cmath
import math

import numpy as np

from .geometry import Geometry


def _taper(t: float, dsig: float, kind: str) -> float:
    if kind == "none":
        return 1.0
    x = math.pi * t * dsig
    s = 1.0 if x == 0.0 else math.sin(x) / x
    if kind == "keys":
        return 1.0 / (s ** 3 * (3.0 * s - 2.0 * math.cos(x)))
    return 1.0 / (s * s)


def _keys(x: float) -> float:
    """Keys cubic convolution weight at distance x, a = -1/2."""
    x = abs(x)
    if x <= 1.0:
        return 1.5 * x ** 3 - 2.5 * x ** 2 + 1.0
    if x < 2.0:
        return -0.5 * x ** 3 + 2.5 * x ** 2 - 4.0 * x + 2.0
    return 0.0


def backproject(sino, geom: Geometry, P_r: int = 2, P_c: int = 2,
                filter: str = "ramp", taper: str = "deapod", interp: str = "linear") -> np.ndarray:
    y = np.asarray(sino, dtype=np.float64)
    V, n, N = geom.V, geom.n, geom.N
    dt, d = geom.dt, geom.d
    M, G = P_r * n, P_c * N
    dsig = 1.0 / (M * dt)
    dk = 1.0 / (G * d)
    half = M // 2

    # P1-P4: spectrum on the polar grid, m = 0 .. M/2 - 1 (m = M/2 and beyond are zero)
    Yh = [[0j] * (half + 2) for _ in range(V)]
    Y0 = [0.0] * V
    for j in range(V):
        for m in range(half):
            acc = 0j
            for i in range(n):
                t = (i - n // 2) * dt
                k = (i - n // 2) % M
                acc += _taper(t, dsig, taper) * y[j][i] * cmath.exp(-2j * math.pi * k * m / M)
            acc *= dt
            if m == 0:
                Y0[j] = acc.real
            if filter == "ramp":
                w = 1.0
            else:
                w = 0.0 if m == 0 else (M * dt) / m
            Yh[j][m] = w * acc

    def sample(j: int, m: int, conj: bool) -> complex:
        if m < 0:  # the spectrum of a real line: Yh(-sigma) = conj Yh(sigma)
            m, conj = -m, not conj
        if m >= half:
            return 0j
        v = Yh[j][m]
        return v.conjugate() if conj else v

    # P5: one Cartesian point at a time
    C = [[0j] * (G // 2 + 1) for _ in range(G)]
    for bi in range(G):
        b = bi if bi < G // 2 else bi - G
        for a in range(G // 2 + 1):
            if a == G // 2:  # the Cartesian Nyquist column is dropped
                continue
            if a == 0 and b == 0:
                mean0 = sum(Y0) / V
                C[bi][a] = mean0 if filter == "ramp" else (4.0 * math.asinh(1.0) / dk) * mean0
                continue
            r = math.hypot(a, b) * P_r / P_c
            phi = math.atan2(b, a)
            if phi >= 0.0:
                theta, conj = phi, False
            else:
                theta, conj = phi + math.pi, True
            conj0 = conj
            if geom.uniform:
                q = theta * V / math.pi
                j0 = int(math.floor(q))
                f = q - j0
                if j0 >= V:
                    j0, f = V - 1, 1.0
            else:
                # the period-pi continuation: scan for the last angle <= theta
                th = list(geom.theta)
                j0 = -1
                for jj in range(V):
                    if th[jj] <= theta:
                        j0 = jj
                if j0 < 0:  # below theta_0: the neighbour is theta_{V-1} - pi, conjugated
                    lo, hi = th[V - 1] - math.pi, th[0]
                    j0, conj0 = V - 1, not conj
                else:
                    lo = th[j0]
                    hi = th[j0 + 1] if j0 + 1 < V else th[0] + math.pi
                f = (theta - lo) / (hi - lo)
            j1, conj1 = j0 + 1, conj
            if j1 == V:
                j1 = 0
                if conj0 == conj:  # theta_0 + pi, conjugated (not when j0 is already the image)
                    conj1 = not conj
            m0 = int(math.floor(r))
            g = r - m0
            if interp == "linear":
                C[bi][a] = ((1 - f) * (1 - g) * sample(j0, m0, conj0)
                            + (1 - f) * g * sample(j0, m0 + 1, conj0)
                            + f * (1 - g) * sample(j1, m0, conj1)
                            + f * g * sample(j1, m0 + 1, conj1))
            else:
                acc = 0j
                for mm in range(m0 - 1, m0 + 3):
                    wr = _keys(r - mm)
                    acc += wr * ((1 - f) * sample(j0, mm, conj0) + f * sample(j1, mm, conj1))
                C[bi][a] = acc

    # P6-P8: explicit real-linear inverse sum, evaluated only on the output pixels
    out = np.zeros((N, N))
    for p in range(N):
        yy = (p - N // 2) % G
        for qq in range(N):
            xx = (qq - N // 2) % G
            acc = 0.0
            for bi in range(G):
                for a in range(G // 2 + 1):
                    ca = 1.0 if a in (0, G // 2) else 2.0
                    e = cmath.exp(2j * math.pi * (a * xx + bi * yy) / G)
                    acc += ca * (C[bi][a] * e).real
            out[p][qq] = dk * dk * acc
    return out
