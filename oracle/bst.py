"""BST backprojection, FP64, steps P0..P8 in the paper's order (Section 2).

The backprojection-slice theorem (Eq. 3) states that the 2D Fourier transform
of b = B y on the ray of direction theta equals the 1D transform of the
projection y(., theta) divided by |sigma|. With the ordinary-frequency
convention f^(k) = int f(x) exp(-2 pi i k.x) dx and the change of variables
k = sigma xi_theta (sigma signed, theta in [0, pi), Jacobian |sigma|), Eq. 2
gives b^(sigma xi_theta) = y^(sigma, theta) / |sigma| with no extra constants.
FBP (x = B F y, F with transfer |sigma|, Section 1) therefore places y^ itself
on the polar grid ("RAMP" mode); plain B divides by |sigma| ("NONE" mode).

Discrete steps (readings where the paper is silent are listed beside each):
  P0  polar re-index: identity, because y(t, theta + pi) = y(-t, theta) lets the
      signed-sigma transform on [0, pi) stand for sigma > 0 on [0, 2 pi).
  P1  taper w[i] in t. Default: 1/sinc^2(t_i dsigma), which undoes the roll-off
      of linear interpolation along the radius in P5 (the paper names a
      Kaiser-Bessel window without parameters; 'kb' and 'none' are options).
  P2  zero pad each projection from n to M = P_r n samples, t = 0 at index 0:
      z[(i - n/2) mod M] = w[i] y[i].
  P3  Y_j[m] = dt * sum_k z_j[k] exp(-2 pi i k m / M), m = 0..M/2,
      sigma_m = m dsigma, dsigma = 1 / (M dt).
  P4  Yh_j[m] = K[m] Y_j[m]; NONE: K[m] = 1/sigma_m (K[0] = 0); RAMP: K[m] = 1.
      Both set K[M/2] = 0 (the Nyquist sample is dropped).
  P5  bilinear interpolation in (radius r = |k|/dsigma, angle index
      q = theta V / pi) at every Cartesian point k = (a, b) dk of the half plane
      a in [0, G/2], b in [-G/2, G/2), G = P_c N, dk = 1/(G d); points on
      the lower half (b < 0) read theta + pi via the conjugate; the angle
      neighbour past theta_{V-1} is theta_0 with sigma reversed (conjugate);
      radial samples m >= M/2 are zero. The origin takes its own rule:
      RAMP: mean_j Y_j[0]; NONE: (kappa / dk) mean_j Y_j[0], kappa = 4 asinh(1),
      the average of 1/|k| over the origin cell times dk.
  P6  2D inverse DFT over the Hermitian plane: b = dk^2 sum_k C[k] e^{+2 pi i k.x / G}
      (the C2R convention drops the imaginary parts of self-conjugate columns).
  P7  fftshift and P8 restriction to the N x N output grid:
      out[p][q] = b[(p - N/2) mod G][(q - N/2) mod G]. Because n dt = N d = 2
      the inverse-DFT pitch equals the pixel pitch, so P8 needs no resampling.
"""
from __future__ import annotations

import numpy as np
from scipy.special import i0 as bessel_i0

from .geometry import Geometry

KAPPA = 4.0 * np.arcsinh(1.0)


class Params:
    def __init__(self, pad_radial: int = 2, pad_cart: int = 2, filter: str = "ramp",
                 taper: str = "deapod", beta: float = 8.0):
        assert filter in ("ramp", "none")
        assert taper in ("deapod", "none", "kb")
        self.P_r = int(pad_radial)
        self.P_c = int(pad_cart)
        self.filter = filter
        self.taper = taper
        self.beta = float(beta)


def sizes(geom: Geometry, prm: Params):
    M = prm.P_r * geom.n
    G = prm.P_c * geom.N
    dsig = 1.0 / (M * geom.dt)
    dk = 1.0 / (G * geom.d)
    return M, G, dsig, dk


# P1 ---------------------------------------------------------------------------
def taper(geom: Geometry, prm: Params) -> np.ndarray:
    M, _, dsig, _ = sizes(geom, prm)
    t = geom.t()
    if prm.taper == "deapod":
        return 1.0 / np.sinc(t * dsig) ** 2  # np.sinc(x) = sin(pi x) / (pi x)
    if prm.taper == "none":
        return np.ones_like(t)
    return bessel_i0(prm.beta * np.sqrt(np.clip(1.0 - t * t, 0.0, None))) / bessel_i0(prm.beta)


# P2 ---------------------------------------------------------------------------
def pad(y: np.ndarray, M: int) -> np.ndarray:
    V, n = y.shape
    z = np.zeros((V, M))
    z[:, (np.arange(n) - n // 2) % M] = y
    return z


# P3 ---------------------------------------------------------------------------
def transform(z: np.ndarray, dt: float) -> np.ndarray:
    return dt * np.fft.rfft(z, axis=-1)


# P4 ---------------------------------------------------------------------------
def radial_weights(M: int, dt: float, filter: str) -> np.ndarray:
    m = np.arange(M // 2 + 1, dtype=np.float64)
    if filter == "ramp":
        K = np.ones_like(m)
    else:
        K = np.zeros_like(m)
        K[1:] = (M * dt) / m[1:]  # 1 / sigma_m
    K[M // 2] = 0.0
    return K


# P5 ---------------------------------------------------------------------------
def gather(Yh: np.ndarray, Y0: np.ndarray, geom: Geometry, prm: Params) -> np.ndarray:
    """Cartesian half-plane spectrum C[b][a], b in FFT order over G rows, a in [0, G/2]."""
    if not geom.uniform:
        raise NotImplementedError("the BST oracle takes uniform angles theta_j = j pi / V")
    M, G, _, dk = sizes(geom, prm)
    V = geom.V
    # radial samples past the data are zero: extend with zeros to cover |k| up to the corner
    ext = np.zeros((V, M + 4), dtype=np.complex128)
    ext[:, :M // 2 + 1] = Yh
    ext[:, M // 2:] = 0.0

    a = np.arange(G // 2 + 1, dtype=np.float64)[None, :]
    b = np.arange(G, dtype=np.float64)
    b = np.where(b < G // 2, b, b - G)[:, None]
    r = np.sqrt(a * a + b * b) * (prm.P_r / prm.P_c)
    phi = np.arctan2(b, a) + 0.0 * a  # in [-pi/2, pi/2]
    lower = phi < 0.0
    theta = np.where(lower, phi + np.pi, phi)
    q = theta * (V / np.pi)
    j0 = np.floor(q)
    f = q - j0
    j0 = j0.astype(np.int64)
    over = j0 >= V  # rounding guard: theta == pi
    j0 = np.where(over, V - 1, j0)
    f = np.where(over, 1.0, f)
    j1 = j0 + 1
    wrap = j1 == V
    j1 = np.where(wrap, 0, j1)
    c0 = lower
    c1 = lower ^ wrap
    m0 = np.floor(r)
    g = r - m0
    m0 = np.minimum(m0.astype(np.int64), M + 2)
    m1 = m0 + 1

    def S(j, m, conj):
        v = ext[j, m]
        return np.where(conj, np.conj(v), v)

    C = ((1 - f) * (1 - g) * S(j0, m0, c0) + (1 - f) * g * S(j0, m1, c0)
         + f * (1 - g) * S(j1, m0, c1) + f * g * S(j1, m1, c1))
    mean0 = np.mean(Y0)
    if prm.filter == "ramp":
        C[0, 0] = mean0
    else:
        C[0, 0] = (KAPPA / dk) * mean0
    return C


# P6 ---------------------------------------------------------------------------
def inverse(C: np.ndarray, G: int, dk: float) -> np.ndarray:
    return (dk * dk * G * G) * np.fft.irfft2(C, s=(G, G))


# P7 + P8 ------------------------------------------------------------------------
def shift_crop(full: np.ndarray, N: int) -> np.ndarray:
    G = full.shape[0]
    idx = (np.arange(N) - N // 2) % G
    return full[np.ix_(idx, idx)]


def spectrum(sino: np.ndarray, geom: Geometry, prm: Params):
    """Steps P0-P4 for one slice: (Yh [V][M/2+1] complex, Y0 = Y_j[0] real [V])."""
    y = np.asarray(sino, dtype=np.float64)
    assert y.shape == (geom.V, geom.n)
    M, _, _, _ = sizes(geom, prm)
    z = pad(y * taper(geom, prm)[None, :], M)
    Y = transform(z, geom.dt)
    Yh = Y * radial_weights(M, geom.dt, prm.filter)[None, :]
    return Yh, Y[:, 0].real.copy()


def backproject(sino: np.ndarray, geom: Geometry, prm: Params = None) -> np.ndarray:
    """BST backprojection of one sinogram [V][n] -> image [N][N], FP64."""
    prm = prm or Params()
    M, G, _, dk = sizes(geom, prm)
    Yh, Y0 = spectrum(sino, geom, prm)
    C = gather(Yh, Y0, geom, prm)
    return shift_crop(inverse(C, G, dk), geom.N)


def backproject_batch(sinos: np.ndarray, geom: Geometry, prm: Params = None) -> np.ndarray:
    return np.stack([backproject(s, geom, prm) for s in sinos])
