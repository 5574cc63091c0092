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
      Kaiser-Bessel window without parameters; 'kb' and 'none' are options;
      'keys' is 1 / Khat(t_i dsigma), the de-apodiser of cubic radial
      interpolation, Khat the Fourier transform of the Keys kernel).
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
      radial samples m >= M/2 are zero. The paper asks only for "an
      interpolation"; the option interp='keys' replaces the linear radial
      weights by the Keys cubic convolution kernel (a = -1/2) over samples
      m0-1 .. m0+2 (sample -1 is conj Yh[1], since Yh(-sigma) = conj Yh(sigma)),
      keeping linear interpolation in angle. The option angular='tent'
      widens the angular kernel where the polar grid is denser in angle than
      the Cartesian one: a tent of half-width h = max(1, V / (pi rho)) angle
      steps (rho = |k| / dk, the point's radius in Cartesian steps), its
      weights normalised to sum 1, so each Cartesian point averages the polar
      angles across its own cell (h = 1 is the bilinear rule; uniform angles
      only). The transpose of this gather then deposits every polar sample
      over the Cartesian cells it covers, which makes the adjoint projector
      a close Radon approximation. The origin takes its own rule:
      RAMP: mean_j Y_j[0]; NONE: (kappa / dk) mean_j Y_j[0], kappa = 4 asinh(1),
      the average of 1/|k| over the origin cell times dk. The Nyquist column
      a = G/2 is set to zero (like the radial Nyquist sample in P4).
      Non-uniform angles (strictly increasing in [0, pi)): the angle sequence
      is continued with period pi (theta_{j+V} = theta_j + pi, conjugated
      sample), j0 is the last angle <= theta in it and f the fraction of the
      bracketing gap, so below theta_0 the j0 neighbour is theta_{V-1} - pi.
  P6  2D inverse DFT over the Hermitian plane: b = dk^2 sum_k C[k] e^{+2 pi i k.x / G}
      (the C2R convention drops the imaginary parts of self-conjugate columns).
  P7  fftshift and P8 restriction to the N x N output grid:
      out[p][q] = b[(p - N/2) mod G][(q - N/2) mod G]. Because n dt = N d = 2
      the inverse-DFT pitch equals the pixel pitch, so P8 needs no resampling.

Monopole subtraction (option of plain B, for the origin artifacts that Section 2
attributes to the sinogram not vanishing at t = 0): B y has a slowly decaying
tail ~ (mass)/|x| whose periodic images on the G-point grid the origin rule can
only approximate. With phi(t) the unit-mass Gaussian of width s centred on the
rotation axis (t = beta dt) and m = mean_j sum_i y[j][i] / sum_i phi(t_i),
  B y = B (y - m phi) + m b_phi,   b_phi(u) = int_0^pi phi(u . xi_theta) dtheta
                                             = (pi / (sqrt(2 pi) s)) e^{-rho} I0(rho),
rho = |u|^2 / (4 s^2) (from int_0^pi exp(-a cos^2 theta) dtheta = pi e^{-a/2} I0(a/2)).
The BST steps run on the residual y - m phi, whose mean projection mass is
zero, and m b_phi is added to the image in closed form.
"""
from __future__ import annotations

import numpy as np
from scipy.special import i0 as bessel_i0
from scipy.special import i0e as bessel_i0e

from .geometry import Geometry

KAPPA = 4.0 * np.arcsinh(1.0)


APODIZATIONS = ("ramlak", "shepp", "hann", "cosine")
INTERPS = ("linear", "keys")
ANGULARS = ("linear", "tent")


class Params:
    """Plan parameters. `apod` is the low-pass window A(sigma) multiplying the
    radial weight (the filtering stage F of Section 3 is named "low-pass");
    `center_shift` is a known rotation-axis offset beta in detector bins: the
    measured sinogram is y(t - beta dt, theta) (Section 1, centering), undone in
    P4 by the phase exp(+2 pi i sigma beta dt). `interp` is the radial
    interpolation of P5: 'linear' or 'keys' (cubic convolution). `monopole` is
    the width s of the subtracted Gaussian (plain B only; 0 = off), in the
    units of t (the detector spans [-1, 1)). `angular` is the angular kernel
    of P5: 'linear', or 'tent' (widened at small radii; with linear radial
    interpolation and uniform angles)."""

    def __init__(self, pad_radial: int = 2, pad_cart: int = 2, filter: str = "ramp",
                 taper: str = "deapod", beta: float = 8.0, apod: str = "ramlak",
                 center_shift: float = 0.0, interp: str = "linear", monopole: float = 0.0,
                 angular: str = "linear"):
        assert filter in ("ramp", "none")
        assert angular in ANGULARS and (angular == "linear" or interp == "linear")
        assert monopole >= 0.0 and (monopole == 0.0 or filter == "none")
        assert taper in ("deapod", "none", "kb", "keys")
        assert apod in APODIZATIONS
        assert interp in INTERPS
        self.P_r = int(pad_radial)
        self.P_c = int(pad_cart)
        self.filter = filter
        self.taper = taper
        self.beta = float(beta)
        self.apod = apod
        self.center_shift = float(center_shift)
        self.interp = interp
        self.monopole = float(monopole)
        self.angular = angular


def sizes(geom: Geometry, prm: Params):
    M = prm.P_r * geom.n
    G = prm.P_c * geom.N
    dsig = 1.0 / (M * geom.dt)
    dk = 1.0 / (G * geom.d)
    return M, G, dsig, dk


# Keys cubic convolution kernel, a = -1/2 (Keys 1981): the interpolant
# sum_k c_k W(x - k) passes through the samples and reproduces quadratics.
KEYS_A = -0.5


def keys_kernel(x: np.ndarray) -> np.ndarray:
    a = KEYS_A
    x = np.abs(np.asarray(x, dtype=np.float64))
    inner = (a + 2.0) * x ** 3 - (a + 3.0) * x ** 2 + 1.0
    outer = a * x ** 3 - 5.0 * a * x ** 2 + 8.0 * a * x - 4.0 * a
    return np.where(x <= 1.0, inner, np.where(x < 2.0, outer, 0.0))


def keys_weights(frac: np.ndarray):
    """Weights of samples m0-1, m0, m0+1, m0+2 for a point at m0 + frac."""
    return (keys_kernel(1.0 + frac), keys_kernel(frac), keys_kernel(1.0 - frac), keys_kernel(2.0 - frac))


def keys_ft(nu: np.ndarray) -> np.ndarray:
    """Khat(nu) = int W(x) exp(-2 pi i nu x) dx for a = -1/2, in closed form:
    sinc^3(nu) (3 sinc(nu) - 2 cos(pi nu)), sinc(nu) = sin(pi nu) / (pi nu)."""
    nu = np.asarray(nu, dtype=np.float64)
    s = np.sinc(nu)
    return s ** 3 * (3.0 * s - 2.0 * np.cos(np.pi * nu))


# P1 ---------------------------------------------------------------------------
def taper(geom: Geometry, prm: Params) -> np.ndarray:
    M, _, dsig, _ = sizes(geom, prm)
    t = geom.t()
    if prm.taper == "deapod":
        return 1.0 / np.sinc(t * dsig) ** 2  # np.sinc(x) = sin(pi x) / (pi x)
    if prm.taper == "keys":
        return 1.0 / keys_ft(t * dsig)
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
def apodization(x: np.ndarray, apod: str) -> np.ndarray:
    """Window A at x = sigma / sigma_Nyquist in [0, 1]."""
    if apod == "ramlak":
        return np.ones_like(x)
    if apod == "shepp":
        return np.sinc(x / 2.0)          # sin(pi x/2) / (pi x/2)
    if apod == "hann":
        return 0.5 * (1.0 + np.cos(np.pi * x))
    return np.cos(np.pi * x / 2.0)       # cosine


def radial_weights(M: int, dt: float, filter: str, apod: str = "ramlak") -> np.ndarray:
    m = np.arange(M // 2 + 1, dtype=np.float64)
    if filter == "ramp":
        K = np.ones_like(m)
    else:
        K = np.zeros_like(m)
        K[1:] = (M * dt) / m[1:]  # 1 / sigma_m
    K = K * apodization(2.0 * m / M, apod)
    K[M // 2] = 0.0
    return K


def shift_phase(M: int, dt: float, center_shift: float) -> np.ndarray:
    """exp(+2 pi i sigma_m beta dt), m = 0..M/2, sigma_m = m / (M dt)."""
    m = np.arange(M // 2 + 1, dtype=np.float64)
    return np.exp(2j * np.pi * m * center_shift / M)


def normalize(counts: np.ndarray, flat: np.ndarray, dark: np.ndarray) -> np.ndarray:
    """Flat/dark correction of Section 1: y = -log((I - D) / (I0 - D))."""
    c = np.asarray(counts, dtype=np.float64)
    return -np.log((c - dark) / (flat - dark))


# P5 ---------------------------------------------------------------------------
def angle_bracket(theta: np.ndarray, geom: Geometry):
    """For directions theta in [0, pi): (j0, j1, f, flip0, flip1): the bracketing
    angle indices in the period-pi continuation of the angle sequence, the
    fraction of the gap and whether each neighbour is a conjugated image
    (theta_j - pi below the first angle, theta_j + pi past the last)."""
    V = geom.V
    if geom.uniform:
        q = theta * (V / np.pi)
        j0 = np.floor(q)
        f = q - j0
        j0 = j0.astype(np.int64)
        over = j0 >= V  # rounding guard: theta == pi
        j0 = np.where(over, V - 1, j0)
        f = np.where(over, 1.0, f)
        flip0 = np.zeros(theta.shape, dtype=bool)
    else:
        th = geom.theta
        k = np.searchsorted(th, theta, side="right") - 1  # last theta_j <= theta, -1 below theta_0
        flip0 = k < 0
        j0 = np.where(flip0, V - 1, k)
        lo = np.where(flip0, th[V - 1] - np.pi, th[j0])
        hi = np.where(j0 + 1 < V, th[np.minimum(j0 + 1, V - 1)], th[0] + np.pi)
        hi = np.where(flip0, th[0], hi)
        f = (theta - lo) / (hi - lo)
    j1 = j0 + 1
    wrap = j1 == V
    j1 = np.where(wrap, 0, j1)
    flip1 = wrap & ~flip0
    return j0, j1, f, flip0, flip1


def tent_taps(theta: np.ndarray, rho: np.ndarray, V: int):
    """Angular taps of the tent rule for directions theta in [0, pi) at
    Cartesian radii rho (flat arrays): (p, j, flip, w) flat arrays, one entry
    per nonzero tap of point p; j in [0, V), flip marking taps taken from the
    continuation past pi or below 0 (the conjugated images theta_j +- pi);
    weights (1 - |q - j| / h)+ with q = theta V / pi, h = max(1, V / (pi rho)),
    normalised to sum 1. Points with h = 1 get the two bilinear taps. (rho is
    at least 1 off the origin, which has its own rule; it is clamped there.)"""
    q = theta * (V / np.pi)
    h = np.maximum(1.0, V / (np.pi * np.maximum(rho, 1.0)))
    ps, js, ws = [], [], []
    idx = np.arange(q.size)
    narrow = h <= 1.0
    # h = 1: the bilinear taps floor(q), floor(q) + 1
    qn = q[narrow]
    j0 = np.floor(qn)
    f = qn - j0
    for jc, w in ((j0, 1.0 - f), (j0 + 1.0, f)):
        ps.append(idx[narrow]); js.append(jc.astype(np.int64)); ws.append(w)
    # h > 1: every integer j with |q - j| < h
    wide = ~narrow
    if np.any(wide):
        qw, hw, pw = q[wide], h[wide], idx[wide]
        lo = np.floor(qw - hw).astype(np.int64)
        # taps lo .. lo + span - 1 cover |q - j| < h; points sorted by span, so
        # step k only visits the points that still have a tap there
        span = np.ceil(2.0 * hw).astype(np.int64) + 2
        order = np.argsort(-span, kind="stable")
        qw, hw, pw, lo, span = qw[order], hw[order], pw[order], lo[order], span[order]
        raw = []
        total = np.zeros(qw.size)
        for k in range(int(span[0])):
            n_act = int(np.searchsorted(-span, -k, side="left"))  # points with span > k
            jc = lo[:n_act] + k
            w = np.maximum(0.0, 1.0 - np.abs(qw[:n_act] - jc) / hw[:n_act])
            raw.append((n_act, jc, w))
            total[:n_act] += w
        for n_act, jc, w in raw:
            ps.append(pw[:n_act]); js.append(jc); ws.append(w / total[:n_act])
    p = np.concatenate(ps)
    jc = np.concatenate(js)
    w = np.concatenate(ws)
    ok = w != 0.0
    p, jc, w = p[ok], jc[ok], w[ok]
    flip = (np.floor_divide(jc, V) % 2) == 1
    return p, np.mod(jc, V), flip, w


def gather(Yh: np.ndarray, Y0: np.ndarray, geom: Geometry, prm: Params) -> np.ndarray:
    """Cartesian half-plane spectrum C[b][a], b in FFT order over G rows, a in [0, G/2]."""
    M, G, _, dk = sizes(geom, prm)
    V = geom.V
    if prm.angular == "tent":
        assert geom.uniform, "the tent angular rule is defined for uniform angles"
        C = np.zeros((G, G // 2 + 1), dtype=np.complex128)
        for bb, aa, jj, mm, ww, cc in _gather_stencil(geom, prm):
            v = Yh[jj, mm]
            np.add.at(C, (bb, aa), ww * np.where(cc, np.conj(v), v))
        mean0 = np.mean(Y0)
        C[0, 0] = mean0 if prm.filter == "ramp" else (KAPPA / dk) * mean0
        C[:, G // 2] = 0.0
        return C
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
    j0, j1, f, flip0, flip1 = angle_bracket(theta, geom)
    c0 = lower ^ flip0
    c1 = lower ^ flip1
    m0 = np.floor(r)
    g = r - m0
    m0 = np.minimum(m0.astype(np.int64), M + 2)
    m1 = m0 + 1

    def S(j, m, conj):
        # a sample at m < 0 is the conjugate of -m (the spectrum of a real line)
        neg = m < 0
        v = ext[j, np.where(neg, -m, m)]
        return np.where(conj ^ neg, np.conj(v), v)

    if prm.interp == "linear":
        C = ((1 - f) * (1 - g) * S(j0, m0, c0) + (1 - f) * g * S(j0, m1, c0)
             + f * (1 - g) * S(j1, m0, c1) + f * g * S(j1, m1, c1))
    else:
        C = np.zeros(r.shape, dtype=np.complex128)
        for off, wr in zip((-1, 0, 1, 2), keys_weights(g)):
            mm = np.minimum(m0 + off, M + 2)
            C += wr * ((1 - f) * S(j0, mm, c0) + f * S(j1, mm, c1))
    mean0 = np.mean(Y0)
    if prm.filter == "ramp":
        C[0, 0] = mean0
    else:
        C[0, 0] = (KAPPA / dk) * mean0
    # The Cartesian Nyquist column |k_x| = G/2 dk is dropped, as P4 drops the
    # radial Nyquist sample. With linear radial taps it is zero anyway (its
    # points lie at r >= M/2); the cubic taps reach one sample further in.
    C[:, G // 2] = 0.0
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
    W = radial_weights(M, geom.dt, prm.filter, prm.apod).astype(np.complex128)
    if prm.center_shift != 0.0:
        W = W * shift_phase(M, geom.dt, prm.center_shift)
    Yh = Y * W[None, :]
    return Yh, Y[:, 0].real.copy()


# Monopole subtraction (plain B) ------------------------------------------------
def monopole_profile(geom: Geometry, prm: Params) -> np.ndarray:
    """phi(t_i - beta dt): the unit-mass Gaussian of width s on the rotation axis."""
    s = prm.monopole
    t = geom.t() - prm.center_shift * geom.dt
    return np.exp(-t * t / (2.0 * s * s)) / (np.sqrt(2.0 * np.pi) * s)


def monopole_mass(sino: np.ndarray, geom: Geometry, prm: Params) -> float:
    """m = mean_j sum_i y[j][i] / sum_i phi(t_i - beta dt)."""
    y = np.asarray(sino, dtype=np.float64)
    return float(np.mean(y.sum(axis=1)) / monopole_profile(geom, prm).sum())


def monopole_image(geom: Geometry, prm: Params) -> np.ndarray:
    """b_phi on the output grid: (pi / (sqrt(2 pi) s)) e^{-rho} I0(rho), rho = |u|^2 / (4 s^2)."""
    s = prm.monopole
    u = geom.u()
    rho = (u[None, :] ** 2 + u[:, None] ** 2) / (4.0 * s * s)
    return (np.pi / (np.sqrt(2.0 * np.pi) * s)) * bessel_i0e(rho)


def backproject(sino: np.ndarray, geom: Geometry, prm: Params = None) -> np.ndarray:
    """BST backprojection of one sinogram [V][n] -> image [N][N], FP64."""
    prm = prm or Params()
    M, G, _, dk = sizes(geom, prm)
    y = np.asarray(sino, dtype=np.float64)
    if prm.monopole > 0.0:
        m = monopole_mass(y, geom, prm)
        y = y - m * monopole_profile(geom, prm)[None, :]
    Yh, Y0 = spectrum(y, geom, prm)
    C = gather(Yh, Y0, geom, prm)
    img = shift_crop(inverse(C, G, dk), geom.N)
    if prm.monopole > 0.0:
        img = img + m * monopole_image(geom, prm)
    return img


def backproject_batch(sinos: np.ndarray, geom: Geometry, prm: Params = None) -> np.ndarray:
    return np.stack([backproject(s, geom, prm) for s in sinos])


# ----------------------------------------------------------------------------
# Adjoint: the exact real-linear transpose of steps P1..P8, stage by stage.
#
# With the weighted inner products <f, f'> = d^2 sum f f' (images) and
# <g, g'> = dt sum_j w_j sum_i g g' (sinograms, w_j = pi/V for uniform angles),
# the projector R = (d^2 / dt) diag(1/w_j) B^T satisfies <R f, g> = <f, B g> exactly,
# mirroring B = R* of Section 1. With a plain-B plan R approximates the Radon
# transform (Eq. 1) through the Fourier-slice theorem: the Cartesian density
# of the transposed gather (~sigma) cancels the 1/sigma weight of P4.
# Transposes used (real-linear maps, complex values as pairs of reals):
#   crop            -> zero-embed
#   C2R inverse     -> forward 2D DFT with c_a = 1 for a in {0, G/2}, else 2,
#                      times dk^2
#   bilinear gather -> scatter-add with the same weights and conjugations;
#                      origin rule -> its factor times Re of the origin value,
#                      added to the unweighted DC of every projection
#   K[m]            -> K[m]
#   real DFT        -> dt * sum_m Re(X[m] e^{+2 pi i k m / M}), m = 0..M/2
#   pad             -> crop;  taper -> taper
# ----------------------------------------------------------------------------
def _gather_stencil(geom: Geometry, prm: Params):
    """Per Cartesian point (b, a) of the half plane: the (j, m, weight,
    conjugate) entries of P5 (two radial taps per angle neighbour, or four for
    the cubic option), as flat arrays; the origin and the Nyquist column
    (which have their own rules) and samples past the data are excluded, and
    a tap at m < 0 becomes the conjugated tap at -m."""
    M, G, _, _ = sizes(geom, prm)
    a = np.arange(G // 2 + 1, dtype=np.float64)[None, :]
    b = np.arange(G, dtype=np.float64)
    b = np.where(b < G // 2, b, b - G)[:, None]
    r = np.sqrt(a * a + b * b) * (prm.P_r / prm.P_c)
    phi = np.arctan2(b, a) + 0.0 * a
    lower = phi < 0.0
    theta = np.where(lower, phi + np.pi, phi)
    j0, j1, f, flip0, flip1 = angle_bracket(theta, geom)
    m0 = np.floor(r)
    g = r - m0
    m0 = m0.astype(np.int64)
    bb, aa = np.meshgrid(np.arange(G), np.arange(G // 2 + 1), indexing="ij")
    keep = ~((bb == 0) & (aa == 0)) & (aa < G // 2)
    if prm.interp == "linear":
        radial = ((0, 1 - g), (1, g))
    else:
        radial = tuple(zip((-1, 0, 1, 2), keys_weights(g)))
    entries = []
    if prm.angular == "tent":
        assert geom.uniform, "the tent angular rule is defined for uniform angles"
        rho = np.sqrt(a * a + b * b) + 0.0 * b
        pp, jj, fl, wa = tent_taps(theta.ravel(), rho.ravel(), geom.V)
        bbf, aaf, m0f, kf, lf = bb.ravel()[pp], aa.ravel()[pp], m0.ravel()[pp], keep.ravel()[pp], lower.ravel()[pp]
        for off, wr in radial:
            mm = m0f + off
            w = wa * wr.ravel()[pp]
            ok = kf & (mm < M // 2) & (w != 0.0)
            entries.append((bbf[ok], aaf[ok], jj[ok], mm[ok], w[ok], (lf ^ fl)[ok]))
        return entries
    for jj, wa, cc in ((j0, 1 - f, lower ^ flip0), (j1, f, lower ^ flip1)):
        for off, wr in radial:
            mm = m0 + off
            neg = mm < 0
            mm = np.where(neg, -mm, mm)
            ok = keep & (mm < M // 2) & (wa * wr != 0.0)
            entries.append((bb[ok], aa[ok], jj[ok], mm[ok], (wa * wr)[ok], (cc ^ neg)[ok]))
    return entries


def project(img: np.ndarray, geom: Geometry, prm: Params = None) -> np.ndarray:
    """R f = (d^2 / dt) diag(1 / w_j) B^T f for one image [N][N] -> sinogram
    [V][n], FP64 (w_j = pi/V for uniform angles, else half the neighbour gap)."""
    prm = prm or Params()
    f = np.asarray(img, dtype=np.float64)
    assert f.shape == (geom.N, geom.N)
    M, G, _, dk = sizes(geom, prm)
    V, n, N = geom.V, geom.n, geom.N
    # P8/P7 transpose: zero-embed at (p - N/2) mod G
    idx = (np.arange(N) - N // 2) % G
    full = np.zeros((G, G))
    full[np.ix_(idx, idx)] = f
    # P6 transpose
    ca = np.full(G // 2 + 1, 2.0)
    ca[0] = 1.0
    ca[G // 2] = 1.0
    Ct = (dk * dk) * np.fft.rfft2(full) * ca[None, :]       # [b][a]
    # P5 transpose: scatter-add, plus the origin rule
    Yh_t = np.zeros((V, M // 2 + 1), dtype=np.complex128)
    for bb, aa, jj, mm, ww, cc in _gather_stencil(geom, prm):
        v = Ct[bb, aa]
        v = np.where(cc, np.conj(v), v)
        np.add.at(Yh_t, (jj, mm), ww * v)
    # P4 transpose (a complex weight transposes to its conjugate)
    W = radial_weights(M, geom.dt, prm.filter, prm.apod).astype(np.complex128)
    if prm.center_shift != 0.0:
        W = W * shift_phase(M, geom.dt, prm.center_shift)
    Y_t = Yh_t * np.conj(W)[None, :]
    dc_rule = 1.0 if prm.filter == "ramp" else KAPPA / dk
    Y_t[:, 0] += (dc_rule / V) * Ct[0, 0].real
    # P3 transpose: dt * sum_m Re(X[m] e^{+2 pi i k m/M}) over m = 0..M/2
    X = np.zeros((V, M), dtype=np.complex128)
    X[:, :M // 2 + 1] = Y_t
    z_t = geom.dt * M * np.fft.ifft(X, axis=-1).real
    # P2 transpose (crop) and P1 (taper)
    y_t = z_t[:, (np.arange(n) - n // 2) % M] * taper(geom, prm)[None, :]
    return (geom.d ** 2 / geom.dt) * y_t / geom.w[:, None]
