"""Pins for the FP64 BST oracle (Section 2, Eq. 3, steps P0-P8). CPU only.

- literal DFT sums and per-point gathering at tiny sizes (bst_naive);
- exact symmetries of the discrete method: 90 and 180 degree rotation, mirror;
- closed forms: FBP of an analytic Gaussian returns the Gaussian (RAMP);
  y = cos(2 pi s0 t) backprojects to pi J0(2 pi s0 |u|) and a Gaussian's
  sinogram to pi sqrt(2 pi) s e^{-z} I0(z), z = r^2/4s^2 (NONE);
- the taper options reduce to each other where they must;
- the projector is the exact adjoint: weighted inner-product identity and the
  transpose of the literal-sum backprojection's dense matrix.
"""
import math

import numpy as np
import pytest
from scipy.special import i0e, j0

import synth
from oracle import bst, bst_naive
from oracle.bruteforce import inner_image, inner_sino
from oracle.geometry import Geometry


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("N,V", [(8, 6), (16, 8), (16, 5)])
@pytest.mark.parametrize("filt", ["ramp", "none"])
@pytest.mark.parametrize("P_r,P_c", [(2, 2), (1, 2), (2, 1), (4, 2)])
def test_fft_oracle_equals_literal_sums(N, V, filt, P_r, P_c):
    rng = np.random.default_rng(N * 7 + V)
    g = Geometry(N, V, N)
    y = rng.standard_normal((V, N))
    a = bst.backproject(y, g, bst.Params(P_r, P_c, filt))
    b = bst_naive.backproject(y, g, P_r, P_c, filt)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))


def _edge_free(rng, V, n):
    y = rng.standard_normal((V, n))
    y[:, 0] = 0.0  # bin 0 (t = -1) has no mirror bin at t = +1
    return y


@pytest.mark.parametrize("filt", ["ramp", "none"])
@pytest.mark.parametrize("N,V", [(32, 24), (64, 40)])
def test_rotation_by_90_degrees(filt, N, V):
    rng = np.random.default_rng(N + V)
    g = Geometry(N, V, N)
    y = _edge_free(rng, V, N)
    h = V // 2
    yr = np.zeros_like(y)
    yr[h:] = y[:h]
    yr[:h, 1:] = y[h:, :0:-1]  # theta - pi/2 < 0: read theta + pi/2 with t reversed
    prm = bst.Params(2, 2, filt)
    b = bst.backproject(y, g, prm)
    br = bst.backproject(yr, g, prm)
    # b'(u1, u2) = b(u2, -u1): b'[p][q] = b[N - q][p]
    expect = b[N - np.arange(1, N)][:, :].T  # [p][q-1] = b[N-q][p]
    assert np.max(np.abs(br[:, 1:] - expect)) <= 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("filt", ["ramp", "none"])
def test_rotation_by_180_degrees(filt):
    rng = np.random.default_rng(5)
    N, V = 32, 21
    g = Geometry(N, V, N)
    y = _edge_free(rng, V, N)
    yr = np.zeros_like(y)
    yr[:, 1:] = y[:, :0:-1]
    prm = bst.Params(2, 2, filt)
    b = bst.backproject(y, g, prm)
    br = bst.backproject(yr, g, prm)
    assert np.max(np.abs(br[1:, 1:] - b[:0:-1, :0:-1])) <= 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("filt", ["ramp", "none"])
def test_mirror_u1(filt):
    rng = np.random.default_rng(6)
    N, V = 32, 19
    g = Geometry(N, V, N)
    y = _edge_free(rng, V, N)
    ym = np.zeros_like(y)
    ym[1:] = y[:0:-1]  # theta -> pi - theta
    ym[0, 1:] = y[0, :0:-1]  # theta = 0 maps to pi: t reversed
    prm = bst.Params(2, 2, filt)
    b = bst.backproject(y, g, prm)
    bm = bst.backproject(ym, g, prm)
    assert np.max(np.abs(bm[:, 1:] - b[:, :0:-1])) <= 1e-12 * np.max(np.abs(b))


def test_linearity():
    rng = np.random.default_rng(8)
    g = Geometry(32, 30, 32)
    y1 = rng.standard_normal((30, 32))
    y2 = rng.standard_normal((30, 32))
    for filt in ("ramp", "none"):
        prm = bst.Params(2, 2, filt)
        lhs = bst.backproject(2.5 * y1 - 0.5 * y2, g, prm)
        rhs = 2.5 * bst.backproject(y1, g, prm) - 0.5 * bst.backproject(y2, g, prm)
        assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(rhs))


def _gauss_case(N, gs):
    sg = synth.Geometry(N, N, N)
    return (synth.gaussian_sinogram(sg, gs).numpy(), synth.gaussian_image(sg, gs).numpy(),
            Geometry(N, N, N))


def test_fbp_of_gaussian_recovers_it_and_converges_with_padding():
    gs = synth.Gaussian(0.2, -0.1, 0.1)
    y, x, g = _gauss_case(128, gs)
    e22 = _rel(bst.backproject(y, g, bst.Params(2, 2, "ramp")), x)
    e44 = _rel(bst.backproject(y, g, bst.Params(4, 4, "ramp")), x)
    e88 = _rel(bst.backproject(y, g, bst.Params(8, 4, "ramp")), x)
    assert e22 < 5e-3
    assert e44 < e22 / 3
    assert e88 < e44
    # the same Gaussian moved elsewhere: no transposed axis or flipped sign survives
    gs2 = synth.Gaussian(-0.3, 0.25, 0.07)
    y2, x2, _ = _gauss_case(128, gs2)
    assert _rel(bst.backproject(y2, g, bst.Params(2, 2, "ramp")), x2) < 1e-2


def test_fbp_independent_of_detector_count():
    # dsigma and dk depend only on the field of view, so the discretisation error
    # of a well-resolved Gaussian is the same at every N (not a resolution effect).
    gs = synth.Gaussian(0.1, 0.1, 0.1)
    errs = []
    for N in (64, 128, 256):
        y, x, g = _gauss_case(N, gs)
        errs.append(_rel(bst.backproject(y, g), x))
    assert max(errs) - min(errs) < 2e-4


def test_deapodising_taper_reduces_error():
    gs = synth.Gaussian(0.2, -0.1, 0.1)
    y, x, g = _gauss_case(128, gs)
    e_deapod = _rel(bst.backproject(y, g, bst.Params(2, 2, "ramp", "deapod")), x)
    e_none = _rel(bst.backproject(y, g, bst.Params(2, 2, "ramp", "none")), x)
    assert e_deapod < 0.6 * e_none


def test_kaiser_bessel_with_zero_beta_is_no_taper():
    rng = np.random.default_rng(2)
    g = Geometry(32, 16, 32)
    y = rng.standard_normal((16, 32))
    a = bst.backproject(y, g, bst.Params(2, 2, "ramp", "kb", 0.0))
    b = bst.backproject(y, g, bst.Params(2, 2, "ramp", "none"))
    assert np.max(np.abs(a - b)) < 1e-13 * np.max(np.abs(b))
    w = bst.taper(g, bst.Params(2, 2, "ramp", "kb", 6.0))
    assert abs(w[g.n // 2] - 1.0) < 1e-15 and np.all(np.diff(w[g.n // 2:]) < 0)


def _i0_series(x):
    """I0(x) = sum_k (x/2)^(2k) / (k!)^2, summed term by term (independent of
    the library routine the oracle calls)."""
    return math.fsum((x / 2.0) ** (2 * k) / math.factorial(k) ** 2 for k in range(80))


def test_kaiser_bessel_taper_closed_form():
    # P1 option: w(t) = I0(beta sqrt(1 - t^2)) / I0(beta); at the detector edge
    # t = -1 (bin 0) it is 1 / I0(beta), at t = 0 it is 1, and in between the
    # square root sits inside the Bessel argument (not 1 - t^2 itself)
    beta = 6.0
    g = Geometry(64, 16, 64)
    w = bst.taper(g, bst.Params(2, 2, "ramp", "kb", beta))
    t = g.t()
    assert t[0] == -1.0
    assert abs(w[0] - 1.0 / _i0_series(beta)) <= 1e-14
    assert abs(w[g.n // 2] - 1.0) <= 1e-15
    for i in (3, 17, 29, 50):
        expect = _i0_series(beta * math.sqrt(1.0 - t[i] ** 2)) / _i0_series(beta)
        assert abs(w[i] - expect) <= 1e-13 * expect, (i, w[i], expect)
    # the wrong reading I0(beta (1 - t^2)) differs by far more than that
    i = 17
    wrong = _i0_series(beta * (1.0 - t[i] ** 2)) / _i0_series(beta)
    assert abs(w[i] - wrong) > 1e-3


# A(x) at x = sigma / sigma_Nyquist = 0, 1/3, 1/2, 1, written out from the
# window definitions: Shepp-Logan sin(pi x/2)/(pi x/2), Hann (1 + cos pi x)/2,
# cosine cos(pi x/2).
_WINDOW_VALUES = {
    "ramlak": (1.0, 1.0, 1.0, 1.0),
    "shepp": (1.0, 3.0 / math.pi, 2.0 * math.sqrt(2.0) / math.pi, 2.0 / math.pi),
    "hann": (1.0, 0.75, 0.5, 0.0),
    "cosine": (1.0, math.sqrt(3.0) / 2.0, math.sqrt(2.0) / 2.0, 0.0),
}


@pytest.mark.parametrize("apod", sorted(_WINDOW_VALUES))
def test_apodization_windows_closed_form(apod):
    x = np.array([0.0, 1.0 / 3.0, 0.5, 1.0])
    got = bst.apodization(x, apod)
    assert np.max(np.abs(got - np.array(_WINDOW_VALUES[apod]))) <= 1e-15


@pytest.mark.parametrize("apod", sorted(_WINDOW_VALUES))
@pytest.mark.parametrize("filt", ["ramp", "none"])
def test_radial_weights_carry_the_window(apod, filt):
    # P4: K[m] A(2m/M); RAMP K = 1, plain B K = 1/sigma_m = M dt / m, K[0] = 0
    # there, and the Nyquist sample M/2 is dropped in both modes
    M, dt = 96, 2.0 / 48
    K = bst.radial_weights(M, dt, filt, apod)
    A = _WINDOW_VALUES[apod]
    for m, a in ((M // 6, A[1]), (M // 4, A[2])):
        base = 1.0 if filt == "ramp" else M * dt / m
        assert abs(K[m] - base * a) <= 1e-14 * base
    assert K[M // 2] == 0.0
    assert K[0] == (1.0 if filt == "ramp" else 0.0)


def test_fbp_of_uniform_disk_level():
    N = 128
    sg = synth.Geometry(N, N, N)
    g = Geometry(N, N, N)
    y = synth.ellipse_sinogram(sg, [synth.Ellipse(0.05, -0.05, 0.5, 0.4, 0.3, 1.0)]).numpy()
    r = bst.backproject(y, g)
    u = g.u()
    inner = np.hypot(u[None, :] - 0.05, u[:, None] + 0.05) < 0.3
    outer = np.hypot(u[None, :], u[:, None]) > 0.7
    assert abs(np.mean(r[inner]) - 1.0) < 5e-3
    assert abs(np.mean(r[outer])) < 5e-3


def test_plain_backprojection_of_cosine_is_bessel():
    s0 = 4.0  # 2 s0 integer: the cosine has zero mean over [-1, 1), so the origin rule is idle
    N = 128
    g = Geometry(N, N, N)
    y = np.tile(np.cos(2 * np.pi * s0 * g.t()), (N, 1))
    u = g.u()
    R = np.hypot(u[None, :], u[:, None])
    disk = R <= 0.9
    ex = np.pi * j0(2 * np.pi * s0 * R)
    e2 = _rel(bst.backproject(y, g, bst.Params(2, 2, "none"))[disk], ex[disk])
    e4 = _rel(bst.backproject(y, g, bst.Params(2, 4, "none"))[disk], ex[disk])
    assert e2 < 3e-2
    assert e4 < e2 / 1.5  # periodisation error falls with Cartesian padding


def test_plain_backprojection_of_gaussian_closed_form():
    gs = synth.Gaussian(0.1, 0.05, 0.08)
    N = 128
    y, _, g = _gauss_case(N, gs)
    u = g.u()
    r = np.hypot(u[None, :] - gs.cx, u[:, None] - gs.cy)
    ex = np.pi * math.sqrt(2 * math.pi) * gs.s * i0e(r * r / (4 * gs.s ** 2))
    disk = np.hypot(u[None, :], u[:, None]) <= 0.9
    b = bst.backproject(y, g, bst.Params(2, 2, "none"))
    assert _rel(b[disk], ex[disk]) < 2e-2


# --- the adjoint (projector) -------------------------------------------------


@pytest.mark.parametrize("N,V,P_r,P_c,filt", [(16, 12, 2, 2, "ramp"), (32, 21, 1, 2, "none"),
                                              (64, 50, 2, 1, "ramp"), (32, 24, 4, 2, "none"),
                                              (64, 64, 2, 4, "ramp")])
def test_project_is_the_adjoint(N, V, P_r, P_c, filt):
    # <R f, g> = <f, B g> under the weighted inner products (B = R*, Section 1)
    rng = np.random.default_rng(N + V + P_r)
    g = Geometry(N, V, N)
    prm = bst.Params(P_r, P_c, filt)
    f = rng.standard_normal((N, N))
    y = rng.standard_normal((V, N))
    lhs = inner_sino(bst.project(f, g, prm), y, g)
    rhs = inner_image(f, bst.backproject(y, g, prm), g)
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


@pytest.mark.parametrize("filt", ["ramp", "none"])
def test_project_equals_transpose_of_literal_backprojection(filt):
    # dense matrix of the literal-sum backprojection at a tiny size, transposed
    N, V = 8, 6
    g = Geometry(N, V, N)
    cols = []
    for k in range(V * N):
        e = np.zeros(V * N)
        e[k] = 1.0
        cols.append(bst_naive.backproject(e.reshape(V, N), g, 2, 2, filt).ravel())
    Bmat = np.stack(cols, axis=1)  # [N*N][V*N]
    rng = np.random.default_rng(4)
    f = rng.standard_normal((N, N))
    scale = g.d ** 2 / (g.dt * np.pi / V)
    expect = scale * (Bmat.T @ f.ravel()).reshape(V, N)
    got = bst.project(f, g, bst.Params(2, 2, filt))
    assert np.max(np.abs(got - expect)) <= 1e-12 * np.max(np.abs(expect))


# --- pre-processing stages folded into P1/P4: apodised ramp, centre shift, flat/dark ---

def _smooth_gauss(N, s=0.03):
    sg = synth.Geometry(N, N, N)
    gs = synth.Gaussian(0.1, -0.2, s)
    return sg, gs, synth.gaussian_sinogram(sg, gs).numpy()


@pytest.mark.parametrize("apod", ["shepp", "hann", "cosine"])
def test_apodised_ramp_equals_prefiltered_sinogram(apod):
    # K[m] = A(sigma_m / sigma_Nyq) in P4 is the same as filtering every
    # projection by A(|sigma|) first (done here with a long zero-padded FFT)
    N = 128
    g = Geometry(N, N, N)
    _, _, y = _smooth_gauss(N)
    L = 8 * N
    x = np.arange(L // 2 + 1) / (L * g.dt) * (2 * g.dt)
    A = bst.apodization(np.minimum(x, 1.0), apod) * (x < 1.0)
    yf = np.fft.irfft(np.fft.rfft(y, L, axis=1) * A, L, axis=1)[:, :N]
    a = bst.backproject(yf, g, bst.Params(apod="ramlak"))
    b = bst.backproject(y, g, bst.Params(apod=apod))
    c = bst.backproject(y, g, bst.Params(apod="ramlak"))
    assert _rel(a, b) < 1e-3
    assert _rel(c, b) > 1e-2


@pytest.mark.parametrize("filt", ["ramp", "none"])
@pytest.mark.parametrize("shift", [3, -5])
def test_integer_centre_shift_is_exact(filt, shift):
    # a sinogram measured with the axis k bins off, y_m[i] = y[i - k]: with no
    # taper (which is not shift invariant) the phase ramp undoes the shift exactly
    rng = np.random.default_rng(10 + shift)
    N, V = 64, 40
    g = Geometry(N, V, N)
    y = np.zeros((V, N))
    y[:, 8:N - 8] = rng.standard_normal((V, N - 16))
    ym = np.roll(y, shift, axis=1)
    a = bst.backproject(y, g, bst.Params(2, 2, filt, "none"))
    b = bst.backproject(ym, g, bst.Params(2, 2, filt, "none", center_shift=shift))
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(a))


def test_fractional_centre_shift_of_analytic_sinogram():
    import torch
    N = 128
    g = Geometry(N, N, N)
    sg, gs, y = _smooth_gauss(N, 0.08)
    beta = 3.37
    t = sg.t()[None, :] - beta * sg.dt
    th = sg.theta()[:, None]
    sc = t - (gs.cx * torch.cos(th) + gs.cy * torch.sin(th))
    ym = (math.sqrt(2 * math.pi) * gs.s * torch.exp(-sc * sc / (2 * gs.s ** 2))).numpy()
    a = bst.backproject(y, g)
    assert _rel(bst.backproject(ym, g, bst.Params(center_shift=beta)), a) < 1e-2
    assert _rel(bst.backproject(ym, g, bst.Params(center_shift=-beta)), a) > 0.3


def test_flat_dark_normalisation_inverts_lambert_beer():
    # I = D + (I0 - D) exp(-y)  =>  -log((I - D)/(I0 - D)) = y
    rng = np.random.default_rng(12)
    y = rng.uniform(0.0, 3.0, (20, 32))
    flat = rng.uniform(900.0, 1100.0, 32)
    dark = rng.uniform(5.0, 20.0, 32)
    counts = dark + (flat - dark) * np.exp(-y)
    assert np.max(np.abs(bst.normalize(counts, flat, dark) - y)) < 1e-12


def test_adjoint_with_shift_and_apodisation():
    rng = np.random.default_rng(13)
    N, V = 64, 48
    g = Geometry(N, V, N)
    f = rng.standard_normal((N, N))
    y = rng.standard_normal((V, N))
    for prm in (bst.Params(center_shift=2.5, apod="hann"),
                bst.Params(filter="none", center_shift=-1.25, apod="shepp")):
        lhs = inner_sino(bst.project(f, g, prm), y, g)
        rhs = inner_image(f, bst.backproject(y, g, prm), g)
        assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
