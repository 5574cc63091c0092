"""Pins for the FP64 BST oracle (Section 2, Eq. 3, steps P0-P8). CPU only.

- literal DFT sums and per-point gathering at tiny sizes (bst_naive);
- exact symmetries of the discrete method: 90 and 180 degree rotation, mirror;
- closed forms: FBP of an analytic Gaussian returns the Gaussian (RAMP);
  y = cos(2 pi s0 t) backprojects to pi J0(2 pi s0 |u|) and a Gaussian's
  sinogram to pi sqrt(2 pi) s e^{-z} I0(z), z = r^2/4s^2 (NONE);
- the taper options reduce to each other where they must.
"""
import math

import numpy as np
import pytest
from scipy.special import i0e, j0

import synth
from oracle import bst, bst_naive
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
