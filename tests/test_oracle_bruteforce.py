"""Pins for the brute-force oracle B_d / R_d (Eq. 1, Eq. 2) against closed forms,
literal loops and the adjoint identity. CPU only."""
import math

import numpy as np
import pytest
from scipy.special import i0e, j0

import synth
from oracle import bruteforce
from oracle.geometry import Geometry


def _disk(g: Geometry, radius: float):
    u = g.u()
    return np.hypot(u[None, :], u[:, None]) <= radius


def test_constant_sinogram_backprojects_to_pi_c():
    # Eq. 2 with y = c: b(u) = c * int_0^pi dtheta = pi c wherever every ray hits a bin.
    g = Geometry(64, 48, 64)
    c = 1.7
    b = bruteforce.backproject(np.full((g.V, g.n), c), g)
    inside = _disk(g, (g.n / 2 - 1) * g.dt)
    assert np.max(np.abs(b[inside] - math.pi * c)) <= 1e-13 * math.pi * c


def test_constant_nonuniform_angles():
    rng = np.random.default_rng(3)
    th = np.sort(rng.uniform(0, np.pi, 40))
    g = Geometry(32, 40, 32, angles=th)
    assert abs(g.w.sum() - np.pi) < 1e-14
    b = bruteforce.backproject(np.ones((g.V, g.n)), g)
    assert np.max(np.abs(b[_disk(g, (g.n / 2 - 1) * g.dt)] - math.pi)) < 1e-13


def test_cosine_sinogram_gives_bessel_j0_and_converges():
    # (1/pi) int_0^pi cos(z cos theta) dtheta = J0(z): y = cos(2 pi s0 t) -> pi J0(2 pi s0 |u|).
    s0 = 3.0
    errs = []
    for N in (64, 128, 256):
        g = Geometry(N, N, N)
        y = np.tile(np.cos(2 * np.pi * s0 * g.t()), (g.V, 1))
        u = g.u()
        R = np.hypot(u[None, :], u[:, None])
        b = bruteforce.backproject(y, g)
        m = _disk(g, 0.9)
        errs.append(np.max(np.abs(b - np.pi * j0(2 * np.pi * s0 * R))[m]))
    # linear interpolation of the cosine loses (2 pi s0 dt)^2 / 8 of its amplitude
    assert errs[-1] < 1e-2
    # error O(dt^2), about 4x smaller per doubling of N
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def test_gaussian_backprojection_closed_form():
    # B R g(u) = pi sqrt(2 pi) s exp(-r^2/4s^2) I0(r^2/4s^2), r = |u - c|.
    gs = synth.Gaussian(0.15, -0.2, 0.08)
    errs = []
    for N in (64, 128, 256):
        sg = synth.Geometry(N, N, N)
        g = Geometry(N, N, N)
        y = synth.gaussian_sinogram(sg, gs).numpy()
        u = g.u()
        r = np.hypot(u[None, :] - gs.cx, u[:, None] - gs.cy)
        z = r * r / (4 * gs.s ** 2)
        ex = np.pi * math.sqrt(2 * math.pi) * gs.s * i0e(z)
        b = bruteforce.backproject(y, g)
        m = _disk(g, 0.9)
        errs.append(np.linalg.norm((b - ex)[m]) / np.linalg.norm(ex[m]))
    assert errs[-1] < 1e-3
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


def _literal_B(y, g):
    out = np.zeros((g.N, g.N))
    for p in range(g.N):
        for q in range(g.N):
            u1 = (q - g.N // 2) * g.d
            u2 = (p - g.N // 2) * g.d
            acc = 0.0
            for j in range(g.V):
                s = (u1 * math.cos(g.theta[j]) + u2 * math.sin(g.theta[j])) / g.dt + g.n / 2
                for i in range(g.n):
                    lam = max(0.0, 1.0 - abs(s - i))
                    acc += g.w[j] * y[j][i] * lam
            out[p][q] = acc
    return out


def _literal_R(f, g):
    out = np.zeros((g.V, g.n))
    for j in range(g.V):
        for i in range(g.n):
            acc = 0.0
            for p in range(g.N):
                for q in range(g.N):
                    u1 = (q - g.N // 2) * g.d
                    u2 = (p - g.N // 2) * g.d
                    s = (u1 * math.cos(g.theta[j]) + u2 * math.sin(g.theta[j])) / g.dt + g.n / 2
                    acc += f[p][q] * max(0.0, 1.0 - abs(s - i))
            out[j][i] = g.d ** 2 / g.dt * acc
    return out


@pytest.mark.parametrize("n,V,N", [(8, 6, 8), (12, 5, 8)])
def test_tiny_literal_loops(n, V, N):
    rng = np.random.default_rng(n * 100 + V)
    g = Geometry(n, V, N)
    y = rng.standard_normal((V, n))
    f = rng.standard_normal((N, N))
    assert np.max(np.abs(bruteforce.backproject(y, g) - _literal_B(y, g))) < 1e-14 * 10
    assert np.max(np.abs(bruteforce.project(f, g) - _literal_R(f, g))) < 1e-14 * 10


def test_pixel_subset_matches_full():
    rng = np.random.default_rng(9)
    g = Geometry(32, 20, 32)
    y = rng.standard_normal((g.V, g.n))
    full = bruteforce.backproject(y, g)
    rows = rng.integers(0, g.N, 50)
    cols = rng.integers(0, g.N, 50)
    sub = bruteforce.backproject_pixels(y, g, rows, cols)
    assert np.max(np.abs(sub - full[rows, cols])) < 1e-13


@pytest.mark.parametrize("n,V,N,angles", [(32, 24, 32, None), (64, 50, 64, None), (40, 17, 32, "rand")])
def test_adjoint_identity(n, V, N, angles):
    rng = np.random.default_rng(n + V + N)
    th = None if angles is None else np.sort(rng.uniform(0, np.pi, V))
    g = Geometry(n, V, N, angles=th)
    f = rng.standard_normal((N, N))
    y = rng.standard_normal((V, n))
    lhs = bruteforce.inner_sino(bruteforce.project(f, g), y, g)
    rhs = bruteforce.inner_image(f, bruteforce.backproject(y, g), g)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_project_of_pixelised_gaussian_matches_analytic_radon():
    gs = synth.Gaussian(-0.1, 0.2, 0.1)
    errs = []
    for N in (64, 128, 256):
        sg = synth.Geometry(N, N, N)
        g = Geometry(N, N, N)
        f = synth.gaussian_image(sg, gs).numpy()
        ex = synth.gaussian_sinogram(sg, gs).numpy()
        r = bruteforce.project(f, g)
        errs.append(np.linalg.norm(r - ex) / np.linalg.norm(ex))
    # a pixel-driven projector aliases near 45 degrees; its L2 error falls like N^-1/2
    assert errs[-1] < 1e-2
    assert errs[0] / errs[1] > 1.3 and errs[1] / errs[2] > 1.3


def test_project_of_pixelised_ellipses_converges_to_analytic_radon():
    ell = synth.head_phantom(11, 6)
    errs = []
    for N in (64, 128, 256):
        sg = synth.Geometry(N, 45, N)
        g = Geometry(N, 45, N)
        f = synth.ellipse_image(sg, ell).numpy()
        ex = synth.ellipse_sinogram(sg, ell).numpy()
        errs.append(np.linalg.norm(bruteforce.project(f, g) - ex) / np.linalg.norm(ex))
    # pixelisation of sharp edges: first-order convergence
    assert errs[-1] < 2e-2
    assert errs[0] / errs[1] > 1.5 and errs[1] / errs[2] > 1.5
