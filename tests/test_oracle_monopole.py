"""Pins of the oracle's monopole subtraction for plain backprojection (the
origin artifacts of Section 2): the closed form of the Gaussian's
backprojection against an angular quadrature, the mass estimate against the
analytic mass of an ellipse phantom, exact recovery of a pure Gaussian
sinogram, and the gap to the brute-force backprojection of Eq. 2, which the
subtraction must shrink. CPU only."""
import numpy as np
import pytest

from oracle import bst as O
from oracle import bruteforce as BF
from oracle.geometry import Geometry
from synth import phantoms as PH


def _phi(t, s):
    return np.exp(-t * t / (2 * s * s)) / (np.sqrt(2 * np.pi) * s)


@pytest.mark.parametrize("s", [0.15, 0.4])
def test_closed_form_matches_angular_quadrature(s):
    # b_phi(u) = int_0^pi phi(u . xi_theta) dtheta; the trapezoid rule over a
    # period is spectrally accurate for this smooth periodic integrand
    geom = Geometry(64, 64, 64)
    prm = O.Params(filter="none", monopole=s)
    img = O.monopole_image(geom, prm)
    u = geom.u()
    V = 8192
    th = np.arange(V) * np.pi / V
    rng = np.random.default_rng(0)
    for p, q in rng.integers(0, 64, size=(12, 2)):
        proj = u[q] * np.cos(th) + u[p] * np.sin(th)
        quad = np.sum(_phi(proj, s)) * np.pi / V
        assert abs(img[p, q] - quad) <= 1e-12 * abs(quad)


def test_mass_estimate_matches_the_phantom_mass():
    n = 512
    g = PH.Geometry(n, 256, n)
    geom = Geometry(n, 256, n)
    ell = PH.head_phantom(3, 10)
    y = PH.ellipse_sinogram(g, ell).numpy()
    mass = sum(e.rho * np.pi * e.A * e.B for e in ell)
    prm = O.Params(filter="none", monopole=0.4)
    m = O.monopole_mass(y, geom, prm)
    # m is the amplitude whose Gaussian, sampled on the detector, carries the
    # mean projection mass: m dt sum_i phi_i = mean_j dt sum_i y_ji ~ the object's mass
    carried = m * geom.dt * O.monopole_profile(geom, prm).sum()
    assert abs(carried - mass) <= 1e-3 * abs(mass)
    # the Gaussian is cut off by the detector ends, so m exceeds the mass by 1/erf(1/(s sqrt 2))
    from scipy.special import erf
    assert abs(m * erf(1.0 / (0.4 * np.sqrt(2.0))) - mass) <= 1e-3 * abs(mass)


@pytest.mark.parametrize("shift", [0.0, 3.5])
def test_pure_gaussian_sinogram_is_recovered_in_closed_form(shift):
    # y = c phi(t - beta dt) at every angle: the residual vanishes and the image is c b_phi
    N, s, c = 64, 0.35, 2.5
    geom = Geometry(N, 48, N)
    prm = O.Params(filter="none", monopole=s, center_shift=shift)
    y = c * np.tile(_phi(geom.t() - shift * geom.dt, s), (geom.V, 1))
    img = O.backproject(y, geom, prm)
    ref = c * O.monopole_image(geom, prm)
    assert np.max(np.abs(img - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_linear_in_the_sinogram():
    N = 32
    geom = Geometry(N, 24, N)
    prm = O.Params(filter="none", monopole=0.4)
    rng = np.random.default_rng(1)
    y1, y2 = rng.standard_normal((2, geom.V, N))
    lhs = O.backproject(2.0 * y1 - 0.5 * y2, geom, prm)
    rhs = 2.0 * O.backproject(y1, geom, prm) - 0.5 * O.backproject(y2, geom, prm)
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * np.max(np.abs(rhs))


@pytest.mark.parametrize("P_c", [2, 4])
def test_gap_to_bruteforce_shrinks(P_c):
    # plain B has a slowly decaying mass tail whose periodic images the origin
    # rule only approximates; subtracting the monopole removes most of it
    N = 128
    g = PH.Geometry(N, N, N)
    geom = Geometry(N, N, N)
    y = PH.ellipse_sinogram(g, PH.head_phantom(3, 10)).numpy()
    ref = BF.backproject(y, geom)
    u = geom.u()
    disk = np.sqrt(u[None, :] ** 2 + u[:, None] ** 2) <= (N / 2 - 2) * geom.d

    def gap(img):
        return np.linalg.norm((img - ref)[disk]) / np.linalg.norm(ref[disk])

    plain = gap(O.backproject(y, geom, O.Params(filter="none", pad_cart=P_c)))
    mono = gap(O.backproject(y, geom, O.Params(filter="none", pad_cart=P_c, monopole=0.4)))
    assert plain > 0.02
    assert mono < 0.01
    assert mono < plain / 3


def test_monopole_is_an_option_of_plain_backprojection():
    with pytest.raises(AssertionError):
        O.Params(filter="ramp", monopole=0.4)
