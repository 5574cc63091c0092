"""Pins for the cubic radial interpolation option of P5 (interp='keys') and
its de-apodising taper. CPU only.

- the Keys kernel (a = -1/2) interpolates the samples and reproduces
  quadratics (its defining moment conditions);
- its Fourier transform in closed form agrees with numerical quadrature;
- the vectorised gather is exact on spectra quadratic in the radius, in both
  half-planes and across sigma = 0 (where the tap at m = -1 is conj Yh[1]);
- the vectorised oracle equals the literal-sum one at tiny sizes;
- on a phantom it narrows the gap to brute-force FBP (the reason it exists).
"""
import numpy as np
import pytest
from scipy.integrate import quad

import synth
from oracle import bst, bst_naive, bruteforce, ramp
from oracle.geometry import Geometry


def test_keys_weights_interpolate_and_reproduce_quadratics():
    frac = np.linspace(0.0, 0.999, 37)
    w = np.stack(bst.keys_weights(frac))          # taps at m0-1 .. m0+2
    k = np.arange(-1, 3, dtype=np.float64)[:, None]
    assert np.allclose(w.sum(axis=0), 1.0, atol=1e-14)
    assert np.allclose((w * (k - frac)).sum(axis=0), 0.0, atol=1e-14)
    assert np.allclose((w * (k - frac) ** 2).sum(axis=0), 0.0, atol=1e-14)
    assert np.allclose(np.stack(bst.keys_weights(np.zeros(1)))[:, 0], [0, 1, 0, 0])
    # a cubic is not reproduced (third moment is non-zero somewhere)
    assert np.max(np.abs((w * (k - frac) ** 3).sum(axis=0))) > 1e-3


@pytest.mark.parametrize("nu", [0.0, 0.05, 0.125, 0.25, 0.4, 0.5, 0.75, 1.0, 1.3])
def test_keys_ft_matches_quadrature(nu):
    val, err = quad(lambda x: float(bst.keys_kernel(np.array(x))) * np.cos(2 * np.pi * nu * x),
                    -2.0, 2.0, points=[-1.0, 0.0, 1.0], limit=200)
    assert abs(float(bst.keys_ft(np.array(nu))) - val) < 1e-10


def test_keys_taper_is_the_inverse_transform():
    g = Geometry(64, 32, 64)
    prm = bst.Params(2, 2, "ramp", "keys", interp="keys")
    M, _, dsig, _ = bst.sizes(g, prm)
    w = bst.taper(g, prm)
    assert w[g.n // 2] == 1.0
    assert np.allclose(w * bst.keys_ft(g.t() * dsig), 1.0)
    assert 1.0 < w.max() < 1.1   # |t dsigma| <= 1/4 at P_r = 2


def _quadratic_spectrum(V, M, alpha, beta, gamma):
    m = np.arange(M // 2 + 1, dtype=np.float64)
    row = alpha + 1j * beta * m + gamma * m * m
    return np.tile(row, (V, 1)), np.full(V, alpha)


@pytest.mark.parametrize("P_r,P_c", [(2, 2), (1, 2), (4, 2)])
def test_keys_gather_exact_on_quadratic_spectra(P_r, P_c):
    N, V = 32, 24
    g = Geometry(N, V, N)
    prm = bst.Params(P_r, P_c, "ramp", "none", interp="keys")
    M, G, _, _ = bst.sizes(g, prm)
    alpha, beta, gamma = 0.7, -0.3, 0.011
    Yh, Y0 = _quadratic_spectrum(V, M, alpha, beta, gamma)
    C = bst.gather(Yh, Y0, g, prm)
    a = np.arange(G // 2 + 1, dtype=np.float64)[None, :]
    b = np.arange(G, dtype=np.float64)
    b = np.where(b < G // 2, b, b - G)[:, None]
    r = np.hypot(a, b) * P_r / P_c
    lower = np.arctan2(b, a + 0 * b) < 0
    q = np.where(lower, np.arctan2(b, a + 0 * b) + np.pi, np.arctan2(b, a + 0 * b)) * V / np.pi
    wrap = np.floor(q) >= V - 1                    # the neighbour past theta_{V-1} flips
    inside = (np.floor(r) + 2 < M // 2) & ~wrap & ~((a == 0) & (b == 0))
    expect = alpha + 1j * beta * r + gamma * r * r
    expect = np.where(lower, np.conj(expect), expect)
    assert inside.sum() > 100
    assert np.max(np.abs(C[inside] - expect[inside])) < 1e-12
    # the linear option is exact only on spectra linear in r
    lin = bst.gather(Yh, Y0, g, bst.Params(P_r, P_c, "ramp", "none"))
    assert np.max(np.abs(lin[inside] - expect[inside])) > 1e-3


@pytest.mark.parametrize("N,V", [(8, 6), (16, 8)])
@pytest.mark.parametrize("filt", ["ramp", "none"])
def test_keys_oracle_equals_literal_sums(N, V, filt):
    rng = np.random.default_rng(N * 11 + V)
    g = Geometry(N, V, N)
    y = rng.standard_normal((V, N))
    a = bst.backproject(y, g, bst.Params(2, 2, filt, "keys", interp="keys"))
    b = bst_naive.backproject(y, g, 2, 2, filt, taper="keys", interp="keys")
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))


def test_keys_narrows_the_gap_to_bruteforce():
    N = 128
    sg = synth.Geometry(N, N, N)
    ell = synth.head_phantom(5, 10)
    y = synth.ellipse_sinogram(sg, ell).numpy().astype(np.float64)
    g = Geometry(N, N, N)
    bf = bruteforce.backproject(ramp.filter_fft(y, g.dt), g)
    u = g.u()
    disk = np.hypot(u[None, :], u[:, None]) <= (N / 2 - 2) * g.d

    def gap(img):
        return float(np.linalg.norm(img[disk] - bf[disk]) / np.linalg.norm(bf[disk]))

    lin = gap(bst.backproject(y, g, bst.Params()))
    cub = gap(bst.backproject(y, g, bst.Params(taper="keys", interp="keys")))
    assert cub < 0.85 * lin
    assert cub < 0.025


@pytest.mark.parametrize("N,V,P_r,P_c,filt", [(16, 12, 2, 2, "ramp"), (32, 21, 1, 2, "none"),
                                              (64, 50, 2, 1, "ramp"), (32, 24, 4, 2, "none")])
def test_keys_project_is_the_adjoint(N, V, P_r, P_c, filt):
    rng = np.random.default_rng(N + V + 7 * P_r)
    g = Geometry(N, V, N)
    prm = bst.Params(P_r, P_c, filt, "keys", interp="keys")
    f = rng.standard_normal((N, N))
    y = rng.standard_normal((V, N))
    lhs = bruteforce.inner_sino(bst.project(f, g, prm), y, g)
    rhs = bruteforce.inner_image(f, bst.backproject(y, g, prm), g)
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


@pytest.mark.parametrize("filt", ["ramp", "none"])
def test_keys_project_equals_transpose_of_literal_backprojection(filt):
    N, V = 8, 6
    g = Geometry(N, V, N)
    cols = []
    for k in range(V * N):
        e = np.zeros(V * N)
        e[k] = 1.0
        cols.append(bst_naive.backproject(e.reshape(V, N), g, 2, 2, filt, taper="keys", interp="keys").ravel())
    Bmat = np.stack(cols, axis=1)
    f = np.random.default_rng(9).standard_normal((N, N))
    expect = (g.d ** 2 / (g.dt * np.pi / V)) * (Bmat.T @ f.ravel()).reshape(V, N)
    got = bst.project(f, g, bst.Params(2, 2, filt, "keys", interp="keys"))
    assert np.max(np.abs(got - expect)) <= 1e-12 * np.max(np.abs(expect))


@pytest.mark.parametrize("interp", ["linear", "keys"])
def test_cartesian_nyquist_column_is_zero(interp):
    """The column |k_x| = G/2 dk is dropped (like the radial Nyquist sample):
    with linear taps all its points already lie at r >= M/2 (P_r = P_c)."""
    N, V = 16, 12
    g = Geometry(N, V, N)
    rng = np.random.default_rng(3)
    y = rng.standard_normal((V, N))
    prm = bst.Params(2, 2, "ramp", "none", interp=interp)
    Yh, Y0 = bst.spectrum(y, g, prm)
    C = bst.gather(Yh, Y0, g, prm)
    M, G, _, _ = bst.sizes(g, prm)
    assert np.all(C[:, G // 2] == 0)
    if interp == "linear":
        a = G // 2
        b = np.arange(G)
        b = np.where(b < G // 2, b, b - G)
        assert np.all(np.hypot(a, b) * prm.P_r / prm.P_c >= M // 2)
