"""Pins of the oracle's tent angular rule of P5 (angular='tent'): at radii
where one Cartesian cell spans several polar angles it averages them with a
tent of half-width V / (pi rho) angle steps; elsewhere it is the bilinear rule.
Pinned by: equality with the bilinear rule where h = 1 and for data that do
not depend on the angle, partition of unity, the weights written out for
single points, the adjoint identity of the projector built from it, and the
projector's closeness to the analytic Radon transform that the bilinear
transpose lacks. CPU only."""
import math

import numpy as np
import pytest

from oracle import bst as O
from oracle import bruteforce as BF
from oracle.geometry import Geometry
from synth import phantoms as PH


def _radius(G):
    a = np.arange(G // 2 + 1, dtype=np.float64)[None, :]
    b = np.arange(G, dtype=np.float64)
    b = np.where(b < G // 2, b, b - G)[:, None]
    return np.sqrt(a * a + b * b)


def _rand_spectrum(V, M, seed):
    rng = np.random.default_rng(seed)
    Yh = rng.standard_normal((V, M // 2 + 1)) + 1j * rng.standard_normal((V, M // 2 + 1))
    Yh[:, M // 2] = 0.0
    return Yh, rng.standard_normal(V)


@pytest.mark.parametrize("N,V", [(32, 24), (64, 64)])
def test_bilinear_where_the_tent_is_one_step_wide(N, V):
    geom = Geometry(N, V, N)
    lin, tent = O.Params(filter="none"), O.Params(filter="none", angular="tent")
    M, G, _, _ = O.sizes(geom, lin)
    Yh, Y0 = _rand_spectrum(V, M, 1)
    Cl = O.gather(Yh, Y0, geom, lin)
    Ct = O.gather(Yh, Y0, geom, tent)
    rho = _radius(G)
    wide = rho < V / np.pi
    wide[0, 0] = False
    assert np.max(np.abs((Ct - Cl)[~wide])) <= 1e-12 * np.max(np.abs(Cl))
    assert np.max(np.abs((Ct - Cl)[wide])) > 1e-3 * np.max(np.abs(Cl))   # it does act at small radii


def test_angle_independent_data_give_the_bilinear_result():
    # a rotationally symmetric object has the same projection at every angle:
    # any normalised angular average of it is the bilinear value
    N = V = 64
    geom = Geometry(N, V, N)
    g = PH.Geometry(N, V, N)
    y = PH.gaussian_sinogram(g, PH.Gaussian(0.0, 0.0, 0.2, 1.0)).numpy()
    # bin 0 (t = -1) has no mirror bin; without it every projection is even in
    # t, so its spectrum is real and a conjugated image equals the sample itself
    y[:, 0] = 0.0
    for filt in ("none", "ramp"):
        bl = O.backproject(y, geom, O.Params(filter=filt))
        bt = O.backproject(y, geom, O.Params(filter=filt, angular="tent"))
        assert np.max(np.abs(bt - bl)) <= 1e-12 * np.max(np.abs(bl))


def test_partition_of_unity():
    N, V = 64, 80
    geom = Geometry(N, V, N)
    prm = O.Params(filter="none", angular="tent")
    M, G, _, _ = O.sizes(geom, prm)
    Yh = np.ones((V, M // 2 + 1), dtype=np.complex128)
    Yh[:, M // 2] = 0.0
    C = O.gather(Yh, np.zeros(V), geom, prm)
    r = _radius(G) * (prm.P_r / prm.P_c)
    inside = (r < M // 2 - 1) & (r > 0)
    inside[:, G // 2] = False
    assert np.max(np.abs(C[inside] - 1.0)) <= 1e-12


@pytest.mark.parametrize("point", [(1, 0), (3, 2), (0, 5), (7, -4), (40, 9)])
def test_weights_written_out_for_single_points(point):
    # the rule restated for one Cartesian point (a, b): theta = atan2 folded to
    # [0, pi), q = theta V / pi, h = max(1, V / (pi rho)), weights over the
    # integer angle indices of the continuation, normalised; index j + V is the
    # conjugated image of angle j
    V = 48
    a, b = point
    rho = math.hypot(a, b)
    phi = math.atan2(b, a)
    th = phi + math.pi if phi < 0 else phi
    q = th * V / math.pi
    h = max(1.0, V / (math.pi * rho))
    raw = {}
    for jc in range(math.floor(q - h) - 1, math.ceil(q + h) + 2):
        w = max(0.0, 1.0 - abs(q - jc) / h)
        if w > 0:
            raw[jc] = w
    tot = sum(raw.values())
    expect = {}
    for jc, w in raw.items():
        key = (jc % V, (jc // V) % 2 == 1)
        expect[key] = expect.get(key, 0.0) + w / tot
    p, j, flip, w = O.tent_taps(np.array([th]), np.array([rho]), V)
    got = {}
    for jj, ff, ww in zip(j, flip, w):
        got[(int(jj), bool(ff))] = got.get((int(jj), bool(ff)), 0.0) + float(ww)
    assert set(got) == set(expect)
    for k in expect:
        assert abs(got[k] - expect[k]) <= 1e-14


@pytest.mark.parametrize("filt", ["none", "ramp"])
def test_adjoint_identity(filt):
    N, V = 32, 40
    geom = Geometry(N, V, N)
    prm = O.Params(filter=filt, angular="tent")
    rng = np.random.default_rng(3)
    f = rng.standard_normal((N, N))
    y = rng.standard_normal((V, N))
    lhs = BF.inner_sino(O.project(f, geom, prm), y, geom)
    rhs = BF.inner_image(f, O.backproject(y, geom, prm), geom)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), abs(rhs))


@pytest.mark.parametrize("N", [64, 128])
def test_projector_approximates_the_radon_transform(N):
    # the transpose of the bilinear gather over-weights lattice angles by up
    # to V / (pi rho); the tent's transpose spreads each polar sample over the
    # Cartesian cells it covers
    V = N
    geom = Geometry(N, V, N)
    g = PH.Geometry(N, V, N)
    ell = PH.head_phantom(4, 8)
    f = PH.ellipse_image(g, ell).numpy()
    radon = PH.ellipse_sinogram(g, ell).numpy()

    def err(prm):
        return np.linalg.norm(O.project(f, geom, prm) - radon) / np.linalg.norm(radon)

    assert err(O.Params(filter="none", angular="tent")) < 0.1
    assert err(O.Params(filter="none")) > 2.0


def test_backprojection_gap_unchanged():
    N = V = 128
    geom = Geometry(N, V, N)
    g = PH.Geometry(N, V, N)
    y = PH.ellipse_sinogram(g, PH.head_phantom(4, 8)).numpy()
    ref = BF.backproject(y, geom)
    u = geom.u()
    disk = np.sqrt(u[None, :] ** 2 + u[:, None] ** 2) <= (N / 2 - 2) * geom.d

    def gap(prm):
        img = O.backproject(y, geom, prm)
        return np.linalg.norm((img - ref)[disk]) / np.linalg.norm(ref[disk])

    assert abs(gap(O.Params(filter="none", angular="tent")) - gap(O.Params(filter="none"))) < 1e-3


def test_tent_options_are_checked():
    with pytest.raises(AssertionError):
        O.Params(angular="tent", interp="keys")
    with pytest.raises(AssertionError):
        O.Params(angular="cubic")
