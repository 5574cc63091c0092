"""Pins for the BST oracle with non-uniform angles (P5 angle bracketing in the
period-pi continuation of the angle sequence). CPU only.

- explicit uniform angles reproduce the uniform path;
- the vectorised oracle equals the literal-sum one for irregular angle sets,
  including sets whose first angle is above 0 (bracket below theta_0);
- a rotationally symmetric object gives the same image for any angle set
  (angular interpolation of angle-independent data is exact);
- for jittered angles the gap to brute force (which weights each angle by its
  neighbour gaps) stays at the uniform level.
"""
import numpy as np
import pytest

import synth
from oracle import bruteforce, bst, bst_naive, ramp
from oracle.geometry import Geometry


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _irregular(V, seed, first=0.0):
    rng = np.random.default_rng(seed)
    th = np.sort(rng.uniform(first, np.pi, V))
    th[0] = max(first, 0.0)
    return np.unique(th)[:V]


@pytest.mark.parametrize("interp", ["linear", "keys"])
def test_explicit_uniform_angles_match_uniform_path(interp):
    N, V = 32, 24
    rng = np.random.default_rng(1)
    y = rng.standard_normal((V, N))
    prm = bst.Params(2, 2, "ramp", "keys" if interp == "keys" else "deapod", interp=interp)
    a = bst.backproject(y, Geometry(N, V, N), prm)
    b = bst.backproject(y, Geometry(N, V, N, np.arange(V) * np.pi / V), prm)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(a))


@pytest.mark.parametrize("first", [0.0, 0.3])
@pytest.mark.parametrize("interp", ["linear", "keys"])
@pytest.mark.parametrize("filt", ["ramp", "none"])
def test_irregular_angles_equal_literal_sums(first, interp, filt):
    N, V = 8, 7
    th = _irregular(V, 11 + int(first * 10), first)
    assert th.size == V
    g = Geometry(N, V, N, th)
    rng = np.random.default_rng(5)
    y = rng.standard_normal((V, N))
    taper = "keys" if interp == "keys" else "deapod"
    a = bst.backproject(y, g, bst.Params(2, 2, filt, taper, interp=interp))
    b = bst_naive.backproject(y, g, 2, 2, filt, taper=taper, interp=interp)
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(b))


def test_bracket_below_first_angle_uses_the_conjugate_image():
    g = Geometry(16, 4, 16, np.array([0.2, 0.9, 1.7, 2.5]))
    th = np.array([0.0, 0.1, 0.2, 2.6, np.pi - 1e-9])
    j0, j1, f, flip0, flip1 = bst.angle_bracket(th, g)
    # below theta_0 = 0.2: between theta_3 - pi = -0.6416 and theta_0
    assert list(j0[:2]) == [3, 3] and list(j1[:2]) == [0, 0]
    assert flip0[:2].all() and not flip1[:2].any()
    assert np.allclose(f[:2], (th[:2] - (2.5 - np.pi)) / (0.2 - (2.5 - np.pi)))
    # exactly on theta_0, and past the last angle (theta_0 + pi is the image)
    assert j0[2] == 0 and f[2] == 0.0 and not flip0[2]
    assert j0[3] == 3 and j1[3] == 0 and flip1[3] and not flip0[3]
    assert np.allclose(f[3], (2.6 - 2.5) / (0.2 + np.pi - 2.5))


def test_symmetric_object_is_independent_of_the_angle_set():
    N, V = 64, 48
    sg = synth.Geometry(N, V, N)
    y = synth.gaussian_sinogram(sg, synth.Gaussian(0.0, 0.0, 0.25, 1.0)).numpy().astype(np.float64)
    # bin 0 (t = -1) has no mirror bin: zero it so every line is even in t and its
    # spectrum real, hence the same for a sample and its conjugated image
    y[:, 0] = 0.0
    a = bst.backproject(y, Geometry(N, V, N), bst.Params())
    b = bst.backproject(y, Geometry(N, V, N, _irregular(V, 3, 0.05)), bst.Params())
    assert _rel(b, a) < 1e-12


def test_jittered_angles_keep_the_gap():
    N, V = 128, 128
    rng = np.random.default_rng(8)
    th = (np.arange(V) + rng.uniform(-0.3, 0.3, V)) * np.pi / V
    th[0] = abs(th[0])
    th = np.sort(th)
    sg = synth.Geometry(N, V, N, angles=tuple(th.tolist()))
    ell = synth.head_phantom(5, 10)
    y = synth.ellipse_sinogram(sg, ell).numpy().astype(np.float64)
    g = Geometry(N, V, N, th)
    bf = bruteforce.backproject(ramp.filter_fft(y, g.dt), g)
    u = g.u()
    disk = np.hypot(u[None, :], u[:, None]) <= (N / 2 - 2) * g.d
    gap = _rel(bst.backproject(y, g, bst.Params())[disk], bf[disk])
    assert gap < 0.035


@pytest.mark.parametrize("interp", ["linear", "keys"])
@pytest.mark.parametrize("first", [0.0, 0.4])
def test_nonuniform_project_is_the_adjoint(interp, first):
    N, V = 32, 27
    g = Geometry(N, V, N, _irregular(V, 21, first))
    prm = bst.Params(2, 2, "ramp", "keys" if interp == "keys" else "deapod", interp=interp)
    rng = np.random.default_rng(2)
    f = rng.standard_normal((N, N))
    y = rng.standard_normal((V, N))
    lhs = bruteforce.inner_sino(bst.project(f, g, prm), y, g)
    rhs = bruteforce.inner_image(f, bst.backproject(y, g, prm), g)
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_nonuniform_project_equals_transpose_of_literal_backprojection():
    N, V = 8, 6
    g = Geometry(N, V, N, np.array([0.15, 0.6, 1.1, 1.3, 2.2, 2.9]))
    cols = []
    for k in range(V * N):
        e = np.zeros(V * N)
        e[k] = 1.0
        cols.append(bst_naive.backproject(e.reshape(V, N), g, 2, 2, "none").ravel())
    Bmat = np.stack(cols, axis=1)
    f = np.random.default_rng(12).standard_normal((N, N))
    expect = (g.d ** 2 / g.dt) * (Bmat.T @ f.ravel()).reshape(V, N) / g.w[:, None]
    got = bst.project(f, g, bst.Params(2, 2, "none"))
    assert np.max(np.abs(got - expect)) <= 1e-12 * np.max(np.abs(expect))
