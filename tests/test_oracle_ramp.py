"""Pins for the brute-force FBP ramp filter (F of Section 1). CPU only."""
import math

import numpy as np

import synth
from oracle import bruteforce, ramp
from oracle.geometry import Geometry


def test_fft_convolution_equals_literal_convolution():
    rng = np.random.default_rng(1)
    for n in (8, 33, 64):
        y = rng.standard_normal((5, n))
        dt = 2.0 / n
        assert np.max(np.abs(ramp.filter_fft(y, dt) - ramp.filter_direct(y, dt))) < 1e-10 / dt ** 2


def test_kernel_transfer_is_the_ramp_inside_the_band():
    # The infinite band-limited kernel has DTFT dt * sum_k h[k] e^{-2 pi i sigma k dt} = |sigma|
    # for |sigma| <= 1/(2 dt); the truncated tail costs O(1/(n dt)).
    n, dt = 512, 2.0 / 512
    h = ramp.kernel(n, dt)
    k = np.arange(-(n - 1), n)
    for sig in (0.0, 3.0, 17.5, 60.0, 120.0):
        H = dt * np.sum(h * np.cos(2 * np.pi * sig * k * dt))
        assert abs(H - abs(sig)) < 2.0 / (np.pi ** 2 * n * dt)


def test_filtered_backprojection_of_gaussian_recovers_it():
    gs = synth.Gaussian(0.2, 0.1, 0.1)
    errs = []
    for N in (64, 128, 256):
        sg = synth.Geometry(N, N, N)
        g = Geometry(N, N, N)
        y = synth.gaussian_sinogram(sg, gs).numpy()
        x = synth.gaussian_image(sg, gs).numpy()
        r = bruteforce.backproject(ramp.filter_fft(y, g.dt), g)
        errs.append(np.linalg.norm(r - x) / np.linalg.norm(x))
    assert errs[-1] < 2e-2
    assert errs[0] > errs[2]


def test_filtered_backprojection_of_constant_disk_level():
    # A centred disk of density 1: FBP returns ~1 inside, away from the edge.
    N = 128
    sg = synth.Geometry(N, N, N)
    g = Geometry(N, N, N)
    e = [synth.Ellipse(0.0, 0.0, 0.5, 0.5, 0.0, 1.0)]
    y = synth.ellipse_sinogram(sg, e).numpy()
    r = bruteforce.backproject(ramp.filter_fft(y, g.dt), g)
    u = g.u()
    inner = np.hypot(u[None, :], u[:, None]) < 0.35
    assert abs(np.mean(r[inner]) - 1.0) < 1e-2
    assert math.isfinite(float(r.sum()))
