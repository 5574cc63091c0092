"""Discrete ramp filter for the brute-force FBP reference (FP64).

FBP is x = B[F y] with F the convolution along t whose transfer function is
|sigma| (Section 1). The paper gives no discrete ramp; this oracle uses the
band-limited spatial kernel of Kak & Slaney (the same reference the paper cites
for its phantom), sampled at the detector pitch dt:

    h[0] = 1 / (4 dt^2),  h[k odd] = -1 / (pi^2 k^2 dt^2),  h[k even != 0] = 0,

applied as a linear (non-circular) convolution q[i] = dt sum_k h[i - k] y[k].
"""
from __future__ import annotations

import numpy as np


def kernel(n: int, dt: float) -> np.ndarray:
    """h[k] for k = -(n-1) .. n-1 (index k + n - 1)."""
    k = np.arange(-(n - 1), n)
    h = np.zeros(k.shape, dtype=np.float64)
    h[k == 0] = 1.0 / (4.0 * dt * dt)
    odd = (k % 2) != 0
    h[odd] = -1.0 / (np.pi ** 2 * k[odd].astype(np.float64) ** 2 * dt * dt)
    return h


def filter_direct(sino: np.ndarray, dt: float) -> np.ndarray:
    """Literal O(n^2) linear convolution, row by row (small sizes)."""
    y = np.asarray(sino, dtype=np.float64)
    n = y.shape[-1]
    h = kernel(n, dt)
    out = np.empty_like(y)
    for j in range(y.shape[0]):
        full = np.convolve(y[j], h)  # length 3n - 2; output i sits at i + n - 1
        out[j] = dt * full[n - 1:2 * n - 1]
    return out


def filter_fft(sino: np.ndarray, dt: float) -> np.ndarray:
    """The same linear convolution through a zero-padded FFT (length >= 3n - 2)."""
    y = np.asarray(sino, dtype=np.float64)
    n = y.shape[-1]
    h = kernel(n, dt)
    L = 1
    while L < 3 * n - 2:
        L *= 2
    Hf = np.fft.rfft(h, L)
    Yf = np.fft.rfft(y, L, axis=-1)
    full = np.fft.irfft(Yf * Hf, L, axis=-1)
    return dt * full[..., n - 1:2 * n - 1]
