"""Seeded phantoms and their analytic parallel-beam sinograms.

Sampling grids (problem statement of Section 1, "Description of the problem"):
  detector  t_i = (i - n/2) * dt,  dt = 2/n,  i = 0..n-1        (t in [-1, 1))
  angles    theta_j = j * pi / V,  j = 0..V-1                    ([0, pi))
  image     u = ((q - N/2) * d, (p - N/2) * d),  d = 2/N          (row p, column q)
A sinogram is stored as [V][n] (detector index fastest); an image as [N][N]
(row = u2, column = u1).

The analytic Radon transforms follow the ellipse formula of Kak & Slaney
(cited by the paper for its synthetic ellipsoid dataset, Section 4):
for an ellipse with centre c, semi-axes (A, B), rotation alpha and density rho,
  a^2(theta) = A^2 cos^2(theta - alpha) + B^2 sin^2(theta - alpha),
  R(t, theta) = 2 rho A B / a^2 * sqrt(a^2 - (t - c.xi)^2)   for |t - c.xi| <= a.
All evaluation is done in float64 with torch on the requested device; callers
cast to float32 where the GPU path consumes the bytes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional
from typing import List, Sequence

import numpy as np
import torch


@dataclass(frozen=True)
class Geometry:
    n_det: int
    n_angles: int
    n_out: int
    angles: Optional[tuple] = None   # non-uniform theta_j (increasing, in [0, pi)), else j pi / V

    @property
    def dt(self) -> float:
        return 2.0 / self.n_det

    @property
    def d(self) -> float:
        return 2.0 / self.n_out

    def t(self, device="cpu") -> torch.Tensor:
        return (torch.arange(self.n_det, dtype=torch.float64, device=device)
                - self.n_det // 2) * self.dt

    def theta(self, device="cpu") -> torch.Tensor:
        if self.angles is not None:
            return torch.tensor(self.angles, dtype=torch.float64, device=device)
        return torch.arange(self.n_angles, dtype=torch.float64,
                            device=device) * (math.pi / self.n_angles)

    def u(self, device="cpu") -> torch.Tensor:
        return (torch.arange(self.n_out, dtype=torch.float64, device=device)
                - self.n_out // 2) * self.d


@dataclass(frozen=True)
class Ellipse:
    cx: float
    cy: float
    A: float
    B: float
    alpha: float
    rho: float


@dataclass(frozen=True)
class Gaussian:
    cx: float
    cy: float
    s: float
    amp: float = 1.0


def random_ellipses(rng: np.random.Generator, count: int,
                    axes=(0.05, 0.7), rho=(0.1, 1.0),
                    fov: float = 0.95) -> List[Ellipse]:
    """Draw `count` ellipses: semi-axes U[axes], rotation U[0, pi),
    density +-U[rho], centre uniform in the disk that keeps |c| + max(A,B) <= fov."""
    out = []
    for _ in range(count):
        A = rng.uniform(*axes)
        B = rng.uniform(*axes)
        big = max(A, B)
        if big > fov:
            big = fov
        rmax = max(fov - big, 0.0)
        rad = rmax * math.sqrt(rng.uniform(0.0, 1.0))
        ang = rng.uniform(0.0, 2 * math.pi)
        alpha = rng.uniform(0.0, math.pi)
        sign = 1.0 if rng.uniform() < 0.5 else -1.0
        r = sign * rng.uniform(*rho)
        out.append(Ellipse(rad * math.cos(ang), rad * math.sin(ang), A, B, alpha, r))
    return out


def head_phantom(seed: int, count: int = 10) -> List[Ellipse]:
    """A seeded 'head' of `count` ellipses: one positive outer skull-like
    ellipse that contains the rest, which are drawn as in random_ellipses."""
    rng = np.random.default_rng(seed)
    outer = Ellipse(0.0, 0.0, 0.69 + 0.02 * rng.uniform(), 0.9 + 0.02 * rng.uniform(),
                    rng.uniform(0, 0.2), 1.0)
    rest = random_ellipses(rng, count - 1, axes=(0.05, 0.7), rho=(0.1, 1.0), fov=0.9)
    return [outer] + rest


def ellipse_sinogram(geom: Geometry, ellipses: Sequence[Ellipse],
                     device="cpu") -> torch.Tensor:
    """Analytic Radon transform sampled on the (theta_j, t_i) grid, float64 [V][n]."""
    t = geom.t(device)[None, :]
    th = geom.theta(device)[:, None]
    ct, st = torch.cos(th), torch.sin(th)
    y = torch.zeros(geom.n_angles, geom.n_det, dtype=torch.float64, device=device)
    for e in ellipses:
        tp = th - e.alpha
        a2 = (e.A * torch.cos(tp)) ** 2 + (e.B * torch.sin(tp)) ** 2
        s = t - (e.cx * ct + e.cy * st)
        inside = (a2 - s * s).clamp_min(0.0)
        y += (2.0 * e.rho * e.A * e.B / a2) * torch.sqrt(inside)
    return y


def ellipse_image(geom: Geometry, ellipses: Sequence[Ellipse],
                  device="cpu") -> torch.Tensor:
    """Indicator-sum image of the ellipses at pixel centres, float64 [N][N]."""
    u = geom.u(device)
    u1 = u[None, :]
    u2 = u[:, None]
    img = torch.zeros(geom.n_out, geom.n_out, dtype=torch.float64, device=device)
    for e in ellipses:
        ca, sa = math.cos(e.alpha), math.sin(e.alpha)
        x = (u1 - e.cx) * ca + (u2 - e.cy) * sa
        z = -(u1 - e.cx) * sa + (u2 - e.cy) * ca
        img += e.rho * (((x / e.A) ** 2 + (z / e.B) ** 2) <= 1.0).to(torch.float64)
    return img


def gaussian_sinogram(geom: Geometry, g: Gaussian, device="cpu") -> torch.Tensor:
    """Radon transform of amp*exp(-|u-c|^2 / (2 s^2)): amp*sqrt(2 pi) s exp(-(t - c.xi)^2/(2 s^2))."""
    t = geom.t(device)[None, :]
    th = geom.theta(device)[:, None]
    sc = t - (g.cx * torch.cos(th) + g.cy * torch.sin(th))
    return g.amp * math.sqrt(2 * math.pi) * g.s * torch.exp(-sc * sc / (2 * g.s * g.s))


def gaussian_image(geom: Geometry, g: Gaussian, device="cpu") -> torch.Tensor:
    u = geom.u(device)
    r2 = (u[None, :] - g.cx) ** 2 + (u[:, None] - g.cy) ** 2
    return g.amp * torch.exp(-r2 / (2 * g.s * g.s))


def add_gaussian_noise(y: torch.Tensor, rel: float, generator: torch.Generator) -> torch.Tensor:
    """y + N(0, (rel * max|y|)^2), per slice when y is [B][V][n]."""
    if y.dim() == 2:
        scale = rel * y.abs().max()
    else:
        scale = rel * y.abs().amax(dim=(-2, -1), keepdim=True)
    noise = torch.randn(y.shape, dtype=y.dtype, device=y.device, generator=generator)
    return y + scale * noise


# --- 3D ellipsoid volume (axis of each ellipsoid along s, as in the paper's footnote) ---

def ellipsoid_volume_params(seed: int, count: int = 30):
    """Ellipsoids (cx, cy, cs, A, B, C, alpha, rho) with |(cx,cy)| + max(A,B) <= 0.95."""
    rng = np.random.default_rng(seed)
    out = []
    for e in random_ellipses(rng, count):
        C = rng.uniform(0.1, 0.9)
        cs = rng.uniform(-0.9 + C * 0.5, 0.9 - C * 0.5)
        out.append((e.cx, e.cy, cs, e.A, e.B, C, e.alpha, e.rho))
    return out


def ellipsoid_slice_ellipses(params, s_k: float) -> List[Ellipse]:
    """Axial cut at height s_k: each ellipsoid gives an ellipse with semi-axes
    scaled by sqrt(1 - ((s_k - cs)/C)^2), or nothing when the plane misses it."""
    out = []
    for (cx, cy, cs, A, B, C, alpha, rho) in params:
        z = (s_k - cs) / C
        if abs(z) < 1.0:
            k = math.sqrt(1.0 - z * z)
            out.append(Ellipse(cx, cy, A * k, B * k, alpha, rho))
    return out


def poisson_like_noise(y: torch.Tensor, I0: float, generator: torch.Generator) -> torch.Tensor:
    """Lambert-Beer counts ~ Poisson(I0 exp(-mu y)) with mu scaled so max(mu y) = 2,
    returned as -ln(max(counts, 1)/I0)/mu (Gaussian approximation of Poisson
    with variance equal to the mean, drawn on y's device)."""
    ymax = float(y.max())
    mu = 2.0 / ymax if ymax > 0 else 1.0
    lam = I0 * torch.exp(-mu * y)
    counts = lam + torch.sqrt(lam) * torch.randn(y.shape, dtype=y.dtype, device=y.device,
                                                  generator=generator)
    counts = torch.round(counts).clamp_min(1.0)
    return -torch.log(counts / I0) / mu


# --- named workloads ---------------------------------------------------------

BASE_SEED = 170408364


def config1_sinogram(device="cpu", noise: bool = True):
    """Single slice, 256 angles x 256 bins, 10-ellipse head phantom, 1% noise.
    Returns (sino float32 [V][n], geometry, ellipses)."""
    geom = Geometry(256, 256, 256)
    ell = head_phantom(BASE_SEED + 1, 10)
    y = ellipse_sinogram(geom, ell, device)
    if noise:
        g = torch.Generator(device=device)
        g.manual_seed(BASE_SEED + 1)
        y = add_gaussian_noise(y, 0.01, g)
    return y.to(torch.float32), geom, ell


def batch_sinograms(batch: int, n: int, V: int, seed: int, device="cpu",
                    min_ell: int = 5, max_ell: int = 20, noise: float = 0.01,
                    ) -> torch.Tensor:
    """`batch` independent slices, each a random 5-20 ellipse phantom's analytic
    sinogram plus `noise` * max Gaussian noise; float32 [batch][V][n]."""
    geom = Geometry(n, V, n)
    rng = np.random.default_rng(seed)
    out = torch.empty(batch, V, n, dtype=torch.float32, device=device)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    for b in range(batch):
        k = int(rng.integers(min_ell, max_ell + 1))
        ell = random_ellipses(rng, k)
        y = ellipse_sinogram(geom, ell, device)
        if noise > 0:
            y = add_gaussian_noise(y, noise, g)
        out[b] = y.to(torch.float32)
    return out
