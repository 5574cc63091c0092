"""torch.autograd wrappers of the BST backprojection B and its adjoint projector R.

The library guarantees <R f, g> = <f, B g> under the weighted inner products
<f, f'> = d^2 sum f f' and <g, g'> = dt sum_j (pi/V) sum_i g g', i.e.
R = c * B^T with c = d^2 / (dt * pi / V) (B^T the Euclidean transpose). The
backward passes therefore are
    d/dsino of  <grad_img, B sino>  = B^T grad_img = R grad_img / c
    d/dimg  of  <grad_sino, R img>  = R^T grad_sino = c * B grad_sino
and both run in the library's kernels (no torch arithmetic beyond the scalar c).
Plans of dtype 'f64' take float64 tensors (the gradient-check path).
"""
from __future__ import annotations

import math

import torch

from .binding import Plan


def adjoint_scale(plan: Plan) -> float:
    """c with R = c B^T; a single scalar only for uniform angles (for others the
    library's R carries the factor d^2 / (dt w_j) per angle)."""
    if plan._angles_keep is not None:
        raise ValueError("the autograd wrappers take plans with uniform angles")
    d = 2.0 / plan.N
    dt = 2.0 / plan.n
    return d * d / (dt * math.pi / plan.V)


class BSTBackproject(torch.autograd.Function):
    """img = B sino (BST backprojection); backward uses the projector."""

    @staticmethod
    def forward(ctx, sino: torch.Tensor, plan: Plan) -> torch.Tensor:
        ctx.plan = plan
        return plan.backproject(sino.contiguous())

    @staticmethod
    def backward(ctx, grad_img: torch.Tensor):
        plan = ctx.plan
        g = plan.project(grad_img.contiguous())
        return g.mul_(1.0 / adjoint_scale(plan)), None


class BSTProject(torch.autograd.Function):
    """sino = R img (the exact adjoint projector); backward uses the backprojection."""

    @staticmethod
    def forward(ctx, img: torch.Tensor, plan: Plan) -> torch.Tensor:
        ctx.plan = plan
        return plan.project(img.contiguous())

    @staticmethod
    def backward(ctx, grad_sino: torch.Tensor):
        plan = ctx.plan
        g = plan.backproject(grad_sino.contiguous())
        return g.mul_(adjoint_scale(plan)), None


def backproject(sino: torch.Tensor, plan: Plan) -> torch.Tensor:
    return BSTBackproject.apply(sino, plan)


def project(img: torch.Tensor, plan: Plan) -> torch.Tensor:
    return BSTProject.apply(img, plan)


def lipschitz(plan: Plan, shape, iters: int = 8, seed: int = 0) -> float:
    """Largest eigenvalue of 2 R^T R by power iteration (for the step size)."""
    gen = torch.Generator(device=f"cuda:{plan.device}")
    gen.manual_seed(seed)
    x = torch.randn(shape, device=f"cuda:{plan.device}", generator=gen, dtype=plan.torch_dtype)
    lam = 1.0
    c = adjoint_scale(plan)
    for _ in range(iters):
        x = x / x.norm()
        y = plan.backproject(plan.project(x)).mul_(c)
        lam = float((x * y).sum())
        x = y
    return 2.0 * lam


def least_squares(plan: Plan, g: torch.Tensor, steps: int = 20, step: float = None):
    """Gradient descent on L(f) = ||R f - g||^2 from f = 0, gradients by autograd.
    Returns (f, losses)."""
    B = g.shape[0]
    shape = (B, plan.N, plan.N)
    if step is None:
        step = 1.0 / lipschitz(plan, shape)
    f = torch.zeros(shape, device=g.device, dtype=plan.torch_dtype, requires_grad=True)
    # the losses stay on the device until the end: reading each one back
    # would stall the stream once per step
    losses = []
    for _ in range(steps):
        r = project(f, plan) - g
        loss = (r * r).sum()
        losses.append(loss.detach())
        (grad,) = torch.autograd.grad(loss, f)
        with torch.no_grad():
            f.add_(grad, alpha=-step)
    r = plan.project(f.detach()) - g
    losses.append((r * r).sum())
    return f.detach(), [float(x) for x in torch.stack(losses).cpu()]
