"""Generic gradient solver for Eq. (1) on the hand-written operator pair.

Eq. (1) minimises ||y - A x||^2 + R(x) over x in a constraint set C, and
Sec. II describes the loop that solves it: project the estimate, form the
residual against the sinogram, backproject it to obtain the gradient, update.
Here the gradient comes from torch autograd through ``XctProject``, so each
iteration runs one projection and one backprojection in ``libxct.so``; the
regulariser, its gradient and the update are small elementwise passes over the
(B, N, N) estimate.

Choices where the paper names none: C is the non-negative orthant (clamp at
zero) or the whole space; R(x) = lam * TV_eps(x), the smoothed isotropic total
variation sum sqrt(dr^2 + dc^2 + eps^2) over pixels, with forward differences
down the rows (dr) and along a row (dc) that are zero past the last row and
column; a fixed step tau; x0 = 0.  The cost has no factor 1/2, as in Eq. (1),
so the data gradient is 2 A^T (A x - y).  Convergence needs tau < 2 / L with
L = 2 ||A||_2^2 + 8 lam / eps (the last term bounds the Hessian of TV_eps);
``lipschitz`` estimates L with the operator pair.
"""
from __future__ import annotations

from typing import Optional, Union

import torch
import torch.nn.functional as Fn

from .xct import Matrix, XctProject, backproject, project


def tv(x: torch.Tensor, eps: float) -> torch.Tensor:
    """TV_eps of each slice of x (B, N, N); returns (B,). Differentiable."""
    dr = Fn.pad(x[:, 1:, :] - x[:, :-1, :], (0, 0, 0, 1))
    dc = Fn.pad(x[:, :, 1:] - x[:, :, :-1], (0, 1))
    return torch.sqrt(dr * dr + dc * dc + eps * eps).sum(dim=(1, 2))


def cost(A: Matrix, x: torch.Tensor, y: torch.Tensor, lam: float = 0.0, eps: float = 1e-2) -> torch.Tensor:
    """Eq. (1) per slice: ||y - A x||^2 + lam * TV_eps(x); differentiable in x."""
    r = XctProject.apply(x, A) - y
    J = (r * r).sum(dim=(1, 2))
    return J + lam * tv(x, eps) if lam != 0.0 else J


def projected_gradient(A: Matrix, y: torch.Tensor, iters: int, step: Union[float, torch.Tensor],
                       lam: float = 0.0, eps: float = 1e-2, nonneg: bool = True,
                       x0: Optional[torch.Tensor] = None, costs: Optional[list] = None) -> torch.Tensor:
    """Projected gradient descent on Eq. (1) for a batch of sinograms.

    y: (B, n_angles, n_channels) FP32 on the matrix's GPU.  step: a float, or a
    (B,) tensor of per-slice steps.  Each iteration takes x <- P_C(x - step * g)
    with g the gradient of ``cost``.  When ``costs`` is a list, the per-slice
    cost of each iterate before its update is appended to it (one host sync per
    iteration).  Returns x (B, n, n) FP32."""
    if not isinstance(y, torch.Tensor) or y.dtype != torch.float32 or y.dim() != 3 or not y.is_cuda:
        raise TypeError("y must be a 3-D float32 CUDA tensor (B, n_angles, n_channels)")
    if tuple(y.shape[1:]) != A.sino_shape:
        raise ValueError(f"y has shape {tuple(y.shape)}, expected (B, {A.sino_shape[0]}, {A.sino_shape[1]})")
    if iters < 0 or eps <= 0.0 or lam < 0.0:
        raise ValueError("need iters >= 0, eps > 0 and lam >= 0")
    B = y.shape[0]
    y = y.contiguous()
    if x0 is None:
        x = torch.zeros((B,) + A.vol_shape, dtype=torch.float32, device=y.device)
    else:
        if x0.shape != (B,) + A.vol_shape or x0.dtype != torch.float32:
            raise ValueError("x0 must be float32 of shape (B, n, n)")
        x = x0.detach().clone()
    tau = step.reshape(B, 1, 1).to(x) if isinstance(step, torch.Tensor) else float(step)
    for _ in range(iters):
        x.requires_grad_(True)
        J = cost(A, x, y, lam, eps)
        (g,) = torch.autograd.grad(J.sum(), x)
        if costs is not None:
            costs.append(J.detach().cpu())
        with torch.no_grad():
            x = x.detach() - tau * g
            if nonneg:
                x.clamp_(min=0.0)
    return x.detach()


def opnorm_sq(A: Matrix, iters: int = 30, seed: int = 0) -> float:
    """||A||_2^2 by power iteration on A^T A with the operator pair (a lower
    bound that tightens with ``iters``)."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    v = torch.rand((1,) + A.vol_shape, generator=g, dtype=torch.float32).to(A.device)
    est = 0.0
    for _ in range(iters):
        w = backproject(A, project(A, v))
        est = float((v * w).sum() / (v * v).sum())
        v = w / w.norm()
    return est


def lipschitz(A: Matrix, lam: float = 0.0, eps: float = 1e-2, iters: int = 30) -> float:
    """Bound on the Lipschitz constant of the gradient of ``cost``:
    2 ||A||^2 (estimated, padded by 1%) + 8 lam / eps."""
    return 2.0 * 1.01 * opnorm_sq(A, iters) + (8.0 * lam / eps if lam else 0.0)
