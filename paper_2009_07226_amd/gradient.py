"""Generic gradient solver for Eq. (1) on the hand-written operator pair.

Eq. (1) minimises ||y - A x||^2 + R(x) over x in a constraint set C, and
Sec. II describes the loop that solves it: project the estimate, form the
residual against the sinogram, backproject it to obtain the gradient, update.
``projected_gradient`` runs the whole loop in ``libxct.so``: per iteration one
projection, one backprojection, a residual pass and one fused pass that
evaluates the TV gradient, takes the step and clamps.  ``cost`` and ``tv`` are
the same objective written with torch autograd through ``XctProject``, for
callers who build their own objectives on the operator pair.

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
from .xct import projected_gradient as _native_pg


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
                       x0: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Projected gradient descent on Eq. (1) for a batch of sinograms, run
    entirely in ``libxct.so`` (``xct_projected_gradient``): each iteration
    takes x <- P_C(x - step * g) with g the gradient of ``cost``.

    y: (B, n_angles, n_channels) FP32 on the matrix's GPU.  step: a float, or a
    (B,) tensor of per-slice steps.  Returns x (B, n, n) FP32."""
    if not isinstance(y, torch.Tensor) or y.dtype != torch.float32 or y.dim() != 3 or not y.is_cuda:
        raise TypeError("y must be a 3-D float32 CUDA tensor (B, n_angles, n_channels)")
    return _native_pg(A, y.contiguous(), iters, step, lam=lam, eps=eps, nonneg=nonneg, x0=x0)


def opnorm_sq(A: Matrix, iters: int = 30, seed: int = 0) -> float:
    """||A||_2^2 by power iteration on A^T A with the operator pair (a lower
    bound that tightens with ``iters``).

    A caller-side helper for choosing the step length, not part of the
    solver: each iteration is one projection and one backprojection through
    the library; the scalar bookkeeping (two dot products and a scaling per
    iteration) is done with torch on the device, once per step-length choice."""
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
