"""FP64 oracle for the generic gradient solver of Eq. (1): constraint C and
regulariser R on top of the projection / backprojection pair.

TEST INFRASTRUCTURE ONLY.  Only the test-suite may import this module; the
product package never imports it and shares no code with it.

Eq. (1) minimises ||y - A x||^2 + R(x) over x in C, and Sec. II describes the
gradient loop that solves it: project the current estimate, form the residual
against the sinogram, backproject the residual to obtain the gradient, update
the estimate.  The paper names neither C nor R nor the step rule, so these
readings are taken:

* C is the non-negative orthant (attenuation is non-negative); the update
  projects onto it by clamping at zero, or C is the whole space.
* R(x) = lam * TV_eps(x), the smoothed isotropic total variation
  sum over pixels of sqrt(dr^2 + dc^2 + eps^2), with forward differences dr
  (down the rows) and dc (along a row) that are zero past the last row and
  column.
* The step is a fixed tau supplied by the caller, x0 = 0, and k iterations
  are k projections and k backprojections.

The cost is taken exactly as Eq. (1) writes it (no factor 1/2), so its data
gradient is 2 A^T (A x - y).

Pins (tests/test_oracle_pins.py): TV_eps and its gradient on a 2 x 3 image
against values derived by hand (tests/golden/tv_eps_2x3.txt: stencil,
orientation and boundary rule), and against the same on the transposed image;
the TV gradient against central finite differences of TV itself; the solver with lam = 0 against scipy's NNLS
active-set solution, without the constraint against Landweber's closed form
in the SVD basis after k steps, and with lam > 0 against L-BFGS-B (with
bounds) applied to the cost evaluated straight from its definition.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import backproject, project


def tv(x: np.ndarray, eps: float) -> np.ndarray:
    """TV_eps of each slice of x (B, N, N); returns (B,)."""
    x = np.asarray(x, np.float64)
    dr = np.zeros_like(x)
    dc = np.zeros_like(x)
    dr[:, :-1, :] = x[:, 1:, :] - x[:, :-1, :]
    dc[:, :, :-1] = x[:, :, 1:] - x[:, :, :-1]
    return np.sqrt(dr * dr + dc * dc + eps * eps).sum(axis=(1, 2))


def tv_grad(x: np.ndarray, eps: float) -> np.ndarray:
    """Gradient of TV_eps with respect to x (B, N, N), derived by hand: pixel
    (i, j) enters dr at (i, j) with sign -1 and at (i-1, j) with sign +1, and
    dc at (i, j) with -1 and at (i, j-1) with +1; each term contributes
    d / m with m = sqrt(dr^2 + dc^2 + eps^2) at that term's pixel."""
    x = np.asarray(x, np.float64)
    dr = np.zeros_like(x)
    dc = np.zeros_like(x)
    dr[:, :-1, :] = x[:, 1:, :] - x[:, :-1, :]
    dc[:, :, :-1] = x[:, :, 1:] - x[:, :, :-1]
    m = np.sqrt(dr * dr + dc * dc + eps * eps)
    u = dr / m
    v = dc / m
    g = np.zeros_like(x)
    g[:, :-1, :] -= u[:, :-1, :]
    g[:, 1:, :] += u[:, :-1, :]
    g[:, :, :-1] -= v[:, :, :-1]
    g[:, :, 1:] += v[:, :, :-1]
    return g


def cost(A: sp.csr_matrix, x: np.ndarray, y: np.ndarray, lam: float, eps: float) -> np.ndarray:
    """Eq. (1) per slice: ||y - A x||^2 + lam * TV_eps(x); x (B, N, N), y (B, M*C)."""
    x = np.asarray(x, np.float64)
    r = project(A, x) - np.asarray(y, np.float64).reshape(x.shape[0], -1)
    return (r * r).sum(axis=1) + lam * tv(x, eps)


def projected_gradient(A: sp.csr_matrix, AT: sp.csr_matrix, y: np.ndarray, iters: int, step: float,
                       lam: float = 0.0, eps: float = 1e-2, nonneg: bool = True) -> np.ndarray:
    """The Sec. II gradient loop for Eq. (1) from x0 = 0, per slice.

    y: (B, M*C) or (B, M, C).  Each iteration: r = A x - y (projection and
    residual), g = 2 A^T r + lam * grad TV_eps(x) (backprojection gives the
    data gradient), x <- x - step * g, then x <- max(x, 0) when C is the
    non-negative orthant.  Returns x (B, N, N)."""
    y = np.asarray(y, np.float64)
    B = y.shape[0]
    y = y.reshape(B, -1)
    N = int(round(np.sqrt(A.shape[1])))
    x = np.zeros((B, N, N), np.float64)
    for _ in range(iters):
        r = project(A, x) - y
        g = 2.0 * backproject(AT, r).reshape(B, N, N)
        if lam != 0.0:
            g = g + lam * tv_grad(x, eps)
        x = x - step * g
        if nonneg:
            x = np.maximum(x, 0.0)
    return x
