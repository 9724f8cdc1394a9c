"""Seeded synthetic inputs: ellipse / ellipsoid phantoms and Gaussian noise.

This module holds no part of the reconstruction arithmetic: it only draws
random shapes and random numbers.  Both the GPU path and the CPU oracle are
fed from it, so a parity test always compares the two on one array.

Recipe (the paper's datasets are not available; these stand in for the
shapes of its Table II workloads):
  * Voxel (i, j) of an N x N slice has its centre at
    (j - N/2 + 1/2, i - N/2 + 1/2); slice b of a B-slice slab sits at
    z = b - B/2 + 1/2.
  * Each ellipse has semi-axes drawn from U[0.05, 0.35] * N/2, a rotation
    from U[0, pi) and a density from U[0, 1]; its centre is uniform over the
    disc that keeps the whole ellipse inside the inscribed circle of radius
    N/2.  Ellipsoids add a z semi-axis from U[0.3, 1.0] * B/2 and a z centre
    from U[-B/2, B/2]; the rotation is in-plane.
  * Densities add where shapes overlap; a voxel takes the sum of the
    densities of the shapes that contain its centre (point sampling).
  * An optional texture adds amplitude * U[0, 1) to every voxel inside the
    inscribed circle.
  * Noise is standard normal, drawn per slice from
    numpy.random.default_rng([seed, b]) so that any subset of slices can be
    regenerated on its own.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def _shapes(rng: np.random.Generator, N: int, n: int, B: int | None):
    out = []
    half = N / 2.0
    for _ in range(n):
        a, b = rng.uniform(0.05, 0.35, size=2) * half
        phi = rng.uniform(0.0, math.pi)
        rho = rng.uniform(0.0, 1.0)
        rin = half - max(a, b)
        rr = rin * math.sqrt(rng.uniform())
        ang = rng.uniform(0.0, 2.0 * math.pi)
        cx, cy = rr * math.cos(ang), rr * math.sin(ang)
        if B is None:
            out.append((cx, cy, a, b, phi, rho, 0.0, math.inf))
        else:
            cz = rng.uniform(-B / 2.0, B / 2.0)
            c = rng.uniform(0.3, 1.0) * B / 2.0
            out.append((cx, cy, a, b, phi, rho, cz, c))
    return out


def _render(shapes, N: int, B: int, device, texture: float, seed: int) -> torch.Tensor:
    dev = torch.device(device)
    vol = torch.zeros((B, N, N), dtype=torch.float64, device=dev)
    half = N / 2.0
    for (cx, cy, a, b, phi, rho, cz, c) in shapes:
        r = max(a, b)
        j0 = max(0, int(math.floor(cx - r + half)) - 1)
        j1 = min(N, int(math.ceil(cx + r + half)) + 1)
        i0 = max(0, int(math.floor(cy - r + half)) - 1)
        i1 = min(N, int(math.ceil(cy + r + half)) + 1)
        if math.isinf(c):
            b0, b1 = 0, B
        else:
            b0 = max(0, int(math.floor(cz - c + B / 2.0)) - 1)
            b1 = min(B, int(math.ceil(cz + c + B / 2.0)) + 1)
        if j0 >= j1 or i0 >= i1 or b0 >= b1:
            continue
        xs = torch.arange(j0, j1, dtype=torch.float64, device=dev) - half + 0.5 - cx
        ys = torch.arange(i0, i1, dtype=torch.float64, device=dev) - half + 0.5 - cy
        cp, sp = math.cos(phi), math.sin(phi)
        u = xs[None, :] * cp + ys[:, None] * sp
        w = ys[:, None] * cp - xs[None, :] * sp
        q2 = u * u * (1.0 / (a * a)) + w * w * (1.0 / (b * b))
        if math.isinf(c):
            inside = (q2 <= 1.0)[None].expand(b1 - b0, -1, -1)
        else:
            zs = torch.arange(b0, b1, dtype=torch.float64, device=dev) - B / 2.0 + 0.5 - cz
            inside = (q2[None] + (zs * zs * (1.0 / (c * c)))[:, None, None]) <= 1.0
        vol[b0:b1, i0:i1, j0:j1] += inside.to(torch.float64) * rho
    if texture > 0.0:
        g = torch.Generator(device="cpu").manual_seed(int(seed) * 7919 + 17)
        tex = torch.rand((B, N, N), generator=g, dtype=torch.float64).to(dev)
        cen = torch.arange(N, dtype=torch.float64, device=dev) - half + 0.5
        disc = (cen[None, :] ** 2 + cen[:, None] ** 2) <= half * half
        vol += texture * tex * disc[None]
    return vol


def ellipse_phantom(N: int, n_ellipses: int, seed: int, device="cpu") -> torch.Tensor:
    """One N x N slice of `n_ellipses` random ellipses, shape (1, N, N), FP64."""
    rng = np.random.default_rng(seed)
    return _render(_shapes(rng, N, n_ellipses, None), N, 1, device, 0.0, seed)


def ellipse_batch(N: int, B: int, n_ellipses: int, seed: int, device="cpu") -> torch.Tensor:
    """B independent 2D ellipse slices; slice b uses seed [seed, b]."""
    out = []
    for b in range(B):
        rng = np.random.default_rng([seed, b])
        out.append(_render(_shapes(rng, N, n_ellipses, None), N, 1, device, 0.0, seed))
    return torch.cat(out, 0)


def ellipsoid_phantom(N: int, B: int, n_ellipsoids: int, seed: int, device="cpu",
                      texture: float = 0.0) -> torch.Tensor:
    """A B x N x N slab of `n_ellipsoids` random ellipsoids, FP64."""
    rng = np.random.default_rng(seed)
    return _render(_shapes(rng, N, n_ellipsoids, B), N, B, device, texture, seed)


def noise(shape_per_slice, slices, seed: int) -> np.ndarray:
    """Standard-normal noise for the listed slice indices, FP64 numpy array of
    shape (len(slices), *shape_per_slice); slice b from default_rng([seed, b])."""
    n = int(np.prod(shape_per_slice))
    out = np.empty((len(slices), n), np.float64)
    for q, b in enumerate(slices):
        out[q] = np.random.default_rng([int(seed), int(b)]).standard_normal(n)
    return out.reshape((len(slices),) + tuple(shape_per_slice))


def noise_torch(shape_per_slice, B: int, seed: int, device) -> torch.Tensor:
    """Standard-normal noise drawn on `device` with torch's generator (for
    sizes where host generation is slow); slice b seeded with seed*1000003+b."""
    out = torch.empty((B,) + tuple(shape_per_slice), dtype=torch.float32, device=device)
    for b in range(B):
        g = torch.Generator(device=device).manual_seed(int(seed) * 1000003 + b)
        out[b].normal_(generator=g)
    return out
