"""Brute-force system matrix for tiny grids (N <= 16): every (ray, voxel) pair.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

For each ray L_{k,c} = {p : p.(cos th_k, sin th_k) = t_c} and each voxel the
chord length is found from the points where the line meets the voxel's four
edges (segment-line intersection); the chord is the largest distance between
those points.  An edge lying on the line is the chord and counts half (the
line is shared by two voxels).  This is a third, independent way of getting
the entries of A (the C oracle traces rays with Siddon's method and clips
voxels with slab clipping).  Geometry readings as in xct_oracle.c.
"""
from __future__ import annotations

import math

import numpy as np

DROP = 1e-9


def _angle(M: int, k: int):
    if k == 0:
        return 1.0, 0.0
    if 2 * k == M:
        return 0.0, 1.0
    th = math.pi * k / M
    return math.cos(th), math.sin(th)


def chord_in_box(x0, x1, y0, y1, cs, sn, t):
    """Chord of the line p.(cs, sn) = t through the boxes [x0,x1]x[y0,y1]
    (arrays), by intersecting the line with each box edge."""
    x0, x1, y0, y1 = map(np.asarray, (x0, x1, y0, y1))
    corners = [(x0, y0), (x1, y0), (x1, y1), (x0, y1)]
    pts_x, pts_y, on_edge = [], [], np.zeros(np.broadcast(x0, y0).shape, bool)
    edge_len = np.zeros(np.broadcast(x0, y0).shape)
    for e in range(4):
        (px, py), (qx, qy) = corners[e], corners[(e + 1) % 4]
        fp = px * cs + py * sn - t
        fq = qx * cs + qy * sn - t
        den = fp - fq
        with np.errstate(divide="ignore", invalid="ignore"):
            s = np.where(den != 0, fp / np.where(den != 0, den, 1.0), np.nan)
        hit = (den != 0) & (s >= 0) & (s <= 1)
        pts_x.append(np.where(hit, px + s * (qx - px), np.nan))
        pts_y.append(np.where(hit, py + s * (qy - py), np.nan))
        lies = (fp == 0) & (fq == 0)
        on_edge |= lies
        edge_len = np.where(lies, np.hypot(qx - px, qy - py), edge_len)
    X = np.stack(pts_x)
    Y = np.stack(pts_y)
    best = np.zeros(X.shape[1:])
    for a in range(4):
        for b in range(a + 1, 4):
            d = np.hypot(X[a] - X[b], Y[a] - Y[b])
            best = np.fmax(best, np.nan_to_num(d, nan=0.0))
    return np.where(on_edge, 0.5 * edge_len, best)


def dense_A(N: int, M: int, C: int) -> np.ndarray:
    """Dense (M*C) x (N*N) matrix, every entry computed independently."""
    assert N <= 32
    h = N / 2.0
    ii, jj = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    x0 = (jj - h).ravel().astype(float)
    y0 = (ii - h).ravel().astype(float)
    A = np.zeros((M * C, N * N))
    for k in range(M):
        cs, sn = _angle(M, k)
        for c in range(C):
            t = c - (C - 1) / 2.0
            L = chord_in_box(x0, x0 + 1, y0, y0 + 1, cs, sn, t)
            L[L < DROP] = 0.0
            A[k * C + c] = L
    return A
