// Parallel-beam geometry on the device, in FP64.
//
// Conventions (see include/xct.h): n x n unit voxels centred on the axis,
// theta_k = k*pi/M, line (k, c) = {p : p.(cos, sin) = c - (C-1)/2}; a line
// on a voxel edge gives half its length to each neighbour; lengths below
// kDrop are dropped.  Sec. II-A of the paper asks for exact intersection
// lengths (Siddon); two independent ways of getting them are used:
//   trace_ray   -- ray-driven incremental Siddon traversal (rows of A),
//   trace_voxel -- voxel-driven closed form (rows of A^T): the chord of a
//                  line through a unit square is a trapezoid in the line's
//                  offset from the square's centre.
//
// The functions only use <cmath>, so the test-suite also compiles this file
// for the host (with __host__/__device__/__forceinline__ defined away) and
// checks it against the CPU oracle.
#pragma once

#include <cmath>

namespace xct {

// Lengths below this are dropped (corner touches).
constexpr double kDrop = 1e-9;

__host__ __device__ __forceinline__ void angle_cs(int M, int k, double &cs, double &sn) {
    if (k == 0) { cs = 1.0; sn = 0.0; return; }
    if (2 * k == M) { cs = 0.0; sn = 1.0; return; }
    double th = M_PI * (double)k / (double)M;
    sincos(th, &sn, &cs);
}

// Visit every voxel (i, j) crossed by ray (k, c) with its length.
template <class V>
__host__ __device__ __forceinline__ void trace_ray(int N, int M, int C, int k, int c, V &&visit) {
    double cs, sn;
    angle_cs(M, k, cs, sn);
    const double t = (double)c - 0.5 * (double)(C - 1);
    const double px = t * cs, py = t * sn;  // foot point
    const double dx = -sn, dy = cs;         // direction
    const double h = 0.5 * (double)N;
    if (dx == 0.0) {  // theta = 0: the line x = px
        if (px < -h || px > h) return;
        const double xg = px + h;
        const double fl = floor(xg);
        if (fl == xg) {  // on a column edge: half to each side
            const int jb = (int)xg;
            for (int i = 0; i < N; ++i) {
                if (jb - 1 >= 0) visit(i, jb - 1, 0.5);
                if (jb < N) visit(i, jb, 0.5);
            }
        } else {
            const int j = (int)fl;
            for (int i = 0; i < N; ++i) visit(i, j, 1.0);
        }
        return;
    }
    if (dy == 0.0) {  // theta = pi/2: the line y = py
        if (py < -h || py > h) return;
        const double yg = py + h;
        const double fl = floor(yg);
        if (fl == yg) {
            const int ib = (int)yg;
            for (int j = 0; j < N; ++j) {
                if (ib - 1 >= 0) visit(ib - 1, j, 0.5);
                if (ib < N) visit(ib, j, 0.5);
            }
        } else {
            const int i = (int)fl;
            for (int j = 0; j < N; ++j) visit(i, j, 1.0);
        }
        return;
    }
    const double ax1 = (-h - px) / dx, ax2 = (h - px) / dx;
    const double ay1 = (-h - py) / dy, ay2 = (h - py) / dy;
    const double amin = fmax(fmin(ax1, ax2), fmin(ay1, ay2));
    const double amax = fmin(fmax(ax1, ax2), fmax(ay1, ay2));
    if (!(amax - amin > kDrop)) return;
    const int sx = dx > 0.0 ? 1 : -1, sy = dy > 0.0 ? 1 : -1;
    // Start one plane behind the entry point and step forward past it, so
    // no crossing after the entry can be missed through rounding.
    // (The entry point may round to just outside the grid: clamp to the
    // boundary plane, whose parameter is then <= amin and is stepped over.)
    int gx = (int)(dx > 0.0 ? floor(px + amin * dx + h) : ceil(px + amin * dx + h));
    int gy = (int)(dy > 0.0 ? floor(py + amin * dy + h) : ceil(py + amin * dy + h));
    gx = gx < 0 ? 0 : (gx > N ? N : gx);
    gy = gy < 0 ? 0 : (gy > N ? N : gy);
    auto ax_of = [&](int g) { return (g >= 0 && g <= N) ? (((double)g - h) - px) / dx : INFINITY; };
    auto ay_of = [&](int g) { return (g >= 0 && g <= N) ? (((double)g - h) - py) / dy : INFINITY; };
    double axn = ax_of(gx), ayn = ay_of(gy);
    for (int guard = 0; axn <= amin && guard < 4; ++guard) { gx += sx; axn = ax_of(gx); }
    for (int guard = 0; ayn <= amin && guard < 4; ++guard) { gy += sy; ayn = ay_of(gy); }
    double acur = amin;
    for (int step = 0; step < 2 * N + 4; ++step) {
        const double anext = fmin(fmin(axn, ayn), amax);
        const double len = anext - acur;
        if (len >= kDrop) {
            const double am = 0.5 * (acur + anext);
            int j = (int)floor(px + am * dx + h);
            int i = (int)floor(py + am * dy + h);
            j = j < 0 ? 0 : (j >= N ? N - 1 : j);
            i = i < 0 ? 0 : (i >= N ? N - 1 : i);
            visit(i, j, len);
        }
        if (anext >= amax) break;
        if (axn == anext) { gx += sx; axn = ax_of(gx); }
        if (ayn == anext) { gy += sy; ayn = ay_of(gy); }
        acur = anext;
    }
}

// Visit every ray (k, c) crossing voxel (i, j) with its length, angle by
// angle.  The chord of the line at offset u from the voxel centre, with
// a = |cos|, b = |sin|, is min(min(a, b), (a + b)/2 - u) / (a b), clipped at
// zero (for b = 0 or a = 0: 1 inside, 1/2 on the edge).
template <class V>
__host__ __device__ __forceinline__ void trace_voxel(int N, int M, int C, int i, int j, V &&visit) {
    const double h = 0.5 * (double)N;
    const double xc = (double)j - h + 0.5, yc = (double)i - h + 0.5;
    const double off = 0.5 * (double)(C - 1);
    for (int k = 0; k < M; ++k) {
        double cs, sn;
        angle_cs(M, k, cs, sn);
        const double a = fabs(cs), b = fabs(sn);
        const double tc = xc * cs + yc * sn;
        const double w = 0.5 * (a + b);
        int clo = (int)ceil(tc - w + off) - 1;
        int chi = (int)floor(tc + w + off) + 1;
        clo = clo < 0 ? 0 : clo;
        chi = chi > C - 1 ? C - 1 : chi;
        for (int c = clo; c <= chi; ++c) {
            const double u = fabs(((double)c - off) - tc);
            double len;
            if (b == 0.0 || a == 0.0)
                len = u < 0.5 ? 1.0 : (u == 0.5 ? 0.5 : 0.0);
            else
                len = fmin(fmin(a, b), fmax(0.0, w - u)) / (a * b);
            if (len >= kDrop) visit(k, c, len);
        }
    }
}

}  // namespace xct
