/*
 * xct_oracle.c -- FP64 CPU oracle for parallel-beam XCT projection,
 * backprojection and CGLS.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into oracle/liboracle.so
 * and may be loaded only by the test-suite, by the smoke check and by the
 * CPU-baseline leg of the benchmark.  The product library never links,
 * loads or calls it, and it shares no source with the GPU path.
 *
 * What it computes (Hidayetoglu et al., "Petascale XCT", SC20):
 *   - Eq. (1) with R = 0 and no constraint: the least-squares problem
 *     min ||y - A x||^2, solved by CG on the normal equations (CGLS)
 *     from x0 = 0 for a fixed iteration count (Sec. II-A, Sec. IV-F and
 *     the note under Table IV: k iterations = k projections and k+1
 *     backprojections).
 *   - A is the Siddon system matrix of a parallel-beam scan (Sec. II-A):
 *     A[(k,c),(i,j)] = length of the line L_{k,c} inside voxel (i,j).
 *     Every slice uses the same A (Sec. II-B, "fuse rays along y").
 *
 * Geometry readings (the paper fixes none of them):
 *   - N x N unit voxels centred on the rotation axis; voxel (i,j) is
 *     [j-N/2, j-N/2+1] x [i-N/2, i-N/2+1]; column index v = i*N + j.
 *   - theta_k = k*pi/M, k = 0..M-1 (the 0..179 degree example of
 *     Sec. II-A); normal n_k = (cos, sin), exact at theta = 0 and pi/2.
 *   - channel offsets t_c = c - (C-1)/2; line L_{k,c} = {p : p.n_k = t_c};
 *     row index r = k*C + c.
 *   - a line lying exactly on a voxel edge gives half its length to each
 *     of the two voxels sharing the edge; lengths below 1e-9 are dropped.
 *
 * Three independent ways of getting entries are implemented:
 *   oracle_siddon_row  -- ray-driven: Siddon's parametric crossing merge
 *                         (all plane crossings, sorted, one voxel per
 *                         interval, found from the interval midpoint);
 *   oracle_voxel_col   -- voxel-driven: for each angle, the channels whose
 *                         line can meet the voxel, each clipped against the
 *                         voxel's two slabs (Liang-Barsky);
 *   brute.py           -- every (ray, voxel) pair by edge intersection.
 *
 * Products: CSR SpMV over rows of A and of the voxel-driven A^T; for scans
 * too large to hold both, A alone (oracle_traced_*) with A^T w taken as the
 * transposed product of A's rows.  CGLS runs on either form and can return
 * every iterate.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_DROP 1e-9

static void orc_angle(int M, int k, double *cs, double *sn)
{
    if (k == 0) { *cs = 1.0; *sn = 0.0; return; }
    if (2 * k == M) { *cs = 0.0; *sn = 1.0; return; }
    double th = M_PI * (double)k / (double)M;
    *cs = cos(th);
    *sn = sin(th);
}

static double orc_offset(int C, int c) { return (double)c - 0.5 * (double)(C - 1); }

static int orc_cmp(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Row r of A by Siddon's method: collect the parameters at which the ray
 * enters and leaves the grid and crosses every grid plane, sort them, and
 * give each interval's length to the voxel holding its midpoint.
 * cols/vals must hold 2N+2 entries.  Returns the entry count. */
int64_t oracle_siddon_row(int N, int M, int C, int64_t r, int32_t *cols, double *vals)
{
    int k = (int)(r / C), c = (int)(r % C);
    double cs, sn;
    orc_angle(M, k, &cs, &sn);
    double t = orc_offset(C, c);
    double px = t * cs, py = t * sn; /* foot of the perpendicular */
    double dx = -sn, dy = cs;        /* unit direction */
    double h = 0.5 * (double)N;
    double amin = -INFINITY, amax = INFINITY;
    if (dx != 0.0) {
        double a1 = (-h - px) / dx, a2 = (h - px) / dx;
        amin = fmax(amin, fmin(a1, a2));
        amax = fmin(amax, fmax(a1, a2));
    } else if (px < -h || px > h) {
        return 0;
    }
    if (dy != 0.0) {
        double a1 = (-h - py) / dy, a2 = (h - py) / dy;
        amin = fmax(amin, fmin(a1, a2));
        amax = fmin(amax, fmax(a1, a2));
    } else if (py < -h || py > h) {
        return 0;
    }
    if (!(amax - amin > ORC_DROP)) return 0;

    double *al = (double *)malloc(sizeof(double) * (size_t)(2 * N + 6));
    int na = 0;
    al[na++] = amin;
    al[na++] = amax;
    for (int g = 0; g <= N; ++g) {
        double plane = (double)g - h;
        if (dx != 0.0) {
            double a = (plane - px) / dx;
            if (a > amin && a < amax) al[na++] = a;
        }
        if (dy != 0.0) {
            double a = (plane - py) / dy;
            if (a > amin && a < amax) al[na++] = a;
        }
    }
    qsort(al, (size_t)na, sizeof(double), orc_cmp);

    /* a line lying on a grid plane (only possible for theta = 0 or pi/2) */
    int on_x = (dx == 0.0) && (floor(px + h) == px + h);
    int on_y = (dy == 0.0) && (floor(py + h) == py + h);

    int64_t n = 0;
    for (int m = 0; m + 1 < na; ++m) {
        double len = al[m + 1] - al[m];
        if (len < ORC_DROP) continue;
        double am = 0.5 * (al[m] + al[m + 1]);
        double x = px + am * dx, y = py + am * dy;
        int j = (int)floor(x + h), i = (int)floor(y + h);
        if (on_x) {
            int jb = (int)(px + h); /* the plane x = jb - h */
            for (int q = jb - 1; q <= jb; ++q) {
                if (q < 0 || q >= N || i < 0 || i >= N) continue;
                cols[n] = i * N + q;
                vals[n] = 0.5 * len;
                ++n;
            }
            continue;
        }
        if (on_y) {
            int ib = (int)(py + h);
            for (int q = ib - 1; q <= ib; ++q) {
                if (q < 0 || q >= N || j < 0 || j >= N) continue;
                cols[n] = q * N + j;
                vals[n] = 0.5 * len;
                ++n;
            }
            continue;
        }
        if (j < 0) j = 0;
        if (j >= N) j = N - 1;
        if (i < 0) i = 0;
        if (i >= N) i = N - 1;
        cols[n] = i * N + j;
        vals[n] = len;
        ++n;
    }
    free(al);
    return n;
}

/* Length of the line {p : p.(cs,sn) = t} inside [x0,x1] x [y0,y1], by
 * clipping its parametric form against the two slabs (Liang-Barsky).  A
 * line lying on an edge of the rectangle counts half. */
static double orc_clip(double x0, double x1, double y0, double y1, double t, double cs, double sn)
{
    double px = t * cs, py = t * sn, dx = -sn, dy = cs;
    double lo = -INFINITY, hi = INFINITY, w = 1.0;
    if (dx != 0.0) {
        double a1 = (x0 - px) / dx, a2 = (x1 - px) / dx;
        lo = fmax(lo, fmin(a1, a2));
        hi = fmin(hi, fmax(a1, a2));
    } else {
        if (px < x0 || px > x1) return 0.0;
        if (px == x0 || px == x1) w = 0.5;
    }
    if (dy != 0.0) {
        double a1 = (y0 - py) / dy, a2 = (y1 - py) / dy;
        lo = fmax(lo, fmin(a1, a2));
        hi = fmin(hi, fmax(a1, a2));
    } else {
        if (py < y0 || py > y1) return 0.0;
        if (py == y0 || py == y1) w = 0.5;
    }
    double len = hi - lo;
    return len > 0.0 ? w * len : 0.0;
}

/* Column v of A (row v of A^T), voxel-driven: for every angle, the
 * channels whose line can reach the voxel (from the corners' projections
 * onto the normal, widened by one channel each way) are clipped against
 * the voxel.  rows/vals must hold 4*M entries.  Returns the entry count. */
int64_t oracle_voxel_col(int N, int M, int C, int64_t v, int32_t *rows, double *vals)
{
    int i = (int)(v / N), j = (int)(v % N);
    double h = 0.5 * (double)N;
    double x0 = (double)j - h, x1 = x0 + 1.0, y0 = (double)i - h, y1 = y0 + 1.0;
    int64_t n = 0;
    for (int k = 0; k < M; ++k) {
        double cs, sn;
        orc_angle(M, k, &cs, &sn);
        double p[4] = {x0 * cs + y0 * sn, x1 * cs + y0 * sn, x0 * cs + y1 * sn, x1 * cs + y1 * sn};
        double tmin = p[0], tmax = p[0];
        for (int q = 1; q < 4; ++q) {
            tmin = fmin(tmin, p[q]);
            tmax = fmax(tmax, p[q]);
        }
        int clo = (int)floor(tmin + 0.5 * (double)(C - 1)) - 1;
        int chi = (int)ceil(tmax + 0.5 * (double)(C - 1)) + 1;
        if (clo < 0) clo = 0;
        if (chi > C - 1) chi = C - 1;
        for (int c = clo; c <= chi; ++c) {
            double len = orc_clip(x0, x1, y0, y1, orc_offset(C, c), cs, sn);
            if (len < ORC_DROP) continue;
            rows[n] = k * C + c;
            vals[n] = len;
            ++n;
        }
    }
    return n;
}

/* ---- explicit CSR forms ------------------------------------------------ */

void oracle_counts_A(int N, int M, int C, int64_t *counts)
{
    int64_t R = (int64_t)M * C;
#pragma omp parallel
    {
        int32_t *cb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * N + 2));
        double *vb = (double *)malloc(sizeof(double) * (size_t)(2 * N + 2));
#pragma omp for schedule(dynamic, 64)
        for (int64_t r = 0; r < R; ++r) counts[r] = oracle_siddon_row(N, M, C, r, cb, vb);
        free(cb);
        free(vb);
    }
}

void oracle_fill_A(int N, int M, int C, const int64_t *rowptr, int32_t *cols, double *vals)
{
    int64_t R = (int64_t)M * C;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < R; ++r) oracle_siddon_row(N, M, C, r, cols + rowptr[r], vals + rowptr[r]);
}

void oracle_counts_AT(int N, int M, int C, int64_t *counts)
{
    int64_t V = (int64_t)N * N;
#pragma omp parallel
    {
        int32_t *rb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(4 * M));
        double *vb = (double *)malloc(sizeof(double) * (size_t)(4 * M));
#pragma omp for schedule(dynamic, 16)
        for (int64_t v = 0; v < V; ++v) counts[v] = oracle_voxel_col(N, M, C, v, rb, vb);
        free(rb);
        free(vb);
    }
}

void oracle_fill_AT(int N, int M, int C, const int64_t *rowptr, int32_t *rows, double *vals)
{
    int64_t V = (int64_t)N * N;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t v = 0; v < V; ++v) oracle_voxel_col(N, M, C, v, rows + rowptr[v], vals + rowptr[v]);
}

/* Y[b][r] = sum_n vals[n] * X[b][cols[n]] over row r, for each of `batch`
 * slices (Sec. II-B: one matrix shared by every slice). */
void oracle_csr_spmm(int64_t nrows, const int64_t *rowptr, const int32_t *cols, const double *vals,
                     int64_t ncols, int batch, const double *x, double *y)
{
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < nrows; ++r) {
        for (int b = 0; b < batch; ++b) {
            const double *xb = x + (int64_t)b * ncols;
            double s = 0.0;
            for (int64_t n = rowptr[r]; n < rowptr[r + 1]; ++n) s += vals[n] * xb[cols[n]];
            y[(int64_t)b * nrows + r] = s;
        }
    }
}

/* ---- matrix-free forms on sampled rows / voxels ------------------------ */

/* out[b][q] = (A x_b)[rows[q]], tracing each requested ray on the fly. */
void oracle_project_rows(int N, int M, int C, int batch, const double *x, int64_t nq,
                         const int64_t *rows, double *out)
{
    int64_t V = (int64_t)N * N;
#pragma omp parallel
    {
        int32_t *cb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * N + 2));
        double *vb = (double *)malloc(sizeof(double) * (size_t)(2 * N + 2));
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < nq; ++q) {
            int64_t n = oracle_siddon_row(N, M, C, rows[q], cb, vb);
            for (int b = 0; b < batch; ++b) {
                double s = 0.0;
                for (int64_t e = 0; e < n; ++e) s += vb[e] * x[(int64_t)b * V + cb[e]];
                out[(int64_t)b * nq + q] = s;
            }
        }
        free(cb);
        free(vb);
    }
}

/* out[b][q] = (A^T y_b)[vox[q]], from the voxel-driven column. */
void oracle_backproject_voxels(int N, int M, int C, int batch, const double *y, int64_t nq,
                               const int64_t *vox, double *out)
{
    int64_t R = (int64_t)M * C;
#pragma omp parallel
    {
        int32_t *rb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(4 * M));
        double *vb = (double *)malloc(sizeof(double) * (size_t)(4 * M));
#pragma omp for schedule(dynamic, 16)
        for (int64_t q = 0; q < nq; ++q) {
            int64_t n = oracle_voxel_col(N, M, C, vox[q], rb, vb);
            for (int b = 0; b < batch; ++b) {
                double s = 0.0;
                for (int64_t e = 0; e < n; ++e) s += vb[e] * y[(int64_t)b * R + rb[e]];
                out[(int64_t)b * nq + q] = s;
            }
        }
        free(rb);
        free(vb);
    }
}

/* ---- CGLS ------------------------------------------------------------- */

static double orc_dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t q = 0; q < n; ++q) s += a[q] * b[q];
    return s;
}

/* The two products of CGLS for one slice: A v (nc -> nr) and A^T w
 * (nr -> nc), through an explicit CSR of A and one of A^T, or through A's
 * CSR alone (A^T w then taken as the transposed product, see below). */
typedef struct {
    int64_t nr, nc;
    const int64_t *a_ptr;
    const int32_t *a_col;
    const double *a_val;
    const int64_t *t_ptr; /* NULL: A^T w as the transposed product of A */
    const int32_t *t_col;
    const double *t_val;
} orc_ops;

/* x_b = A^T w_b from the rows of A for `batch` slices: x_b[c] = sum over
 * rows r of A[r][c] w_b[r].  Each thread adds a fixed (static) range of rows
 * into its own copy of x; the copies are then added in thread order. */
static void orc_transposed_product(const orc_ops *o, int batch, const double *w, double *x)
{
    const size_t nx = (size_t)batch * (size_t)o->nc;
    int nt = 1;
#pragma omp parallel
    {
#pragma omp single
        nt = omp_get_num_threads();
    }
    double *part = (double *)calloc((size_t)nt * nx, sizeof(double));
#pragma omp parallel num_threads(nt)
    {
        double *xt = part + (size_t)omp_get_thread_num() * nx;
#pragma omp for schedule(static)
        for (int64_t r = 0; r < o->nr; ++r)
            for (int b = 0; b < batch; ++b) {
                const double wr = w[(int64_t)b * o->nr + r];
                double *xb = xt + (size_t)b * (size_t)o->nc;
                for (int64_t n = o->a_ptr[r]; n < o->a_ptr[r + 1]; ++n) xb[o->a_col[n]] += o->a_val[n] * wr;
            }
    }
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < (int64_t)nx; ++c) {
        double v = 0.0;
        for (int t = 0; t < nt; ++t) v += part[(size_t)t * nx + (size_t)c];
        x[c] = v;
    }
    free(part);
}

/* out_b = A v_b for `batch` slices */
static void orc_apply_A(const orc_ops *o, int batch, const double *v, double *out)
{
    oracle_csr_spmm(o->nr, o->a_ptr, o->a_col, o->a_val, o->nc, batch, v, out);
}

/* out_b = A^T w_b for `batch` slices */
static void orc_apply_AT(const orc_ops *o, int batch, const double *w, double *out)
{
    if (o->t_ptr)
        oracle_csr_spmm(o->nc, o->t_ptr, o->t_col, o->t_val, o->nr, batch, w, out);
    else
        orc_transposed_product(o, batch, w, out);
}

/* CGLS (CG on A^T A x = A^T y) for each slice independently, from x = 0,
 * for exactly `iters` iterations: iters products with A and iters+1 with
 * A^T (Sec. IV-F; Table IV note).  The slices share each product (one pass
 * over the matrix for all of them) but nothing else: every slice has its own
 * alpha, beta, gamma and delta, and its sums are the same as in a run on that
 * slice alone.  resid[k*batch + b] = ||y_b - A x_k|| / ||y_b|| for
 * k = 0..iters (0 when ||y_b|| = 0).  status[b] = 1 when the slice stopped
 * early because a step length or direction became zero (gamma = 0 or
 * delta = 0), else 0; a stopped slice keeps its iterate.  xhist (nullable):
 * xhist[((k-1)*batch + b)*nc ...] = x_k of slice b for k = 1..iters. */
static void orc_cgls(const orc_ops *o, int batch, const double *y, int iters, double *x, double *resid, int *status,
                     double *xhist)
{
    const int64_t nr = o->nr, nc = o->nc;
    const size_t B = (size_t)batch;
    double *r = (double *)malloc(sizeof(double) * B * (size_t)nr);
    double *q = (double *)malloc(sizeof(double) * B * (size_t)nr);
    double *s = (double *)malloc(sizeof(double) * B * (size_t)nc);
    double *p = (double *)malloc(sizeof(double) * B * (size_t)nc);
    double *gamma = (double *)malloc(sizeof(double) * B);
    double *ynorm = (double *)malloc(sizeof(double) * B);
    int *stepped = (int *)malloc(sizeof(int) * B);
    memset(x, 0, sizeof(double) * B * (size_t)nc);
    memcpy(r, y, sizeof(double) * B * (size_t)nr);
    orc_apply_AT(o, batch, r, s);
    memcpy(p, s, sizeof(double) * B * (size_t)nc);
    for (int b = 0; b < batch; ++b) {
        const double *yb = y + (int64_t)b * nr;
        ynorm[b] = sqrt(orc_dot(nr, yb, yb));
        gamma[b] = orc_dot(nc, s + (int64_t)b * nc, s + (int64_t)b * nc);
        status[b] = 0;
        resid[b] = ynorm[b] > 0.0 ? sqrt(orc_dot(nr, yb, yb)) / ynorm[b] : 0.0;
    }
    for (int k = 0; k < iters; ++k) {
        orc_apply_A(o, batch, p, q);
        for (int b = 0; b < batch; ++b) {
            double *xb = x + (int64_t)b * nc, *pb = p + (int64_t)b * nc;
            double *rb = r + (int64_t)b * nr, *qb = q + (int64_t)b * nr;
            stepped[b] = 0;
            if (status[b]) continue;
            const double delta = orc_dot(nr, qb, qb);
            if (gamma[b] == 0.0 || delta == 0.0) {
                status[b] = 1;
                continue;
            }
            const double alpha = gamma[b] / delta;
            for (int64_t n = 0; n < nc; ++n) xb[n] += alpha * pb[n];
            for (int64_t n = 0; n < nr; ++n) rb[n] -= alpha * qb[n];
            stepped[b] = 1;
        }
        orc_apply_AT(o, batch, r, s);
        for (int b = 0; b < batch; ++b) {
            double *pb = p + (int64_t)b * nc, *sb = s + (int64_t)b * nc, *rb = r + (int64_t)b * nr;
            if (stepped[b]) {
                const double gnew = orc_dot(nc, sb, sb);
                const double beta = gnew / gamma[b];
                for (int64_t n = 0; n < nc; ++n) pb[n] = sb[n] + beta * pb[n];
                gamma[b] = gnew;
            }
            resid[(int64_t)(k + 1) * batch + b] = ynorm[b] > 0.0 ? sqrt(orc_dot(nr, rb, rb)) / ynorm[b] : 0.0;
            if (xhist)
                memcpy(xhist + ((int64_t)k * batch + b) * nc, x + (int64_t)b * nc, sizeof(double) * (size_t)nc);
        }
    }
    free(r);
    free(q);
    free(s);
    free(p);
    free(gamma);
    free(ynorm);
    free(stepped);
}

/* CGLS with an explicit CSR of A (nr x nc) and of its transpose At. */
void oracle_cgls(int64_t nr, const int64_t *a_ptr, const int32_t *a_col, const double *a_val,
                 int64_t nc, const int64_t *t_ptr, const int32_t *t_col, const double *t_val,
                 int batch, const double *y, int iters, double *x, double *resid, int *status, double *xhist)
{
    orc_ops o = {nr, nc, a_ptr, a_col, a_val, t_ptr, t_col, t_val};
    orc_cgls(&o, batch, y, iters, x, resid, status, xhist);
}

/* The scan (N, M, C) with only A stored: its CSR is traced ray by ray
 * (Siddon, as oracle_fill_A) and A^T is applied as the transposed product,
 * for scans whose A and A^T would not both fit in host memory (A alone takes
 * 12 bytes per entry).  oracle_traced_build returns NULL when the matrix
 * cannot be allocated. */
typedef struct {
    int N, M, C;
    orc_ops o;
} orc_traced;

void *oracle_traced_build(int N, int M, int C)
{
    const int64_t R = (int64_t)M * C, V = (int64_t)N * N;
    orc_traced *t = (orc_traced *)calloc(1, sizeof(orc_traced));
    int64_t *ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(R + 1));
    if (!t || !ptr) {
        free(t);
        free(ptr);
        return NULL;
    }
    oracle_counts_A(N, M, C, ptr + 1);
    ptr[0] = 0;
    for (int64_t r = 0; r < R; ++r) ptr[r + 1] += ptr[r];
    int32_t *cols = (int32_t *)malloc(sizeof(int32_t) * (size_t)ptr[R]);
    double *vals = (double *)malloc(sizeof(double) * (size_t)ptr[R]);
    if (!cols || !vals) {
        free(t);
        free(ptr);
        free(cols);
        free(vals);
        return NULL;
    }
    oracle_fill_A(N, M, C, ptr, cols, vals);
    t->N = N;
    t->M = M;
    t->C = C;
    orc_ops o = {R, V, ptr, cols, vals, NULL, NULL, NULL};
    t->o = o;
    return t;
}

int64_t oracle_traced_nnz(const void *h)
{
    const orc_traced *t = (const orc_traced *)h;
    return t->o.a_ptr[t->o.nr];
}

/* y_b = A x_b for `batch` slices (B x N^2 -> B x M C). */
void oracle_traced_project(const void *h, int batch, const double *x, double *y)
{
    const orc_traced *t = (const orc_traced *)h;
    oracle_csr_spmm(t->o.nr, t->o.a_ptr, t->o.a_col, t->o.a_val, t->o.nc, batch, x, y);
}

/* x_b = A^T w_b for `batch` slices (B x M C -> B x N^2), as the transposed
 * product of A's rows. */
void oracle_traced_backproject(const void *h, int batch, const double *w, double *x)
{
    const orc_traced *t = (const orc_traced *)h;
    orc_transposed_product(&t->o, batch, w, x);
}

/* CGLS as oracle_cgls on the traced scan. */
void oracle_traced_cgls(const void *h, int batch, const double *y, int iters, double *x, double *resid, int *status,
                        double *xhist)
{
    const orc_traced *t = (const orc_traced *)h;
    orc_cgls(&t->o, batch, y, iters, x, resid, status, xhist);
}

void oracle_traced_free(void *h)
{
    orc_traced *t = (orc_traced *)h;
    if (!t) return;
    free((void *)t->o.a_ptr);
    free((void *)t->o.a_col);
    free((void *)t->o.a_val);
    free(t);
}
