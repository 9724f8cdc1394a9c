/* Drives every entry point of the C oracle on small scans so that the CPU
 * test-suite can run it under AddressSanitizer and UndefinedBehaviorSanitizer
 * (the oracle's source is compiled into this program).  Exits non-zero if a
 * product disagrees with its transpose or CGLS leaves its invariants. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/xct_oracle.c"

static int check_scan(int N, int M, int C)
{
    const int64_t R = (int64_t)M * C, V = (int64_t)N * N;
    int64_t *ca = calloc((size_t)R + 1, sizeof *ca), *ct = calloc((size_t)V + 1, sizeof *ct);
    oracle_counts_A(N, M, C, ca + 1);
    oracle_counts_AT(N, M, C, ct + 1);
    for (int64_t r = 0; r < R; ++r) ca[r + 1] += ca[r];
    for (int64_t v = 0; v < V; ++v) ct[v + 1] += ct[v];
    if (ca[R] != ct[V]) return 1;
    const int64_t nnz = ca[R];
    int32_t *ac = malloc(sizeof(int32_t) * (size_t)(nnz + 1)), *tc = malloc(sizeof(int32_t) * (size_t)(nnz + 1));
    double *av = malloc(sizeof(double) * (size_t)(nnz + 1)), *tv = malloc(sizeof(double) * (size_t)(nnz + 1));
    oracle_fill_A(N, M, C, ca, ac, av);
    oracle_fill_AT(N, M, C, ct, tc, tv);
    const int B = 2;
    double *x = malloc(sizeof(double) * (size_t)(B * V)), *y = malloc(sizeof(double) * (size_t)(B * R));
    double *ax = malloc(sizeof(double) * (size_t)(B * R)), *aty = malloc(sizeof(double) * (size_t)(B * V));
    for (int64_t q = 0; q < B * V; ++q) x[q] = (double)((q * 7919) % 101) / 101.0;
    for (int64_t q = 0; q < B * R; ++q) y[q] = (double)((q * 104729) % 97) / 97.0;
    oracle_csr_spmm(R, ca, ac, av, V, B, x, ax);
    oracle_csr_spmm(V, ct, tc, tv, R, B, y, aty);
    for (int b = 0; b < B; ++b) {  /* adjoint identity between the two builds */
        double s1 = 0, s2 = 0, n1 = 0, n2 = 0;
        for (int64_t r = 0; r < R; ++r) { s1 += ax[b * R + r] * y[b * R + r]; n1 += y[b * R + r] * y[b * R + r]; }
        for (int64_t v = 0; v < V; ++v) { s2 += x[b * V + v] * aty[b * V + v]; n2 += x[b * V + v] * x[b * V + v]; }
        if (fabs(s1 - s2) > 1e-10 * (1 + fabs(s1))) return 2;
    }
    int64_t rows[3] = {0, R / 2, R - 1}, vox[3] = {0, V / 2, V - 1};
    double pr[3 * 2], bv[3 * 2];
    oracle_project_rows(N, M, C, B, x, 3, rows, pr);
    oracle_backproject_voxels(N, M, C, B, y, 3, vox, bv);
    for (int b = 0; b < B; ++b)
        for (int q = 0; q < 3; ++q) {
            if (fabs(pr[b * 3 + q] - ax[b * R + rows[q]]) > 1e-12) return 3;
            if (fabs(bv[b * 3 + q] - aty[b * V + vox[q]]) > 1e-12) return 4;
        }
    const int K = 4;
    double *xs = malloc(sizeof(double) * (size_t)(B * V)), *res = malloc(sizeof(double) * (size_t)((K + 1) * B));
    double *xh = malloc(sizeof(double) * (size_t)(K * B * V));
    int st[2];
    oracle_cgls(R, ca, ac, av, V, ct, tc, tv, B, y, K, xs, res, st, xh);
    for (int k = 0; k < K; ++k)
        for (int b = 0; b < B; ++b)
            if (res[(k + 1) * B + b] > res[k * B + b] + 1e-12) return 5;
    void *h = oracle_traced_build(N, M, C);
    if (!h || oracle_traced_nnz(h) != nnz) return 6;
    double *tx = malloc(sizeof(double) * (size_t)(B * V)), *tr = malloc(sizeof(double) * (size_t)((K + 1) * B));
    oracle_traced_project(h, B, x, ax);
    oracle_traced_backproject(h, B, y, aty);
    oracle_traced_cgls(h, B, y, K, tx, tr, st, NULL);
    for (int64_t q = 0; q < B * V; ++q)
        if (fabs(tx[q] - xs[q]) > 1e-9 * (1 + fabs(xs[q]))) return 7;
    oracle_traced_free(h);
    free(ca); free(ct); free(ac); free(tc); free(av); free(tv); free(x); free(y); free(ax); free(aty);
    free(xs); free(res); free(xh); free(tx); free(tr);
    return 0;
}

int main(void)
{
    const int scans[][3] = {{1, 1, 1}, {2, 4, 2}, {5, 7, 6}, {16, 12, 16}, {37, 23, 41}, {24, 10, 23}, {64, 1, 64}};
    for (size_t s = 0; s < sizeof scans / sizeof scans[0]; ++s) {
        const int rc = check_scan(scans[s][0], scans[s][1], scans[s][2]);
        if (rc) {
            fprintf(stderr, "scan %d x %d x %d: check %d failed\n", scans[s][0], scans[s][1], scans[s][2], rc);
            return rc;
        }
    }
    puts("oracle sanitizer run ok");
    return 0;
}
