// Projected gradient descent on Eq. (1), ||y - A x||^2 + lam * TV_eps(x)
// over x in C, with the gradient loop of Sec. II: project the estimate, form
// the residual, backproject it (the data gradient is 2 A^T (A x - y)), update.
// C is the non-negative orthant (clamp at zero) or the whole space; TV_eps is
// the smoothed isotropic total variation, sum over pixels of
// sqrt(dr^2 + dc^2 + eps^2) with forward differences dr (down the rows) and
// dc (along a row) that are zero past the last row and column.
//
// Per iteration: one projection and one backprojection (the staged SpMM),
// one residual pass over the sinograms, and one fused pass over the volume
// that evaluates the TV gradient from a 3 x 3 neighbourhood, takes the step
// and clamps.  The volume update is out of place (the stencil reads the old
// iterate), so the iterate alternates between the caller's buffer and one in
// the workspace.
#include <algorithm>
#include <climits>
#include <utility>

#include "common.hpp"

namespace xct {

static size_t align256g(size_t b) { return (b + 255) & ~(size_t)255; }

struct PgWs {
    float *q, *s, *xalt;
    void *spmm;
};

// q = A x and r = q - y (in place) [B][M*C]; s = A^T r [B][N*N]; the other
// iterate buffer [B][N*N]; then the SpMM workspace.
static size_t pg_ws_layout(const xct_matrix *m, int batch, char *base, PgWs *w) {
    const size_t vol = align256g((size_t)batch * m->n * m->n * sizeof(float));
    const size_t sino = align256g((size_t)batch * m->M * m->C * sizeof(float));
    if (w) {
        w->q = (float *)base;
        w->s = (float *)(base + sino);
        w->xalt = (float *)(base + sino + vol);
        w->spmm = base + sino + 2 * vol;
    }
    return sino + 2 * vol + spmm_workspace(m, batch);
}

__global__ void __launch_bounds__(256) k_residual(float *__restrict__ q, const float *__restrict__ y, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) q[i] = q[i] - y[i];
}

// Rows of one column handled by one thread of k_pg_update.
constexpr int kPgRows = 8;

// x_out = P_C(x - tau_b (2 s + lam grad TV_eps(x))).  With u = dr / m and
// v = dc / m at a pixel (m = sqrt(dr^2 + dc^2 + eps^2)), the TV gradient at
// (i, j) is -(u + v)(i, j) + u(i-1, j) + v(i, j-1).
// One thread per column and kPgRows consecutive rows; one workgroup per
// 256-column segment of a kPgRows-row strip of one slice.  Every load of the
// strip (rows i0-1 .. i0+kPgRows at columns j-1, j, j+1, clamped into the
// slice) is issued before any arithmetic, so each wave waits for memory once
// per kPgRows rows, and u of the row above is carried from the previous row.
// Workgroups are dealt round-robin to the 8 XCDs, so the linear id is
// remapped to give each XCD a contiguous range of (slice, strip, segment):
// the rows just above and below a strip are then read by the same XCD.
__global__ void __launch_bounds__(256) k_pg_update(const float *__restrict__ x, const float *__restrict__ s,
                                                   float *__restrict__ xo, const float *__restrict__ tau, int N,
                                                   int nseg, int nstrip, int nblocks, float lam, float eps2,
                                                   int nonneg) {
    constexpr int R = kPgRows;
    int L = blockIdx.x;
    if ((nblocks & 7) == 0) L = (L & 7) * (nblocks >> 3) + (L >> 3);
    const int seg = L % nseg;
    const int q = L / nseg;  // b * nstrip + strip
    const int i0 = (q % nstrip) * R;
    const int b = q / nstrip;
    const int j = seg * 256 + (int)threadIdx.x;
    if (j >= N) return;
    const bool left = j > 0, right = j + 1 < N;
    const int jm = left ? j - 1 : j, jp = right ? j + 1 : j;
    const float *xs = x + (int64_t)b * N * N;
    auto row = [&](int i) { return xs + (int64_t)min(max(i, 0), N - 1) * N; };
    // cj[k], cr[k]: rows i0-1+k at columns j, j+1; cl[k]: row i0+k at column j-1.
    float cj[R + 2], cr[R + 1], cl[R + 1], sp[R];
#pragma unroll
    for (int k = 0; k < R + 2; ++k) cj[k] = row(i0 - 1 + k)[j];
#pragma unroll
    for (int k = 0; k < R + 1; ++k) cr[k] = row(i0 - 1 + k)[jp];
#pragma unroll
    for (int k = 0; k < R + 1; ++k) cl[k] = row(i0 + k)[jm];
    const int64_t p0 = ((int64_t)b * N + i0) * N + j;
    const float *ss = s + (int64_t)b * N * N;
#pragma unroll
    for (int r = 0; r < R; ++r) sp[r] = ss[(int64_t)min(i0 + r, N - 1) * N + j];  // rows past N unused
    const float tb = tau[b];
    // u at row i0-1 (used only when i0 > 0, where its dr is x[i0][j] - x[i0-1][j])
    float u_up;
    {
        const float dr = cj[1] - cj[0], dc = right ? cr[0] - cj[0] : 0.0f;
        u_up = dr / sqrtf(dr * dr + dc * dc + eps2);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = i0 + r;
        const bool up = i > 0, down = i + 1 < N;
        const float c = cj[r + 1];
        // (i, j): dr = x[i+1][j] - x[i][j], dc = x[i][j+1] - x[i][j]
        const float dr0 = down ? cj[r + 2] - c : 0.0f, dc0 = right ? cr[r + 1] - c : 0.0f;
        const float m0 = sqrtf(dr0 * dr0 + dc0 * dc0 + eps2);
        const float u0 = dr0 / m0, v0 = dc0 / m0;
        // (i, j-1): dr = x[i+1][j-1] - x[i][j-1], dc = x[i][j] - x[i][j-1]
        const float dr2 = down ? cl[r + 1] - cl[r] : 0.0f, dc2 = c - cl[r];
        const float v2 = dc2 / sqrtf(dr2 * dr2 + dc2 * dc2 + eps2);
        // Branch-free: every term is finite (eps2 > 0) and the edge rules
        // select it; lam = 0 adds 0 * t = 0.
        const float t = -(u0 + v0) + (up ? u_up : 0.0f) + (left ? v2 : 0.0f);
        float xn = c - tb * (2.0f * sp[r] + lam * t);
        if (nonneg) xn = fmaxf(xn, 0.0f);
        if (i < N) xo[p0 + (int64_t)r * N] = xn;
        u_up = u0;
    }
}

static unsigned grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    return (unsigned)std::min<int64_t>(g, 8 * 256 * 16);
}

}  // namespace xct

using namespace xct;

extern "C" size_t xct_pgrad_workspace_bytes(const xct_matrix *m, int batch) {
    if (!m || batch < 1) return 0;
    return pg_ws_layout(m, batch, nullptr, nullptr);
}

extern "C" int xct_projected_gradient(const xct_matrix *m, const float *y, float *x, int batch, int iters,
                                      const float *step, float lam, float eps, int nonneg, void *workspace,
                                      void *stream) {
    if (!m || !y || !x || !step || !workspace) return fail(XCT_ERR_INVALID, "NULL argument");
    if (batch < 1) return fail(XCT_ERR_INVALID, "batch must be >= 1");
    if (iters < 0) return fail(XCT_ERR_INVALID, "iters must be >= 0");
    if (!(lam >= 0.0f) || !(eps > 0.0f)) return fail(XCT_ERR_INVALID, "need lam >= 0 and eps > 0");
    if (((uintptr_t)workspace & 255) != 0) return fail(XCT_ERR_INVALID, "workspace must be 256-byte aligned");
    PgWs w;
    pg_ws_layout(m, batch, (char *)workspace, &w);
    hipStream_t st = (hipStream_t)stream;
    const int64_t n_vol = (int64_t)batch * m->n * m->n, n_sino = (int64_t)batch * m->M * m->C;
    const int nseg = (m->n + 255) / 256;
    const int nstrip = (m->n + kPgRows - 1) / kPgRows;
    const int64_t nblocks = (int64_t)nseg * nstrip * batch;
    if (nblocks > INT32_MAX) return fail(XCT_ERR_INVALID, "batch too large for one call");
    float *cur = x, *nxt = w.xalt;
    for (int k = 0; k < iters; ++k) {
        int rc;
        if (m->vdt == XCT_F64) {  // r = A x, then r -= y
            rc = spmm_call(m, 0, cur, w.q, batch, XCT_F32, w.spmm, stream);
            if (rc != XCT_OK) return rc;
            hipLaunchKernelGGL(k_residual, dim3(grid_for(n_sino)), dim3(256), 0, st, w.q, y, n_sino);
            XCT_HIP_TRY(hipGetLastError());
        } else {  // r = A x - y as the projection is written out
            rc = spmm_residual(m, cur, y, w.q, batch, w.spmm, st);
            if (rc != XCT_OK) return rc;
        }
        rc = spmm_call(m, 1, w.q, w.s, batch, XCT_F32, w.spmm, stream);
        if (rc != XCT_OK) return rc;
        hipLaunchKernelGGL(k_pg_update, dim3((unsigned)nblocks), dim3(256), 0, st, cur, w.s, nxt, step, m->n, nseg,
                           nstrip, (int)nblocks, lam, eps * eps, nonneg ? 1 : 0);
        XCT_HIP_TRY(hipGetLastError());
        std::swap(cur, nxt);
    }
    if (cur != x) XCT_HIP_TRY(hipMemcpyAsync(x, cur, (size_t)n_vol * sizeof(float), hipMemcpyDeviceToDevice, st));
    return XCT_OK;
}
