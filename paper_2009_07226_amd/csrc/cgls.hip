// Device-resident CGLS (CG on A^T A x = A^T y) for a batch of slices.
//
// The paper solves Eq. (1) with "CG iterations" whose k-th step costs one
// projection and one backprojection, plus one backprojection to start
// (Table IV note: 30 iterations = 30 projections, 31 backprojections), from
// x = 0 and for a fixed count (Sec. IV-F).  That is CGLS:
//   r = y, s = A^T r, p = s, gamma = |s|^2
//   repeat: q = A p, delta = |q|^2, alpha = gamma/delta,
//           x += alpha p, r -= alpha q, s = A^T r, gamma' = |s|^2,
//           beta = gamma'/gamma, p = s + beta p, gamma = gamma'.
// Slices are independent (Sec. II-A), so every slice has its own alpha,
// beta, gamma and delta.  Vectors stay in the internal tile layout and in
// FP32 for the whole solve; the scalars are FP64 in device memory and the
// dot products accumulate in FP64 in a fixed order (bitwise reproducible).
// |q|^2 and |s|^2 come out of the SpMM epilogue.  With a 16-bit matrix the
// operand of each product is scaled per slice by a power of two no smaller
// than its max-norm and rounded to 16 bits, and the FP32 sums are scaled
// back (Sec. III-C, adaptive normalisation, re-tuned at every product).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "common.hpp"

namespace xct {

constexpr int kVecThreads = 256;
constexpr int kVecBlocks = 1024;

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// T: the solver vectors' type, FP64 for FP64 matrices (the double-precision
// variant), else FP32.
template <class T>
struct CglsWs {
    int F = 0, n_mb = 0, Bp = 0;
    int64_t nv = 0, ns = 0;  // elements of one group's volume / sinogram vector
    T *x = nullptr, *p = nullptr, *s = nullptr, *r = nullptr, *q = nullptr;
    void *op16 = nullptr;    // one group's 16-bit operand (volume or sinogram sized)
    double *dotp = nullptr;  // [n_mb][kVecBlocks][F]
    double *sqp = nullptr;   // [n_mb][max blocks][F]
    double *gamma = nullptr, *delta = nullptr, *alpha = nullptr, *beta = nullptr, *yy = nullptr, *sum = nullptr;
    int32_t *stopped = nullptr;
    double *resid = nullptr;  // [iters+1][Bp]
    uint32_t *amax = nullptr;
    float *scale = nullptr, *inv = nullptr;
    int64_t sq_stride = 0;    // max blocks
};

template <class T>
static size_t cgls_layout(const xct_matrix *m, int batch, int iters, char *base, CglsWs<T> *w) {
    CglsWs<T> c;
    c.F = run_fuse(batch, m->fuse);
    c.n_mb = (batch + c.F - 1) / c.F;
    c.Bp = c.n_mb * c.F;
    c.nv = m->vol.n_tiles * kTileSlots * c.F;
    c.ns = m->sino.n_tiles * kTileSlots * c.F;
    c.sq_stride = std::max(m->A.n_blocks, m->AT.n_blocks);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += al256(bytes);
        return base ? (void *)(base + o) : nullptr;
    };
    c.x = (T *)take(sizeof(T) * c.nv * c.n_mb);
    c.p = (T *)take(sizeof(T) * c.nv * c.n_mb);
    c.s = (T *)take(sizeof(T) * c.nv * c.n_mb);
    c.r = (T *)take(sizeof(T) * c.ns * c.n_mb);
    c.q = (T *)take(sizeof(T) * c.ns * c.n_mb);
    if (m->vdt == XCT_F16 || m->vdt == XCT_BF16) c.op16 = take(2 * (size_t)std::max(c.nv, c.ns));
    c.dotp = (double *)take(sizeof(double) * (size_t)c.n_mb * kVecBlocks * c.F);
    c.sqp = (double *)take(sizeof(double) * (size_t)c.n_mb * c.sq_stride * c.F);
    c.gamma = (double *)take(sizeof(double) * c.Bp);
    c.delta = (double *)take(sizeof(double) * c.Bp);
    c.alpha = (double *)take(sizeof(double) * c.Bp);
    c.beta = (double *)take(sizeof(double) * c.Bp);
    c.yy = (double *)take(sizeof(double) * c.Bp);
    c.sum = (double *)take(sizeof(double) * c.Bp);
    c.stopped = (int32_t *)take(sizeof(int32_t) * c.Bp);
    c.resid = (double *)take(sizeof(double) * (size_t)(iters + 1) * c.Bp);
    c.amax = (uint32_t *)take(sizeof(uint32_t) * (size_t)c.Bp);
    c.scale = (float *)take(sizeof(float) * kMaxFuse);
    c.inv = (float *)take(sizeof(float) * kMaxFuse);
    if (w) *w = c;
    return off;
}

// ---- vector kernels (one fused group at a time) -------------------------------

// Block partial sums per slice of v^2 into part[blockIdx.x][F]; the grid
// stride is a multiple of F so each thread always sees the same slice.
__device__ __forceinline__ void block_partial(double acc, int F, double *part) {
    __shared__ double red[kVecThreads];
    red[threadIdx.x] = acc;
    __syncthreads();
    if ((int)threadIdx.x < F) {
        double s = 0.0;
        for (int t = threadIdx.x; t < kVecThreads; t += F) s += red[t];
        part[(int64_t)blockIdx.x * F + threadIdx.x] = s;
    }
}

template <class T>
__global__ void k_sqnorm(const T *v, int64_t n, int F, double *part) {
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double t = v[i];
        acc += t * t;
    }
    block_partial(acc, F, part);
}

// Per-slice max of non-negative floats across the grid (their bits order
// like the values); the grid stride is a multiple of F, so each thread's
// values all belong to one slice.
__device__ __forceinline__ void block_max(float m, int F, uint32_t *amax) {
    __shared__ float red[kVecThreads];
    red[threadIdx.x] = m;
    __syncthreads();
    if ((int)threadIdx.x < F) {
        for (int t = threadIdx.x + F; t < kVecThreads; t += F) m = fmaxf(m, red[t]);
        atomicMax(&amax[threadIdx.x], __float_as_uint(m));
    }
}

// r -= alpha q, with block partials of |r|^2 (sinogram) and, when amax is
// given, the per-slice max |r| (the next product's operand scale)
template <class T>
__global__ void k_axpy_res(T *r, const T *q, int64_t n, int F, const double *alpha, double *part, uint32_t *amax) {
    double acc = 0.0;
    float m = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T a = (T)alpha[i & (F - 1)];
        const T t = fma(-a, q[i], r[i]);
        r[i] = t;
        acc += (double)t * (double)t;
        m = fmaxf(m, fabsf((float)t));
    }
    block_partial(acc, F, part);
    if (amax) block_max(m, F, amax);
}

// x += alpha p, then p = s + beta p, in one pass (the iterate's update is
// deferred to here from the step where alpha is found: p is unchanged in
// between); when amax is given, also the per-slice max |p| of the new p
template <class T>
__global__ void k_update_xp(T *x, T *p, const T *s, int64_t n, int F, const double *alpha, const double *beta,
                            uint32_t *amax) {
    float m = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T a = (T)alpha[i & (F - 1)], bt = (T)beta[i & (F - 1)];
        const T pv = p[i];
        if (a != (T)0) x[i] = fma(a, pv, x[i]);  // a stopped slice keeps its iterate, also if p is not finite
        const T t = fma(bt, pv, s[i]);
        p[i] = t;
        m = fmaxf(m, fabsf((float)t));
    }
    if (amax) block_max(m, F, amax);
}

// Per-slice max |v| of an internal-layout group vector (the solver's first
// operands; later ones get their max from the kernel that produces them).
__global__ void k_absmax_int(const float *v, int64_t n, int F, uint32_t *amax) {
    float m = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(v[i]));
    block_max(m, F, amax);
}

// Clear n words (a kernel rather than a memset node, so the solver can be
// captured into a graph).
__global__ void k_zero_words(uint32_t *v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[i] = 0u;
}

__device__ __forceinline__ uint32_t to16(float v, int fmt) {
    if (fmt == XCT_F16) return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)v);
    uint32_t u = __builtin_bit_cast(uint32_t, v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}

// o16 = round16(v * inv[slice])
__global__ void k_cast16(const float *v, int64_t n, int F, const float *inv, uint16_t *o16, int fmt) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        o16[i] = (uint16_t)to16(v[i] * inv[i & (F - 1)], fmt);
}

// ---- per-slice scalar updates --------------------------------------------------

// sum[b] = sum over blocks of part[m][blk][f], b = m*F + f: one workgroup per
// slice, thread t adding blocks t, t + 256, ... in order, then a fixed
// pairwise tree in LDS, so the result is the same on every run.
constexpr int kReduceThreads = 256;
__global__ void __launch_bounds__(kReduceThreads) k_reduce(const double *part, int64_t stride, int nblk, int F,
                                                           double *sum) {
    __shared__ double red[kReduceThreads];
    const int b = blockIdx.x, t = threadIdx.x;
    const int m = b / F, f = b % F;
    const double *p = part + (int64_t)m * stride * F;
    double s = 0.0;
    for (int k = t; k < nblk; k += kReduceThreads) s += p[(int64_t)k * F + f];
    red[t] = s;
    __syncthreads();
    for (int h = kReduceThreads / 2; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    if (t == 0) sum[b] = red[0];
}

enum { kSetGamma = 0, kSetAlpha = 1, kSetBeta = 2, kSetYY = 3, kSetResid = 4 };

__global__ void k_scalars(int mode, int Bp, const double *sum, double *gamma, double *delta, double *alpha,
                          double *beta, double *yy, int32_t *stopped, double *resid_row) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= Bp) return;
    const double v = sum[b];
    switch (mode) {
        case kSetYY:
            // a slice whose sinogram holds a non-finite value is not solved
            // (status 2, x stays 0, residuals NaN); the others are unaffected
            yy[b] = v;
            stopped[b] = isfinite(v) ? 0 : 2;
            resid_row[b] = !isfinite(v) ? v - v : (v > 0.0 ? 1.0 : 0.0);
            break;
        case kSetGamma:
            gamma[b] = v;
            break;
        case kSetAlpha: {
            delta[b] = v;
            const double g = gamma[b];
            if (stopped[b]) {
                alpha[b] = 0.0;  // keeps its status (1 or 2)
            } else if (g == 0.0 || v == 0.0) {
                stopped[b] = 1;
                alpha[b] = 0.0;
            } else {
                alpha[b] = g / v;
            }
            break;
        }
        case kSetResid:
            resid_row[b] = stopped[b] == 2 ? yy[b] - yy[b] : (yy[b] > 0.0 ? sqrt(v / yy[b]) : 0.0);
            break;
        case kSetBeta:
            if (stopped[b]) {
                beta[b] = 0.0;
            } else {
                beta[b] = v / gamma[b];
                gamma[b] = v;
            }
            break;
    }
}

// ---- orchestration -----------------------------------------------------------

template <class T>
struct Cgls {
    const xct_matrix *m;
    CglsWs<T> w;
    hipStream_t st;
    int grid_v, grid_s;

    int vec_grid(int64_t n) const {
        return (int)std::max<int64_t>(1, std::min<int64_t>(kVecBlocks, (n + kVecThreads - 1) / kVecThreads));
    }

    int scalars(int mode, double *resid_row) {
        hipLaunchKernelGGL(k_scalars, dim3((w.Bp + 255) / 256), dim3(256), 0, st, mode, w.Bp, (const double *)w.sum,
                           w.gamma, w.delta, w.alpha, w.beta, w.yy, w.stopped, resid_row);
        XCT_HIP_TRY(hipGetLastError());
        return XCT_OK;
    }

    int reduce(const double *part, int64_t stride, int nblk) {
        hipLaunchKernelGGL(k_reduce, dim3(w.Bp), dim3(kReduceThreads), 0, st, part, stride, nblk, w.F, w.sum);
        XCT_HIP_TRY(hipGetLastError());
        return XCT_OK;
    }

    // Per-slice max |v| of every group of an operand vector into amax (the
    // solver's first operands; the updates produce it for later ones).
    int absmax(const float *v, int64_t n) {
        for (int g = 0; g < w.n_mb; ++g)
            hipLaunchKernelGGL(k_absmax_int, dim3(vec_grid(n)), dim3(kVecThreads), 0, st, v + (int64_t)g * n, n, w.F,
                               w.amax + (int64_t)g * w.F);
        XCT_HIP_TRY(hipGetLastError());
        return XCT_OK;
    }

    // One product (dir 0: q = A p, dir 1: s = A^T r) for every group, with
    // the per-block squared-output partials, then their per-slice sums.  With
    // a 16-bit matrix, amax holds the operand's per-slice max |v| (cleared
    // here once read).
    int product(int dir) {
        const OpPlan &op = dir ? m->AT : m->A;
        const int64_t nin = dir ? w.ns : w.nv, nout = dir ? w.nv : w.ns;
        T *in = dir ? w.r : w.p;
        T *out = dir ? w.s : w.q;
        for (int g = 0; g < w.n_mb; ++g) {
            T *gin = in + (int64_t)g * nin;
            const void *opnd = gin;
            const float *scale = nullptr;
            if (m->vdt == XCT_F16 || m->vdt == XCT_BF16) {
                const int gg = vec_grid(nin);
                int rc0 = launch_pow2_scale(w.amax + (int64_t)g * w.F, w.F, w.scale, w.inv, st);
                if (rc0) return rc0;
                hipLaunchKernelGGL(k_cast16, dim3(gg), dim3(kVecThreads), 0, st, (const float *)(const void *)gin, nin, w.F,
                                   (const float *)w.inv, (uint16_t *)w.op16, (int)m->vdt);
                XCT_HIP_TRY(hipGetLastError());
                opnd = w.op16;
                scale = w.scale;
            }
            SpmmLaunch L{&op, opnd, out + (int64_t)g * nout, scale, w.sqp + (int64_t)g * w.sq_stride * w.F, w.F,
                         m->vdt, m->remap};
            int rc = launch_spmm(L, st);
            if (rc) return rc;
        }
        return reduce(w.sqp, w.sq_stride, op.n_blocks);
    }
};

template <class T>
static int run_cgls(const xct_matrix *m, const void *y, xct_dtype y_dtype, float *x, int batch, int iters,
                    void *workspace, double *resid, int32_t *status, hipStream_t st) {
    constexpr bool kF64 = sizeof(T) == 8;
    Cgls<T> c;
    c.m = m;
    c.st = st;
    cgls_layout<T>(m, batch, iters, (char *)workspace, &c.w);
    CglsWs<T> &w = c.w;
    const int gv = c.vec_grid(w.nv), gs = c.vec_grid(w.ns);
    int rc;
    const bool narrow = m->vdt == XCT_F16 || m->vdt == XCT_BF16;  // 16-bit operands: max of each product's input
    uint32_t *amax = narrow ? w.amax : nullptr;
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, st, w.amax, (int64_t)w.Bp);
    // r = y ; x = 0 ; yy = |y|^2
    for (int g = 0; g < w.n_mb; ++g) {
        rc = launch_to_internal(m->sino, y, y_dtype, batch, g * w.F, w.F, w.r + (int64_t)g * w.ns,
                                kF64 ? XCT_F64 : XCT_F32, nullptr, st);
        if (rc) return rc;
    }
    hipLaunchKernelGGL(k_zero_words, dim3(gv), dim3(kVecThreads), 0, st, (uint32_t *)w.x,
                       w.nv * w.n_mb * (int64_t)(sizeof(T) / 4));
    XCT_HIP_TRY(hipGetLastError());
    for (int g = 0; g < w.n_mb; ++g) {
        hipLaunchKernelGGL(k_sqnorm<T>, dim3(gs), dim3(kVecThreads), 0, st, (const T *)(w.r + (int64_t)g * w.ns), w.ns,
                           w.F, w.dotp + (int64_t)g * kVecBlocks * w.F);
    }
    XCT_HIP_TRY(hipGetLastError());
    if ((rc = c.reduce(w.dotp, kVecBlocks, gs))) return rc;
    if ((rc = c.scalars(kSetYY, w.resid))) return rc;
    // s = A^T r ; gamma = |s|^2 ; p = s
    if (narrow && (rc = c.absmax((const float *)(const void *)w.r, w.ns))) return rc;
    if ((rc = c.product(1))) return rc;
    if ((rc = c.scalars(kSetGamma, nullptr))) return rc;
    XCT_HIP_TRY(hipMemcpyAsync(w.p, w.s, sizeof(T) * w.nv * w.n_mb, hipMemcpyDeviceToDevice, st));
    if (narrow && (rc = c.absmax((const float *)(const void *)w.p, w.nv))) return rc;
    for (int k = 0; k < iters; ++k) {
        if ((rc = c.product(0))) return rc;  // q = A p, delta
        if ((rc = c.scalars(kSetAlpha, nullptr))) return rc;
        for (int g = 0; g < w.n_mb; ++g)  // r -= alpha q (and |r|^2, max |r|)
            hipLaunchKernelGGL(k_axpy_res<T>, dim3(gs), dim3(kVecThreads), 0, st, w.r + (int64_t)g * w.ns,
                               (const T *)(w.q + (int64_t)g * w.ns), w.ns, w.F, (const double *)(w.alpha + g * w.F),
                               w.dotp + (int64_t)g * kVecBlocks * w.F, amax ? amax + (int64_t)g * w.F : nullptr);
        XCT_HIP_TRY(hipGetLastError());
        if ((rc = c.reduce(w.dotp, kVecBlocks, gs))) return rc;
        if ((rc = c.scalars(kSetResid, w.resid + (int64_t)(k + 1) * w.Bp))) return rc;
        if ((rc = c.product(1))) return rc;  // s = A^T r, gamma'
        if ((rc = c.scalars(kSetBeta, nullptr))) return rc;
        for (int g = 0; g < w.n_mb; ++g)  // x += alpha p ; p = s + beta p (and max |p|)
            hipLaunchKernelGGL(k_update_xp<T>, dim3(gv), dim3(kVecThreads), 0, st, w.x + (int64_t)g * w.nv,
                               w.p + (int64_t)g * w.nv, (const T *)(w.s + (int64_t)g * w.nv), w.nv, w.F,
                               (const double *)(w.alpha + g * w.F), (const double *)(w.beta + g * w.F),
                               amax ? amax + (int64_t)g * w.F : nullptr);
        XCT_HIP_TRY(hipGetLastError());
    }
    for (int g = 0; g < w.n_mb; ++g) {
        if constexpr (kF64)
            rc = launch_from_internal64(m->vol, w.x + (int64_t)g * w.nv, batch, g * w.F, w.F, x, XCT_F32, st);
        else
            rc = launch_from_internal(m->vol, w.x + (int64_t)g * w.nv, batch, g * w.F, w.F, x, XCT_F32, st);
        if (rc) return rc;
    }
    // the residual rows (padded batch Bp on the device) and the status words
    // straight into the caller's arrays
    if (resid)
        XCT_HIP_TRY(hipMemcpy2DAsync(resid, sizeof(double) * batch, w.resid, sizeof(double) * w.Bp,
                                     sizeof(double) * batch, iters + 1, hipMemcpyDeviceToHost, st));
    if (status)
        XCT_HIP_TRY(hipMemcpyAsync(status, w.stopped, sizeof(int32_t) * batch, hipMemcpyDeviceToHost, st));
    if (resid || status) XCT_HIP_TRY(hipStreamSynchronize(st));
    return XCT_OK;
}

}  // namespace xct

using namespace xct;

extern "C" size_t xct_cgls_workspace_bytes(const xct_matrix *m, int batch, int iters) {
    if (!m || batch < 1 || iters < 0) return 0;
    return m->vdt == XCT_F64 ? cgls_layout<double>(m, batch, iters, nullptr, nullptr)
                             : cgls_layout<float>(m, batch, iters, nullptr, nullptr);
}

extern "C" int xct_cgls(const xct_matrix *m, const void *y, xct_dtype y_dtype, float *x, int batch, int iters,
                        void *workspace, double *resid, int32_t *status, void *stream) {
    if (!m || !y || !x || !workspace) return fail(XCT_ERR_INVALID, "NULL argument");
    if (batch < 1 || iters < 0) return fail(XCT_ERR_INVALID, "batch must be >= 1 and iters >= 0");
    if (!valid_dtype(y_dtype)) return fail(XCT_ERR_INVALID, "bad y dtype");
    if (((uintptr_t)workspace & 255) != 0) return fail(XCT_ERR_INVALID, "workspace must be 256-byte aligned");
    hipStream_t st = (hipStream_t)stream;
    if (m->vdt == XCT_F64) return run_cgls<double>(m, y, y_dtype, x, batch, iters, workspace, resid, status, st);
    return run_cgls<float>(m, y, y_dtype, x, batch, iters, workspace, resid, status, st);
}
