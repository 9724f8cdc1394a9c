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
    double *gamma = nullptr, *delta = nullptr, *alpha = nullptr, *beta = nullptr, *yy = nullptr;
    int32_t *stopped = nullptr;
    double *resid = nullptr;  // [iters+1][Bp]
    uint32_t *amax = nullptr;   // per-slice max |r| of the next backprojection's operand
    uint32_t *amaxp = nullptr;  // per-slice max |p| of the next projection's operand
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
    c.stopped = (int32_t *)take(sizeof(int32_t) * c.Bp);
    c.resid = (double *)take(sizeof(double) * (size_t)(iters + 1) * c.Bp);
    c.amax = (uint32_t *)take(sizeof(uint32_t) * (size_t)c.Bp);
    c.amaxp = (uint32_t *)take(sizeof(uint32_t) * (size_t)c.Bp);
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

// The elementwise kernels read and write V consecutive elements per access
// (16 bytes: 4 FP32 or 2 FP64 values; V = 1 when F is not a multiple of
// that).  The grid stride (kVecBlocks * kVecThreads * V elements) is a
// multiple of F, so a thread's elements always belong to the same V slices
// f0 .. f0 + V - 1, whose scalars it loads once.
template <class T> struct Vec16;
template <> struct Vec16<float> { typedef float t __attribute__((ext_vector_type(4))); static constexpr int V = 4; };
template <> struct Vec16<double> { typedef double t __attribute__((ext_vector_type(2))); static constexpr int V = 2; };
template <class T, int V> struct VecOf { typedef typename Vec16<T>::t t; };
template <class T> struct VecOf<T, 1> { typedef T t; };
template <int V, class VT, class T>
__device__ __forceinline__ T lane_of(const VT &v, int k) {
    if constexpr (V == 1) return v; else return v[k];
}
template <int V, class VT, class T>
__device__ __forceinline__ void set_lane(VT &v, int k, T x) {
    if constexpr (V == 1) v = x; else v[k] = x;
}

// Block partial sums per slice of the V running sums of each thread into
// part[blockIdx.x][F] (element t*V + k of a block's sums belongs to slice
// (t*V + k) mod F), in a fixed order.
template <int V>
__device__ __forceinline__ void block_partial_v(const double (&acc)[V], int F, double *part) {
    __shared__ double red[kVecThreads * V];
#pragma unroll
    for (int k = 0; k < V; ++k) red[threadIdx.x * V + k] = acc[k];
    __syncthreads();
    if ((int)threadIdx.x < F) {
        double s = 0.0;
        for (int t = threadIdx.x; t < kVecThreads * V; t += F) s += red[t];
        part[(int64_t)blockIdx.x * F + threadIdx.x] = s;
    }
}

// Per-slice max of the V running maxima of each thread (non-negative
// floats: their bits order like the values) into amax.
template <int V>
__device__ __forceinline__ void block_max_v(const float (&m)[V], int F, uint32_t *amax) {
    __shared__ float red[kVecThreads * V];
#pragma unroll
    for (int k = 0; k < V; ++k) red[threadIdx.x * V + k] = m[k];
    __syncthreads();
    if ((int)threadIdx.x < F) {
        float mx = 0.f;
        for (int t = threadIdx.x; t < kVecThreads * V; t += F) mx = fmaxf(mx, red[t]);
        atomicMax(&amax[threadIdx.x], __float_as_uint(mx));
    }
}

// r -= alpha q, with block partials of |r|^2 (sinogram) and, when amax is
// given, the per-slice max |r| (the next product's operand scale).  n: a
// multiple of V.
template <class T, int V>
__global__ void __launch_bounds__(kVecThreads) k_axpy_res(T *r, const T *q, int64_t n, int F, const double *alpha,
                                                          double *part, uint32_t *amax) {
    typedef typename VecOf<T, V>::t VT;
    const int64_t nv = n / V, stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int f0 = (int)((i * V) & (F - 1));
    T a[V];
    double acc[V];
    float m[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
        a[k] = (T)alpha[f0 + k];
        acc[k] = 0.0;
        m[k] = 0.f;
    }
    for (; i < nv; i += stride) {
        VT rv = ((const VT *)r)[i];
        const VT qv = ((const VT *)q)[i];
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const T t = fma(-a[k], lane_of<V, VT, T>(qv, k), lane_of<V, VT, T>(rv, k));
            set_lane<V>(rv, k, t);
            acc[k] += (double)t * (double)t;
            m[k] = fmaxf(m[k], fabsf((float)t));
        }
        ((VT *)r)[i] = rv;
    }
    block_partial_v<V>(acc, F, part);
    if (amax) block_max_v<V>(m, F, amax);
}

// x += alpha p, then p = s + beta p, in one pass (the iterate's update is
// deferred to here from the step where alpha is found: p is unchanged in
// between); when amax is given, also the per-slice max |p| of the new p.
// A stopped slice (alpha = 0) keeps its iterate, also if p is not finite.
template <class T, int V>
__global__ void __launch_bounds__(kVecThreads) k_update_xp(T *x, T *p, const T *s, int64_t n, int F,
                                                           const double *alpha, const double *beta, uint32_t *amax) {
    typedef typename VecOf<T, V>::t VT;
    const int64_t nv = n / V, stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int f0 = (int)((i * V) & (F - 1));
    T a[V], bt[V];
    float m[V];
#pragma unroll
    for (int k = 0; k < V; ++k) {
        a[k] = (T)alpha[f0 + k];
        bt[k] = (T)beta[f0 + k];
        m[k] = 0.f;
    }
    for (; i < nv; i += stride) {
        const VT pv = ((const VT *)p)[i], sv = ((const VT *)s)[i];
        VT xv = ((const VT *)x)[i], np;
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const T pk = lane_of<V, VT, T>(pv, k);
            if (a[k] != (T)0) set_lane<V>(xv, k, fma(a[k], pk, lane_of<V, VT, T>(xv, k)));
            const T t = fma(bt[k], pk, lane_of<V, VT, T>(sv, k));
            set_lane<V>(np, k, t);
            m[k] = fmaxf(m[k], fabsf((float)t));
        }
        ((VT *)x)[i] = xv;
        ((VT *)p)[i] = np;
    }
    if (amax) block_max_v<V>(m, F, amax);
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

// o16 = round16(v / m[slice]) with m = pow2_at_least(max |v| of the slice)
// taken from amax (complete: written by the kernel that produced v); block 0
// also stores m for the product that scales its sums back, and clears
// amax_next, the maxima that the product after this one accumulates (the
// solver alternates two arrays, so no block clears what another still
// reads).  n: a multiple of V.
template <int V>
__global__ void __launch_bounds__(kVecThreads) k_cast16(const float *v, int64_t n, int F, const uint32_t *amax,
                                                        float *scale, uint32_t *amax_next, uint16_t *o16, int fmt) {
    typedef typename VecOf<float, V>::t VT;
    const int64_t nv = n / V, stride = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int f0 = (int)((i * V) & (F - 1));
    if (blockIdx.x == 0 && (int)threadIdx.x < F) {
        scale[threadIdx.x] = pow2_at_least(__uint_as_float(amax[threadIdx.x]));
        amax_next[threadIdx.x] = 0u;
    }
    float inv[V];
#pragma unroll
    for (int k = 0; k < V; ++k) inv[k] = 1.f / pow2_at_least(__uint_as_float(amax[f0 + k]));  // exact
    for (; i < nv; i += stride) {
        const VT x = ((const VT *)v)[i];
        if constexpr (V == 4) {
            const uint32_t h0 = to16(x[0] * inv[0], fmt) | (to16(x[1] * inv[1], fmt) << 16);
            const uint32_t h1 = to16(x[2] * inv[2], fmt) | (to16(x[3] * inv[3], fmt) << 16);
            ((uint2 *)o16)[i] = make_uint2(h0, h1);
        } else {
            o16[i] = (uint16_t)to16(x * inv[0], fmt);
        }
    }
}

// ---- per-slice scalar updates --------------------------------------------------

constexpr int kReduceThreads = 256;

enum { kSetGamma = 0, kSetAlpha = 1, kSetBeta = 2, kSetYY = 3, kSetResid = 4 };

// The per-slice scalar update of `mode` for slice b from its new sum v.
__device__ __forceinline__ void scalar_update(int mode, int b, double v, double *gamma, double *delta, double *alpha,
                                              double *beta, double *yy, int32_t *stopped, double *resid_row) {
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

// The sum over blocks of part[m][blk][f] for slice b = m*F + f (one
// workgroup per slice: thread t adds blocks t, t + 256, ... in order, then a
// fixed pairwise tree in LDS, so the result is the same on every run), then
// the slice's scalar update.
__global__ void __launch_bounds__(kReduceThreads) k_reduce_scalars(const double *part, int64_t stride, int nblk, int F,
                                                                   int mode, double *gamma, double *delta,
                                                                   double *alpha, double *beta, double *yy,
                                                                   int32_t *stopped, double *resid_row) {
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
    if (t == 0) scalar_update(mode, b, red[0], gamma, delta, alpha, beta, yy, stopped, resid_row);
}

// ---- orchestration -----------------------------------------------------------

template <class T>
struct Cgls {
    const xct_matrix *m;
    CglsWs<T> w;
    hipStream_t st;

    int vec_grid(int64_t n) const {
        return (int)std::max<int64_t>(1, std::min<int64_t>(kVecBlocks, (n + kVecThreads - 1) / kVecThreads));
    }
    // elements per access of the elementwise kernels for this group size
    int vec_width() const { return w.F % Vec16<T>::V == 0 ? Vec16<T>::V : 1; }

    // Per-slice sums of the partials, then the scalar update `mode`.
    int reduce_scalars(const double *part, int64_t stride, int nblk, int mode, double *resid_row) {
        hipLaunchKernelGGL(k_reduce_scalars, dim3(w.Bp), dim3(kReduceThreads), 0, st, part, stride, nblk, w.F, mode,
                           w.gamma, w.delta, w.alpha, w.beta, w.yy, w.stopped, resid_row);
        XCT_HIP_TRY(hipGetLastError());
        return XCT_OK;
    }

    // Per-slice max |v| of every group of an operand vector into amax (the
    // solver's first operands; the updates produce it for later ones).
    int absmax(const float *v, int64_t n, uint32_t *amax) {
        for (int g = 0; g < w.n_mb; ++g)
            hipLaunchKernelGGL(k_absmax_int, dim3(vec_grid(n)), dim3(kVecThreads), 0, st, v + (int64_t)g * n, n, w.F,
                               amax + (int64_t)g * w.F);
        XCT_HIP_TRY(hipGetLastError());
        return XCT_OK;
    }

    int axpy_res(uint32_t *amax) {  // r -= alpha q (and |r|^2, max |r|)
        const int gs = vec_grid(w.ns);
        for (int g = 0; g < w.n_mb; ++g) {
            T *r = w.r + (int64_t)g * w.ns;
            const T *q = w.q + (int64_t)g * w.ns;
            const double *al = w.alpha + g * w.F;
            double *part = w.dotp + (int64_t)g * kVecBlocks * w.F;
            uint32_t *am = amax ? amax + (int64_t)g * w.F : nullptr;
            if (vec_width() > 1)
                hipLaunchKernelGGL((k_axpy_res<T, Vec16<T>::V>), dim3(gs), dim3(kVecThreads), 0, st, r, q, w.ns, w.F, al,
                                   part, am);
            else
                hipLaunchKernelGGL((k_axpy_res<T, 1>), dim3(gs), dim3(kVecThreads), 0, st, r, q, w.ns, w.F, al, part, am);
        }
        XCT_HIP_TRY(hipGetLastError());
        return XCT_OK;
    }

    int update_xp(uint32_t *amax) {  // x += alpha p ; p = s + beta p (and max |p|)
        const int gv = vec_grid(w.nv);
        for (int g = 0; g < w.n_mb; ++g) {
            T *x = w.x + (int64_t)g * w.nv, *p = w.p + (int64_t)g * w.nv;
            const T *s = w.s + (int64_t)g * w.nv;
            const double *al = w.alpha + g * w.F, *be = w.beta + g * w.F;
            uint32_t *am = amax ? amax + (int64_t)g * w.F : nullptr;
            if (vec_width() > 1)
                hipLaunchKernelGGL((k_update_xp<T, Vec16<T>::V>), dim3(gv), dim3(kVecThreads), 0, st, x, p, s, w.nv, w.F,
                                   al, be, am);
            else
                hipLaunchKernelGGL((k_update_xp<T, 1>), dim3(gv), dim3(kVecThreads), 0, st, x, p, s, w.nv, w.F, al, be,
                                   am);
        }
        XCT_HIP_TRY(hipGetLastError());
        return XCT_OK;
    }

    // One product (dir 0: q = A p, dir 1: s = A^T r) for every group, with
    // the per-block squared-output partials, then their per-slice sums and
    // the scalar update `mode`.  With a 16-bit matrix, amax holds the
    // operand's per-slice max |v| and amax_next (the other array) is
    // cleared for the update that follows the product.
    int product(int dir, int mode, uint32_t *amax, uint32_t *amax_next) {
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
                const float *vin = (const float *)(const void *)gin;
                const uint32_t *am = amax + (int64_t)g * w.F;
                uint32_t *amn = amax_next + (int64_t)g * w.F;
                if (vec_width() > 1)
                    hipLaunchKernelGGL(k_cast16<4>, dim3(gg), dim3(kVecThreads), 0, st, vin, nin, w.F, am, w.scale, amn,
                                       (uint16_t *)w.op16, (int)m->vdt);
                else
                    hipLaunchKernelGGL(k_cast16<1>, dim3(gg), dim3(kVecThreads), 0, st, vin, nin, w.F, am, w.scale, amn,
                                       (uint16_t *)w.op16, (int)m->vdt);
                XCT_HIP_TRY(hipGetLastError());
                opnd = w.op16;
                scale = w.scale;
            }
            SpmmLaunch L{&op, opnd, out + (int64_t)g * nout, scale, w.sqp + (int64_t)g * w.sq_stride * w.F, w.F,
                         m->vdt, m->remap};
            int rc = launch_spmm(L, st);
            if (rc) return rc;
        }
        return reduce_scalars(w.sqp, w.sq_stride, op.n_blocks, mode, nullptr);
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
    // 16-bit operands: the per-slice max of each product's input, r's in
    // amax and p's in amaxp (each product's cast clears the other array)
    const bool narrow = m->vdt == XCT_F16 || m->vdt == XCT_BF16;
    uint32_t *amr = narrow ? w.amax : nullptr, *amp = narrow ? w.amaxp : nullptr;
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, st, w.amax, (int64_t)w.Bp);
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(256), 0, st, w.amaxp, (int64_t)w.Bp);
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
    if ((rc = c.reduce_scalars(w.dotp, kVecBlocks, gs, kSetYY, w.resid))) return rc;
    // s = A^T r ; gamma = |s|^2 ; p = s
    if (narrow && (rc = c.absmax((const float *)(const void *)w.r, w.ns, amr))) return rc;
    if ((rc = c.product(1, kSetGamma, amr, amp))) return rc;
    XCT_HIP_TRY(hipMemcpyAsync(w.p, w.s, sizeof(T) * w.nv * w.n_mb, hipMemcpyDeviceToDevice, st));
    if (narrow && (rc = c.absmax((const float *)(const void *)w.p, w.nv, amp))) return rc;
    for (int k = 0; k < iters; ++k) {
        if ((rc = c.product(0, kSetAlpha, amp, amr))) return rc;  // q = A p, delta, alpha
        if ((rc = c.axpy_res(amr))) return rc;                     // r -= alpha q, |r|^2, max |r|
        if ((rc = c.reduce_scalars(w.dotp, kVecBlocks, gs, kSetResid, w.resid + (int64_t)(k + 1) * w.Bp))) return rc;
        if ((rc = c.product(1, kSetBeta, amr, amp))) return rc;  // s = A^T r, gamma', beta
        if ((rc = c.update_xp(amp))) return rc;                  // x += alpha p ; p = s + beta p, max |p|
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
