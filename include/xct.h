/*
 * xct.h -- C ABI of the MI355X (gfx950) library for parallel-beam XCT:
 * system-matrix build, forward projection, backprojection and CGLS.
 *
 * The operations follow Hidayetoglu et al., "Petascale XCT: 3D Image
 * Reconstruction with Hierarchical Communications on Multi-GPU Nodes"
 * (SC20):
 *   - the least-squares problem of Eq. (1) with R = 0 and no constraint;
 *   - the parallel-beam Siddon system matrix A (Sec. II-A), memoised once
 *     and shared by every slice of a batch (Sec. II-B, Sec. III-A.4);
 *   - projection y = A x and backprojection x = A^T y as sparse
 *     matrix-times-many-vectors products with staged input buffers, fused
 *     slices and register accumulators (Sec. III-B, Listing 1);
 *   - storage of matrix values and kernel operands in 16 bits with FP32
 *     arithmetic and adaptive max-norm scaling (Sec. III-C);
 *   - CG on the normal equations (CGLS) from x = 0 for a fixed iteration
 *     count: k iterations use k projections and k+1 backprojections
 *     (Sec. IV-F; note under Table IV).
 *
 * Geometry (the paper fixes none of it; these are this library's
 * conventions):
 *   - a slice is n x n unit voxels centred on the rotation axis; voxel
 *     (i, j) covers [j - n/2, j - n/2 + 1] x [i - n/2, i - n/2 + 1];
 *     volumes are stored [batch][n][n] (row i, column j, j fastest);
 *   - angle k in [0, n_angles) is theta_k = k*pi/n_angles; channel c in
 *     [0, n_channels) is the line {p : p.(cos theta_k, sin theta_k) =
 *     c - (n_channels-1)/2}; sinograms are stored
 *     [batch][n_angles][n_channels] (channel fastest);
 *   - A[(k, c), (i, j)] is the length of line (k, c) inside voxel (i, j);
 *     a line lying on a voxel edge gives half its length to each of the
 *     two voxels; lengths below 1e-9 are dropped.
 *
 * Conventions for every call:
 *   - Pointers named x, y, workspace are DEVICE pointers owned by the
 *     caller.  Host pointers are marked "host".
 *   - `stream` is a hipStream_t (NULL = the default stream).  All device
 *     work is enqueued on it; no call synchronises the host except
 *     xct_build_matrix, xct_matrix_to_coo and xct_cgls (only when it is
 *     given host result arrays).
 *   - Functions return XCT_OK or a negative status and never abort; the
 *     message of the last failure on the calling thread is returned by
 *     xct_last_error().  Kernel faults surface at the next synchronisation
 *     as XCT_ERR_HIP.
 *   - A built matrix is immutable: concurrent calls that share one matrix
 *     but use separate outputs and workspaces may run on different streams.
 */
#ifndef XCT_H
#define XCT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xct_matrix xct_matrix; /* opaque; owns the device copies of A and A^T */

typedef enum { XCT_F32 = 0, XCT_F16 = 1, XCT_BF16 = 2, XCT_F64 = 3 } xct_dtype;

enum {
    XCT_OK = 0,
    XCT_ERR_INVALID = -1,     /* bad argument */
    XCT_ERR_OOM = -2,         /* device or host allocation failed */
    XCT_ERR_HIP = -3,         /* a HIP runtime call failed */
    XCT_ERR_UNSUPPORTED = -4, /* valid request outside what this build supports */
    XCT_ERR_INTERNAL = -5     /* an internal consistency check failed */
};

/* Build options; zero in any field selects the default. */
typedef struct {
    int tile_waves; /* row tiles (64 rows each) per workgroup: 1..16 (one wavefront each) or 32
                       (16 wavefronts holding two row tiles each); default 16 */
    int fuse;       /* largest number of slices fused per matrix pass (F); 1, 2, 4, 8, 16 or 32
                       (32: F16/BF16 matrices with tile_waves <= 16 only; FP64 matrices at most 8);
                       default 16 (8 for FP64) */
    int lds_bytes;  /* LDS bytes per workgroup at F = fuse: one stage of staged input
                       (T = lds_bytes / (64 * F * element size) input tiles, at most 1024);
                       default: all of the device's LDS per workgroup (160 KiB on gfx950) */
    int xcd_remap;  /* how workgroups map to the 8 XCDs (each with its own L2): runs of n
                       consecutive workgroups of the Hilbert order dealt to the XCDs in turn,
                       n >= 2 as given, 4 for 0 (default); 1 one contiguous run per XCD;
                       -1 plain order */
    int stage_order; /* order in which a workgroup stages its input tiles:
                        0 (default) sweep: for A, by distance along the workgroup's mean ray
                          direction; for A^T, angle-major;
                        1 Hilbert: along the pseudo-Hilbert curve of the input tiles */
    int lane_order;  /* tuning: assignment of a tile's 64 rows to the lanes of a wavefront;
                        0 default (row-major), 1 transposed */
    int slab_order;  /* order of a lane's entries within a (stage, wavefront) slab:
                        0 (default) scheduled so that the lanes served together by one
                          16-byte LDS read hit distinct bank groups (rows of 32 or 64 B);
                        1 ray/voxel tracing order */
    int arith;       /* arithmetic of the products: 0 (default) FP32 accumulation; 1 FP16
                        accumulation with packed FP16 FMAs (FP16 matrices only; the paper's
                        "half precision" variant, for measurement: sums keep ~11 bits, so
                        results deviate by ~1e-2 relative; a single fused slice keeps FP32) */
    int debug_poison_lds; /* debug: 1 fills a workgroup's LDS stage buffer with NaN before each
                             stage is copied in, so that an entry reading a slot its stage did
                             not stage turns its sums into NaN (tests compare such a build with
                             a plain one bit for bit); 0 (default) off */
} xct_build_opts;

/* Statistics of one operator (A or A^T). */
typedef struct {
    int64_t nnz;          /* structural nonzeros: chord lengths above 1e-9 that do not round
                             to zero in the stored format (FP16 drops lengths <= 2^-25) */
    int64_t padded;       /* stored entries including ELL padding */
    int64_t bytes;        /* device bytes of the operator (entries + maps) */
    int64_t stages;       /* total staging rounds over all workgroups */
    int64_t staged_slots; /* input slots loaded over all stages (64 per tile) */
    int32_t blocks;       /* workgroups per pass */
    int32_t tiles_per_stage;
    int64_t slabs;          /* (stage, wavefront) slabs */
    int64_t balanced_slabs; /* slabs scheduled against LDS bank conflicts (empty ones included);
                               equals slabs unless scheduling is off or a slab is too long for it */
} xct_op_stats;

typedef struct {
    int n, n_angles, n_channels;
    xct_dtype value_dtype;
    int fuse;
    xct_op_stats A;  /* projection operator */
    xct_op_stats AT; /* backprojection operator */
    double build_seconds;
} xct_matrix_info_t;

/*
 * Build A (rays x voxels) and A^T (voxels x rays) on the GPU
 * (Sec. II-A, II-B; memoisation as in Sec. II-B "avoids repetitive
 * computation of A").
 *   n           slice edge in voxels, 1..8192
 *   n_angles    angles over [0, pi), >= 1
 *   n_channels  detector channels, >= 1
 *   value_dtype storage of matrix values and of the staged kernel operand:
 *               XCT_F32 (16-bit stage-local index + FP32 value, 6 B per
 *               entry), XCT_F16 / XCT_BF16 (index and value packed in
 *               4 B, Sec. III-C "data packing"), or XCT_F64 (index + FP64
 *               value, 10 B per entry, FP64 operand and sums: the
 *               double-precision variant of Sec. IV; at most 8 fused
 *               slices); lengths are computed in
 *               FP64 and rounded to nearest-even once.
 *   opts        nullable; see xct_build_opts
 *   stream      stream for the build kernels; the call returns after they finish
 *   out         receives the handle; release with xct_free_matrix.
 * Errors: XCT_ERR_INVALID (sizes), XCT_ERR_OOM, XCT_ERR_UNSUPPORTED (a
 * grid too large for the builder's LDS bitmaps), XCT_ERR_HIP.
 */
int xct_build_matrix(int n, int n_angles, int n_channels, xct_dtype value_dtype,
                     const xct_build_opts *opts, void *stream, xct_matrix **out);

/* Release a handle (NULL is ignored).  The caller must make sure no work
 * that uses it is still queued. */
void xct_free_matrix(xct_matrix *A);

/* Fill *info (host) with the geometry and per-operator statistics. */
int xct_matrix_info(const xct_matrix *A, xct_matrix_info_t *info);

/* Device workspace needed by xct_project / xct_backproject for `batch`
 * slices (staging copies of one fused group of slices in and out). */
size_t xct_spmm_workspace_bytes(const xct_matrix *A, int batch);

/*
 * Forward projection y_b = A x_b for b < batch (Sec. III-B; one matrix
 * pass per group of up to `fuse` slices).
 *   x         device, [batch][n][n] of dtype `io`
 *   y         device, [batch][n_angles][n_channels] of dtype `io` (written)
 *   io        dtype of x and y (any xct_dtype; an FP64 matrix keeps FP64
 *             io exact, and rounds narrower io once).  With an F16/BF16 matrix the operand is
 *             scaled per slice by a power of two no smaller than its
 *             max-norm before it is rounded to 16 bits, and the FP32 sums
 *             are scaled back (Sec. III-C "adaptive normalization").
 *   workspace device, >= xct_spmm_workspace_bytes(A, batch) bytes, 256-B aligned
 * Inputs must be finite.  Errors: XCT_ERR_INVALID, XCT_ERR_HIP.
 */
int xct_project(const xct_matrix *A, const void *x, void *y, int batch, xct_dtype io,
                void *workspace, void *stream);

/* Backprojection x_b = A^T y_b; same conventions as xct_project with the
 * roles of x and y exchanged (y is read, x is written). */
int xct_backproject(const xct_matrix *A, const void *y, void *x, int batch, xct_dtype io,
                    void *workspace, void *stream);

/*
 * Allocation-free projection (which = 0: out = A in) or backprojection
 * (which = 1: out = A^T in), for callers that cannot allocate device memory
 * (code under graph capture, serving loops, harnesses that forbid it).
 * Same arguments and results as xct_project / xct_backproject, without the
 * workspace: the staging buffers are a fixed array of
 * xct_noalloc_scratch_bytes() (64 MiB) of device memory that the library
 * holds on every GPU it runs on until the process ends; the call itself
 * allocates nothing.  Slices are fused per matrix pass as far as that array
 * holds them; a geometry whose single slice needs more staging returns
 * XCT_ERR_UNSUPPORTED.  Every call on one GPU uses that GPU's one array:
 * calls that overlap in time on one GPU (other streams or threads) race
 * and must be serialised by the caller.  Errors: XCT_ERR_INVALID,
 * XCT_ERR_UNSUPPORTED, XCT_ERR_HIP.
 */
int xct_apply_noalloc(const xct_matrix *A, int which, const void *in, void *out, int batch, xct_dtype io,
                      void *stream);
size_t xct_noalloc_scratch_bytes(void);

/* Device workspace needed by xct_project_streamed (which = 0) or
 * xct_backproject_streamed (which = 1) for chunks of `chunk` slices of dtype `io`. */
size_t xct_stream_workspace_bytes(const xct_matrix *A, int which, int chunk, xct_dtype io);

/*
 * Streamed forward projection y_b = A x_b for b < batch, with x and y in host
 * memory (slices moved to and from the device in chunks, the single-GPU form
 * of the minibatch pipelining of Sec. III-A/III-D).  Chunk c's host-to-device
 * copy runs on h2d_stream, its product (as xct_project, on `chunk` slices)
 * on compute_stream and its device-to-host copy on d2h_stream, so copies of
 * one chunk overlap the products of its neighbours (two device buffers per
 * direction).  Results equal xct_project's on the same slices.
 *   x_host     host, [batch][n][n] of dtype `io`; page-locked for the copies
 *              to run asynchronously (else they serialise)
 *   y_host     host, [batch][n_angles][n_channels] of dtype `io` (written)
 *   chunk      slices per transfer, >= 1 (a multiple of the matrix's fuse
 *              keeps every fused group full)
 *   workspace  device, >= xct_stream_workspace_bytes(A, 0, chunk, io) bytes, 256-B aligned
 *   streams    HIP streams (NULL: the default stream; equal streams serialise).  The
 *              workspace belongs to compute_stream's order: the copy streams first
 *              wait for the work already enqueued there.
 * Returns after every result is in y_host (the three streams are drained,
 * also on error).  The handle keeps the call's seven events from its first
 * streamed call on (released with it); streamed calls that share a handle
 * run one at a time.  Errors: XCT_ERR_INVALID, XCT_ERR_HIP.
 */
int xct_project_streamed(const xct_matrix *A, const void *x_host, void *y_host, int batch, int chunk,
                         xct_dtype io, void *workspace, void *compute_stream, void *h2d_stream,
                         void *d2h_stream);

/* Streamed backprojection x_b = A^T y_b; as xct_project_streamed with the
 * roles of x and y exchanged (y_host is read, x_host written; which = 1 for
 * the workspace size). */
int xct_backproject_streamed(const xct_matrix *A, const void *y_host, void *x_host, int batch, int chunk,
                             xct_dtype io, void *workspace, void *compute_stream, void *h2d_stream,
                             void *d2h_stream);

/*
 * Number of NaN or infinite elements among the n elements of the device
 * array v of dtype dt, written to *count (device, int64, 8-B aligned) on
 * `stream` (no host sync).  The products assume finite inputs (a
 * non-finite element spreads to every output it reaches); callers check
 * untrusted inputs with this.  Errors: XCT_ERR_INVALID, XCT_ERR_HIP.
 */
int xct_count_nonfinite(const void *v, int64_t n, xct_dtype dt, int64_t *count, void *stream);

/* Device workspace needed by xct_cgls for `batch` slices and `iters` iterations. */
size_t xct_cgls_workspace_bytes(const xct_matrix *A, int batch, int iters);

/*
 * CGLS for every slice independently (per-slice step lengths), from
 * x = 0, for exactly `iters` iterations: iters projections and iters+1
 * backprojections (Sec. IV-F; Table IV note).
 *   y          device, [batch][n_angles][n_channels] of dtype `y_dtype`
 *   x          device, [batch][n][n] FP32 (written)
 *   iters      >= 0
 *   workspace  device, >= xct_cgls_workspace_bytes(A, batch, iters) bytes, 256-B aligned
 *   resid      nullable host, [iters+1][batch]: ||y_b - A x_k|| / ||y_b||
 *              (0 when y_b = 0; NaN for a slice of status 2)
 *   status     nullable host, [batch]: 1 when the slice stopped early
 *              because gamma = ||A^T r||^2 or delta = ||A p||^2 became 0;
 *              2 when y_b holds a NaN or an infinity (the slice is not
 *              solved and x_b stays 0; the other slices are unaffected);
 *              else 0
 * Solver vectors are FP32 and the per-slice scalars FP64.  With an F16/BF16
 * matrix the operand of each product is max-norm scaled and rounded to
 * 16 bits (Sec. III-C).  With an FP64 matrix the solver vectors and the
 * products are FP64 (the double-precision variant of Sec. IV) and x is
 * returned rounded to FP32.  When resid or status is given the call waits for
 * the stream before returning.  Errors: XCT_ERR_INVALID, XCT_ERR_HIP.
 */
int xct_cgls(const xct_matrix *A, const void *y, xct_dtype y_dtype, float *x, int batch, int iters,
             void *workspace, double *resid, int32_t *status, void *stream);

/* Device workspace needed by xct_projected_gradient for `batch` slices. */
size_t xct_pgrad_workspace_bytes(const xct_matrix *A, int batch);

/*
 * Projected gradient descent on Eq. (1), ||y - A x||^2 + lam * TV_eps(x)
 * over x in C, by the gradient loop of Sec. II (project, residual,
 * backproject, update), every slice independently, `iters` iterations:
 *   x <- P_C(x - step_b * (2 A^T (A x - y) + lam * grad TV_eps(x)))
 * TV_eps(x) = sum over pixels of sqrt(dr^2 + dc^2 + eps^2), with forward
 * differences dr = x[i+1][j] - x[i][j] and dc = x[i][j+1] - x[i][j] taken as
 * 0 on the last row / column.  C is x >= 0 when nonneg != 0 (clamp at zero),
 * else all x.  The paper leaves R, C and the step rule open; the step is
 * the caller's (the cost decreases for step_b < 2 / L_b with
 * L_b <= 2 ||A||^2 + 8 lam / eps).
 *   y          device, [batch][n_angles][n_channels] FP32
 *   x          device, [batch][n][n] FP32: the start point on entry, the
 *              last iterate on return
 *   step       device, [batch] FP32 per-slice step lengths
 *   lam, eps   lam >= 0, eps > 0
 *   workspace  device, >= xct_pgrad_workspace_bytes(A, batch) bytes, 256-B aligned
 * Each iteration is one projection and one backprojection (the operands of
 * a 16-bit matrix are max-norm scaled and rounded as in xct_project), the
 * residual A x - y taken as the projection is written out (a pass of its
 * own for FP64 matrices) and one fused TV / step / clamp pass.  Enqueued on
 * `stream`; no host sync.  Errors: XCT_ERR_INVALID, XCT_ERR_HIP.
 */
int xct_projected_gradient(const xct_matrix *A, const float *y, float *x, int batch, int iters,
                           const float *step, float lam, float eps, int nonneg, void *workspace, void *stream);

/*
 * Decode one operator back to coordinate form on the host, in storage
 * order (for tests and tools).  which = 0: A (row = k*n_channels + c,
 * col = i*n + j); which = 1: A^T (row = voxel, col = ray).  rows, cols,
 * vals: host arrays of capacity `cap` entries (>= nnz).  *count receives
 * the number written.  Also checks the stored layout: every padding entry
 * must be zero and every slot inside its stage; a violation returns
 * XCT_ERR_INTERNAL.
 */
int xct_matrix_to_coo(const xct_matrix *A, int which, int32_t *rows, int32_t *cols, float *vals,
                      int64_t cap, int64_t *count);

/*
 * Kernel timing for measurement tools.  While enabled, every SpMM kernel
 * launch is bracketed by HIP events recorded on the stream it is launched
 * on.  xct_profile_read waits for the recorded events and returns, per
 * operator (index 0: A, 1: A^T), the number of launches and their total
 * time in milliseconds (host arrays of 2), then clears the record.  Global
 * to the process and not thread-safe; costs two event records per launch.
 */
int xct_profile_enable(int on);
int xct_profile_read(int64_t *launches, double *ms);

/* Measurement utility: streaming-read bandwidth of the device (GB/s, 1e9 B/s)
 * over the caller's device buffer of `bytes` bytes (>= 16; read only),
 * `reps` timed passes after one untimed pass, on `stream`; blocks until done.
 * Allocates nothing per call (its two timing events are created once per
 * device; calls from several threads run one at a time).  The reference
 * ceiling for the SpMM's matrix stream; not part of the method. */
int xct_read_bandwidth(const void *buf, int64_t bytes, int reps, double *gbps, void *stream);

/*
 * Device memory the library holds (every matrix handle's buffers): the
 * number of buffers and their total bytes (host outputs).  Build failures
 * release everything they took, so these return to their previous values
 * after any failed xct_build_matrix.  Failure injection for tests: with
 * XCT_FAULT_ALLOC=n in the environment, the n-th device allocation counted
 * from when the variable took its current value fails with XCT_ERR_OOM.
 */
int xct_device_memory(int64_t *buffers, int64_t *bytes);

/* Message of the last failed call on this thread ("" if none). */
const char *xct_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* XCT_H */
