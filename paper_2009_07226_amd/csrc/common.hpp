// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/xct.h"

namespace xct {

// A tile is 8 x 8 elements of a 2D grid (voxels of a slice, or angles x
// channels of a sinogram): 64 slots, one wavefront of rows.
constexpr int kTile = 8;
constexpr int kTileSlots = 64;
// ELL entries are stored in groups of kGroup consecutive steps per lane so
// one lane reads a group with a single wide load.
constexpr int kGroup = 4;
// Most slices fused per matrix pass (32 with 16-bit operands, 16 with FP32).
constexpr int kMaxFuse = 32;
// One operator (A or A^T) in staged-ELL form.
//
// Output rows are grouped in tiles of 64 (one wavefront of lanes); W
// consecutive row tiles in Hilbert order make one workgroup ("block") of
// P = W / R wavefronts, wavefront w holding row tiles h * P + w (h < R).  The
// input tiles a block touches, in its staging order, form its tile list; the
// list is cut into stages of at most T tiles, each loaded into LDS in turn.
// For stage s and row tile the entries of its 64 rows that fall in the stage
// form one ELL slab; slabs are stored wavefront by wavefront (each
// wavefront's stages in order, its R row tiles interleaved per stage), so
// slab[blk_stage[b]*W + (w*nst_b + s)*R + h] .. [+1] bounds the groups of
// (s, h * P + w) in block b (nst_b stages) and a wavefront's slabs are one
// contiguous stream.
// Entry (group g, lane l, step q) lives at index (g*64 + l)*kGroup + q and
// holds the stage-local slot (tile position * 64 + offset in tile: the row of
// the staged input in LDS) and the length.
struct OpPlan {
    int which = 0;  // 0: A (projection), 1: A^T (backprojection)
    int64_t n_row_tiles = 0;
    int64_t n_in_tiles = 0;
    int W = 0;  // row tiles per block
    int R = 1;  // row tiles per wavefront (W / R wavefronts per block)
    int arith16 = 0;  // FP16 arithmetic (FP16 matrix; measurement variant)
    int poison = 0;   // debug: NaN-fill the LDS stage buffer before each stage copy
    int T = 0;  // input tiles per stage
    int n_blocks = 0;
    int lanes = 0;  // lane_slot order of the rows within a row tile
    int64_t n_stages = 0;
    int64_t n_groups = 0;
    int64_t n_list = 0;
    int32_t *blk_stage = nullptr;  // [n_blocks+1]
    int32_t *blk_tile = nullptr;   // [n_blocks+1]
    int32_t *tile_list = nullptr;  // [n_list] input tile ranks
    int64_t *slab = nullptr;       // [n_stages*W+1] group offsets, wave-major within a block
    // Entries, one buffer (ent) holding n_groups groups:
    //  F32 format: a group is 1536 bytes, 64 lanes x 4 u16 slots (512 B) then
    //    64 lanes x 4 f32 lengths (1 KB); slot of (g, lane, q) is
    //    slot[g*768 + lane*4 + q], its length val[g*384 + 128 + lane*4 + q];
    //  F64 format: a group is 2560 bytes, 64 lanes x 4 u16 slots (512 B) then
    //    64 lanes x 4 f64 lengths (2 KB); slot of (g, lane, q) is
    //    slot[g*1280 + lane*4 + q], its length val64[g*320 + 64 + lane*4 + q];
    //  F16/BF16 format: a group is 1024 bytes, packed[(g*64 + lane)*4 + q] =
    //    slot << 16 | value bits.
    // slot, val, val64 and packed are views of ent.
    void *ent = nullptr;
    uint16_t *slot = nullptr;
    float *val = nullptr;
    double *val64 = nullptr;
    uint32_t *packed = nullptr;
    int64_t nnz = 0, padded = 0, staged_slots = 0, bytes = 0;
    int64_t n_slabs = 0, balanced = 0;  // (stage, wavefront) slabs; those reordered against bank conflicts
};

// Lane -> slot of the row tile: 0 row-major (lane = slot), 1 transposed.
__host__ __device__ inline int lane_slot(int lane, int order) {
    return order ? (((lane & 7) << 3) | (lane >> 3)) : lane;
}
// Geometry of one tiled 2D grid (H rows x Wd columns).
struct Grid {
    int H = 0, Wd = 0;
    int TH = 0, TW = 0;            // tiles per column / per row
    int64_t n_tiles = 0;
    int32_t *rank_of = nullptr;    // [TH*TW] raster tile -> Hilbert rank (device)
    int32_t *coord_of = nullptr;   // [n_tiles] Hilbert rank -> raster tile (device)
    std::vector<int32_t> h_rank_of, h_coord_of;  // host copies
};

}  // namespace xct

struct xct_matrix {
    int n = 0, M = 0, C = 0;
    xct_dtype vdt = XCT_F32;
    int fuse = 16;
    int remap = 0;  // the xcd_remap build option
    xct::Grid vol, sino;
    xct::OpPlan A, AT;
    double build_seconds = 0.0;
    // The streamed calls' events, created at the first such call on the
    // handle and released with it; the mutex serialises streamed calls that
    // share the handle (each returns only once its streams are drained).
    std::mutex stream_mu;
    hipEvent_t stream_ev[7] = {};
};

namespace xct {

// thread-local last error
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

// The library's device allocations (counted for xct_device_memory; see
// build.hip for the failure injection).
hipError_t dev_alloc(void **p, size_t bytes);
void dev_free(void *p);

#define XCT_HIP_TRY(expr)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::xct::fail(e_ == hipErrorOutOfMemory ? XCT_ERR_OOM : XCT_ERR_HIP,       \
                               std::string(#expr) + ": " + hipGetErrorString(e_));          \
    } while (0)

inline int elem_bytes(xct_dtype d) { return d == XCT_F64 ? 8 : d == XCT_F32 ? 4 : 2; }
inline bool valid_dtype(int d) { return d == XCT_F32 || d == XCT_F16 || d == XCT_BF16 || d == XCT_F64; }
// Stored bytes per matrix entry: a 16-bit stage-local slot plus the value
// (FP32, FP64), or slot and 16-bit value packed in one word.
inline size_t entry_bytes(xct_dtype d) { return d == XCT_F64 ? 10 : d == XCT_F32 ? 6 : 4; }

// Fused slice count used for a batch: the smallest supported F >= min(batch, fuse).
inline int run_fuse(int batch, int fuse) {
    int want = batch < fuse ? batch : fuse;
    int f = 1;
    while (f < want) f <<= 1;
    return f;
}

// Launch of one staged SpMM pass over a single fused group of F slices.
struct SpmmLaunch {
    const OpPlan *op;
    const void *xin;      // internal layout [in tiles][64][F], storage dtype
    void *yout;           // internal layout [row tiles][64][F], FP32 (FP64 for FP64 matrices)
    const float *scale;   // [F] per-slice output scale or nullptr
    double *sq_partial;   // [n_blocks][F] per-block sums of squared outputs or nullptr
    int F;
    xct_dtype vdt;
    int remap;
    // 16-bit matrices only: write the natural [batch][H][Wd] output of grid *gout
    // directly (slices s0 .. s0 + F - 1, io dtype, minus sub if set) instead
    // of the internal rows at yout
    void *nat = nullptr;
    const float *sub = nullptr;
    const Grid *gout = nullptr;
    int io = 0, batch = 0, s0 = 0;
};
int launch_spmm(const SpmmLaunch &L, hipStream_t s);
// One projection (dir 0) or backprojection (dir 1) of `batch` device slices
// in natural layout, as xct_project / xct_backproject; workspace of
// spmm_workspace(m, batch) bytes, 256-byte aligned.
int spmm_call(const xct_matrix *m, int dir, const void *src, void *dst, int batch, xct_dtype io, void *workspace,
              void *stream);
// r = A x - y for FP32 slices in natural layout (the projection, with the
// subtraction done as its sums are written out); FP32 / 16-bit matrices.
int spmm_residual(const xct_matrix *m, const float *x, const float *y, float *r, int batch, void *workspace,
                  hipStream_t st);
size_t spmm_workspace(const xct_matrix *m, int batch);

// Natural <-> internal layout conversion for one fused group.
//   natural: [batch][H][Wd] of dtype io; group covers slices s0 .. s0+F-1
//   internal: [n_tiles][64][F]
//   to_internal: optional per-slice inverse scale (1/m) read from device
//   memory `inv_scale` [F]; values for slices >= batch are zero.
int launch_to_internal(const Grid &g, const void *nat, xct_dtype io, int batch, int s0, int F,
                       void *internal, xct_dtype storage, const float *inv_scale, hipStream_t s);
//   from_internal: with `sub` (natural layout like nat, io FP32), writes
//   the values minus sub.
int launch_from_internal(const Grid &g, const float *internal, int batch, int s0, int F, void *nat,
                         xct_dtype io, hipStream_t s, const float *sub = nullptr);
// The same from FP64 internal rows (FP64 matrices).
int launch_from_internal64(const Grid &g, const double *internal, int batch, int s0, int F, void *nat,
                           xct_dtype io, hipStream_t s);
// From per-slice max |v| bits in amax[F]: scale[f] = m = 2^ceil(log2 max)
// (1 for zero), inv[f] = 1/m; clears amax for reuse.
int launch_pow2_scale(uint32_t *amax, int F, float *scale, float *inv, hipStream_t s);
// The normalisation of a 16-bit operand with max |v| = mx: the smallest power
// of two m >= mx (1 for zero or a non-finite max), so v / m lies in [-1, 1].
__device__ __forceinline__ float pow2_at_least(float mx) {
    float m = 1.f;
    if (mx > 0.f && mx <= 3.0e38f) {
        int e;
        const float mant = frexpf(mx, &e);  // mx = mant * 2^e, mant in [0.5, 1)
        m = ldexpf(1.f, mant == 0.5f ? e - 1 : e);
    }
    return m;
}
// Per-slice max |v| of a natural-layout group, accumulated as float bits into
// amax[F] (zero on entry), then launch_pow2_scale.
int launch_natural_scale(const Grid &g, const void *nat, xct_dtype io, int batch, int s0, int F,
                         uint32_t *amax, float *scale, float *inv, hipStream_t s);

}  // namespace xct
