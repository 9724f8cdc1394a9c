// Staged sparse-matrix times fused-slices product (projection with A,
// backprojection with A^T), and the layout conversions around it.
//
// The paper's XCT-optimised SpMM (Sec. III-B, Listing 1): one thread per
// output row holds the partial sums of F fused slices in registers
// ("3D output buffering"); each (index, length) pair is read once and used
// for all F slices ("register reuse"); the input footprint of a block is
// staged through on-chip memory stage by stage ("3D input buffering",
// "multi-stage"), indices being stage-local.  The same kernel serves A and
// A^T.  16-bit storage with FP32 arithmetic follows Sec. III-C.
//
// gfx950 design:
//   * a row tile of 64 rows is exactly one wave64; a workgroup is W row
//     tiles, consecutive along the Hilbert curve;
//   * vectors live in a tile-interleaved layout [tile][64][F] so a stage
//     load copies whole 64*F-element tiles (contiguous, 16 B per lane) and a
//     lane's F operands of one slot are one contiguous LDS row, read with
//     16-byte LDS loads;
//   * ELL entries are grouped four steps per lane so one lane fetches four
//     (slot, length) pairs with one wide non-temporal load (the matrix is
//     streamed once per pass and should not evict the vectors from L2/MALL);
//   * workgroup ids are remapped so that each XCD takes runs of consecutive
//     blocks of the Hilbert order (which share most of their input
//     footprint, in its L2) while the eight XCDs advance through the order
//     together (their staged tiles shared in the memory-side cache).
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "common.hpp"

namespace xct {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float h16_to_f32(uint32_t bits) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)bits);
}
__device__ __forceinline__ float bf16_to_f32(uint32_t bits) { return __builtin_bit_cast(float, bits << 16); }
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Storage element of the staged operand.
template <int FMT> struct Stor;
template <> struct Stor<XCT_F32> { typedef float T; };
template <> struct Stor<XCT_F16> { typedef uint16_t T; };
template <> struct Stor<XCT_BF16> { typedef uint16_t T; };
template <> struct Stor<XCT_F64> { typedef double T; };

// Accumulator (and output) type: FP64 for FP64 matrices, else FP32.
template <int FMT> struct Acc { typedef float T; };
template <> struct Acc<XCT_F64> { typedef double T; };

__device__ __forceinline__ float fma_acc(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fma_acc(double a, double b, double c) { return fma(a, b, c); }

// Shape of one staged row (the F operands of one slot).
template <int FMT, int F>
struct RowShape {
    typedef typename Stor<FMT>::T XT;
    static constexpr int RB = F * (int)sizeof(XT);   // bytes per row
    static constexpr int CH = RB >= 16 ? RB / 16 : 1; // 16-byte chunks per row (rows below 16 B: one piece)
    static constexpr int SPC = F / CH;                // slices per chunk
};

// Expand one 16-byte chunk (or a sub-16-byte row) into SPC values of the
// accumulator type.
template <int FMT, int SPC>
__device__ __forceinline__ void expand(const u32x4 w, typename Acc<FMT>::T (&x)[SPC]) {
    if constexpr (FMT == XCT_F64) {
        const uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int t = 0; t < SPC; ++t)
            x[t] = __builtin_bit_cast(double, (uint64_t)u[2 * t] | ((uint64_t)u[2 * t + 1] << 32));
    } else if constexpr (FMT == XCT_F32) {
        const uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int t = 0; t < SPC; ++t) x[t] = __builtin_bit_cast(float, u[t]);
    } else {
        const uint32_t u[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int t = 0; t < SPC; ++t) {
            const uint32_t b = (t & 1) ? (u[t >> 1] >> 16) : (u[t >> 1] & 0xffffu);
            x[t] = FMT == XCT_F16 ? h16_to_f32(b) : bf16_to_f32(b);
        }
    }
}

// LDS addresses are 32-bit byte offsets into the workgroup's LDS.
#define XCT_LDS __attribute__((address_space(3)))
template <class T> __device__ __forceinline__ const XCT_LDS T *lds_ptr(uint32_t addr) {
    return (const XCT_LDS T *)(uintptr_t)addr;
}
__device__ __forceinline__ uint32_t lds_addr(const char *generic_smem) {
    return (uint32_t)(uintptr_t)(XCT_LDS const char *)generic_smem;
}

// Address of a staged row's chunk: slot * RB + cb, the slot being the low
// (HI = false) or high half of `packed`.  One v_mad_u32_u16 whose operand
// select picks the half, so extracting the slot costs nothing.
template <int RB, bool HI>
__device__ __forceinline__ uint32_t row_addr(uint32_t packed, uint32_t cb) {
    static_assert(RB > 0 && RB <= 64, "RB must be an inline constant");
    uint32_t r;
    if constexpr (HI)
        asm("v_mad_u32_u16 %0, %1, %2, %3 op_sel:[1,0,0,0]" : "=v"(r) : "v"(packed), "i"(RB), "v"(cb));
    else
        asm("v_mad_u32_u16 %0, %1, %2, %3" : "=v"(r) : "v"(packed), "i"(RB), "v"(cb));
    return r;
}

// Load a row of fewer than 16 bytes.
template <int RB>
__device__ __forceinline__ u32x4 load_small(uint32_t addr) {
    u32x4 w = {0u, 0u, 0u, 0u};
    if constexpr (RB == 8) {
        const u32x2 v = *lds_ptr<u32x2>(addr);
        w.x = v.x;
        w.y = v.y;
    } else if constexpr (RB == 4) {
        w.x = *lds_ptr<uint32_t>(addr);
    } else {
        w.x = *lds_ptr<uint16_t>(addr);
    }
    return w;
}

// ---- natural-layout element access (any io dtype) --------------------------

__device__ __forceinline__ float load_io(const void *p, int64_t i, int io) {
    if (io == XCT_F32) return ((const float *)p)[i];
    if (io == XCT_F64) return (float)((const double *)p)[i];
    const uint16_t b = ((const uint16_t *)p)[i];
    return io == XCT_F16 ? h16_to_f32(b) : bf16_to_f32(b);
}

__device__ __forceinline__ uint32_t f32_to_h16(float v) {
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)v);
}
__device__ __forceinline__ uint32_t f32_to_bf16(float v) {
    uint32_t u = __builtin_bit_cast(uint32_t, v);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;  // NaN stays NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                  // nearest-even
    return u >> 16;
}

__device__ __forceinline__ void store_io(void *p, int64_t i, float v, int io) {
    if (io == XCT_F32)
        ((float *)p)[i] = v;
    else if (io == XCT_F64)
        ((double *)p)[i] = (double)v;
    else
        ((uint16_t *)p)[i] = (uint16_t)(io == XCT_F16 ? f32_to_h16(v) : f32_to_bf16(v));
}

struct SpmmArgs {
    const int32_t *blk_stage, *blk_tile, *tile_list;
    const int64_t *slab;
    const uint16_t *slot;
    const float *val;
    const uint32_t *packed;
    const void *xin;
    void *yout;  // FP32 sums, FP64 for FP64 matrices
    const float *scale;
    double *sq_partial;
    int64_t n_row_tiles;
    int n_blocks, T, remap, lanes;  // remap: consecutive blocks per XCD chunk (0: plain order)
    int W;  // row tiles per block (R per wavefront)
    // Sums written straight to the natural [batch][H][Wd] output (16-bit
    // matrices) when nat is set, instead of the internal rows at yout: slice
    // s0 + f of the group, minus sub at the same index when sub is set.
    void *nat;
    const float *sub;
    const int32_t *row_coord;  // row tile (Hilbert rank) -> raster tile of the output grid
    int64_t plane;
    int H, Wd, rowTW, io, batch, s0;
};

// One group: kGroup consecutive ELL steps of one lane.
template <int FMT> struct Group;
template <> struct Group<XCT_F32> { u32x2 s; f32x4 v; };
template <> struct Group<XCT_F16> { u32x4 p; };
template <> struct Group<XCT_BF16> { u32x4 p; };
template <> struct Group<XCT_F64> { u32x2 s; u32x4 v01, v23; };

// Bytes of one group (64 lanes x kGroup entries; layout: see OpPlan).
template <int FMT> struct GroupBytes { static constexpr int value = 1024; };
template <> struct GroupBytes<XCT_F32> { static constexpr int value = 1536; };
template <> struct GroupBytes<XCT_F64> { static constexpr int value = 2560; };

// Lane `lane`'s part of group g of a wavefront's entry stream, read through
// a buffer descriptor of the stream: the group offset is a scalar operand, so
// the address arithmetic costs no vector instructions.  Streamed once:
// non-temporal.
constexpr int kRsrcWord3 = 0x00020000;  // raw buffer, 32-bit data format
constexpr int kNonTemporal = 2;
template <int FMT>
__device__ __forceinline__ Group<FMT> load_group(__amdgpu_buffer_rsrc_t rs, int g, int lane) {
    Group<FMT> r;
    const int so = g * GroupBytes<FMT>::value;
    if constexpr (FMT == XCT_F32) {
        r.s = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, lane * 8, so, kNonTemporal));
        r.v = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, 512 + lane * 16, so, kNonTemporal));
    } else if constexpr (FMT == XCT_F64) {
        r.s = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, lane * 8, so, kNonTemporal));
        r.v01 = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, 512 + lane * 32, so, kNonTemporal));
        r.v23 =
            __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, 528 + lane * 32, so, kNonTemporal));
    } else {
        r.p = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, lane * 16, so, kNonTemporal));
    }
    return r;
}

template <int FMT, int F, int KB>
__device__ __forceinline__ void use_group(const Group<FMT> &g, const uint32_t (&cb)[RowShape<FMT, F>::CH],
                                          typename Acc<FMT>::T (&acc)[F]) {
    typedef RowShape<FMT, F> R;
    typedef typename Acc<FMT>::T AT;
    // the word holding step q's slot, and whether it is the high half
    uint32_t sw[kGroup];
    AT v[kGroup];
    if constexpr (FMT == XCT_F64) {
        sw[0] = sw[1] = g.s.x;
        sw[2] = sw[3] = g.s.y;
        v[0] = __builtin_bit_cast(double, (uint64_t)g.v01.x | ((uint64_t)g.v01.y << 32));
        v[1] = __builtin_bit_cast(double, (uint64_t)g.v01.z | ((uint64_t)g.v01.w << 32));
        v[2] = __builtin_bit_cast(double, (uint64_t)g.v23.x | ((uint64_t)g.v23.y << 32));
        v[3] = __builtin_bit_cast(double, (uint64_t)g.v23.z | ((uint64_t)g.v23.w << 32));
    } else if constexpr (FMT == XCT_F32) {
        sw[0] = sw[1] = g.s.x;
        sw[2] = sw[3] = g.s.y;
        v[0] = g.v.x;
        v[1] = g.v.y;
        v[2] = g.v.z;
        v[3] = g.v.w;
    } else {
        const uint32_t p[4] = {g.p.x, g.p.y, g.p.z, g.p.w};
#pragma unroll
        for (int q = 0; q < kGroup; ++q) {
            sw[q] = p[q];
            v[q] = FMT == XCT_F16 ? h16_to_f32(p[q] & 0xffffu) : bf16_to_f32(p[q] & 0xffffu);
        }
    }
    // The LDS reads of KB steps are issued together ahead of their FMAs, so
    // a wavefront waits for LDS latency once per KB steps.
    static_assert(kGroup % KB == 0, "KB must divide the group");
#pragma unroll
    for (int q0 = 0; q0 < kGroup; q0 += KB) {
        u32x4 w[KB][R::CH];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const int q = q0 + k;
            constexpr bool kHiAlways = FMT == XCT_F16 || FMT == XCT_BF16;  // 16-bit entries: slot << 16 | value
#pragma unroll
            for (int j = 0; j < R::CH; ++j) {
                const uint32_t ad = (kHiAlways || (q & 1)) ? row_addr<R::RB, true>(sw[q], cb[j])
                                                            : row_addr<R::RB, false>(sw[q], cb[j]);
                if constexpr (R::RB >= 16)
                    w[k][j] = *lds_ptr<u32x4>(ad);
                else
                    w[k][j] = load_small<R::RB>(ad);
            }
        }
        __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the FMAs
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            if constexpr (FMT == XCT_BF16 && R::SPC >= 2) {
                // BF16: one v_dot2c_f32_bf16 per slice takes the packed pair
                // of operands as stored, against (value, 0) for the even
                // slice and (0, value) for the odd one: the product of two
                // BF16 values is exact in FP32, so each step is a single
                // FP32 rounding of the sum, as with the FMA after widening
                // (which costs one more instruction per slice).
                const uint32_t pv = sw[q0 + k];  // slot << 16 | value
                const bf16x2 vlo = __builtin_bit_cast(bf16x2, pv & 0xffffu);
                const bf16x2 vhi = __builtin_bit_cast(bf16x2, pv << 16);
#pragma unroll
                for (int j = 0; j < R::CH; ++j) {
                    const uint32_t u[4] = {w[k][j].x, w[k][j].y, w[k][j].z, w[k][j].w};
#pragma unroll
                    for (int t = 0; t < R::SPC / 2; ++t) {
                        const bf16x2 x2 = __builtin_bit_cast(bf16x2, u[t]);
                        float &a0 = acc[j * R::SPC + 2 * t], &a1 = acc[j * R::SPC + 2 * t + 1];
                        a0 = __builtin_amdgcn_fdot2_f32_bf16(vlo, x2, a0, false);
                        a1 = __builtin_amdgcn_fdot2_f32_bf16(vhi, x2, a1, false);
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < R::CH; ++j) {
                    AT x[R::SPC];
                    expand<FMT, R::SPC>(w[k][j], x);
#pragma unroll
                    for (int t = 0; t < R::SPC; ++t)
                        acc[j * R::SPC + t] = fma_acc(v[q0 + k], x[t], acc[j * R::SPC + t]);
                }
            }
        }
    }
}

// FP16 arithmetic (the paper's "half precision" variant, measurement only):
// F/2 packed FP16 accumulators, one v_pk_fma_f16 per two slices and entry.
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

template <int F, int KB>
__device__ __forceinline__ void use_group_h16(const Group<XCT_F16> &g,
                                              const uint32_t (&cb)[RowShape<XCT_F16, F>::CH], h2 (&acc)[F / 2]) {
    typedef RowShape<XCT_F16, F> R;
    static_assert(R::SPC % 2 == 0, "pairs of slices per chunk");
    const uint32_t p[4] = {g.p.x, g.p.y, g.p.z, g.p.w};
#pragma unroll
    for (int q0 = 0; q0 < kGroup; q0 += KB) {
        u32x4 w[KB][R::CH];
#pragma unroll
        for (int k = 0; k < KB; ++k) {
#pragma unroll
            for (int j = 0; j < R::CH; ++j) {
                const uint32_t ad = row_addr<R::RB, true>(p[q0 + k], cb[j]);
                if constexpr (R::RB >= 16)
                    w[k][j] = *lds_ptr<u32x4>(ad);
                else
                    w[k][j] = load_small<R::RB>(ad);
            }
        }
        __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of the FMAs
#pragma unroll
        for (int k = 0; k < KB; ++k) {
            const _Float16 vh = __builtin_bit_cast(_Float16, (uint16_t)(p[q0 + k] & 0xffffu));
            const h2 v2 = {vh, vh};
#pragma unroll
            for (int j = 0; j < R::CH; ++j) {
                const uint32_t u[4] = {w[k][j].x, w[k][j].y, w[k][j].z, w[k][j].w};
#pragma unroll
                for (int t = 0; t < R::SPC / 2; ++t) {
                    const h2 x2 = __builtin_bit_cast(h2, u[t]);
                    acc[j * (R::SPC / 2) + t] = __builtin_elementwise_fma(v2, x2, acc[j * (R::SPC / 2) + t]);
                }
            }
        }
    }
}

// Scalar loads of wave-uniform metadata (p wave-uniform).  Once the stage
// loop holds the global-to-LDS copy (which the compiler treats as a write to
// memory), it no longer proves these read-only arrays unwritten and turns
// plain loads of them into vector loads followed by full vmcnt waits, which
// would drain the entry ring; these stay on the scalar unit.
typedef int i32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ i32x4 sload_x4(const void *p) {
    i32x4 v;
    asm volatile("s_load_dwordx4 %0, %1, 0x0\n\ts_waitcnt lgkmcnt(0)" : "=s"(v) : "s"(p));
    return v;
}

// Issue priority of a wavefront from the groups it has left in the stage.
// The SIMD arbiter otherwise favours the oldest wavefronts of the workgroup,
// so the youngest ones finish each stage last and the stage barrier waits
// for them (measured: 2.3x spread in time per group between the waves of a
// SIMD).  Favouring the wavefronts with the most work left keeps all four
// waves of a SIMD busy until the end of the stage.
constexpr int kPrioStep = 8;  // groups per priority level
__device__ __forceinline__ void prio_for_remaining(int rem) {
    if (rem >= 3 * kPrioStep)
        __builtin_amdgcn_s_setprio(3);
    else if (rem >= 2 * kPrioStep)
        __builtin_amdgcn_s_setprio(2);
    else if (rem >= kPrioStep)
        __builtin_amdgcn_s_setprio(1);
    else
        __builtin_amdgcn_s_setprio(0);
}

// Entries in flight per wavefront: the ring holds the next D groups of the
// wave's entry stream, which runs through all stages of the block.  In the
// stage-by-stage loop (16-bit matrices) every pass reloads all D slots, so a
// stage whose group count is not a multiple of D re-reads some groups: D = 3
// or 4 measured fastest (2, 6 and 8 slower).  The flat loop (FP32) reloads a
// slot only once consumed: D = 5 with the LDS reads of two steps issued
// together (F = 16) measured best there (D = 4 with whole-group reads: +0.7%
// at 16 x 1024^2, +1.4% at 64 x 2048^2; D = 6 spills registers).
template <int FMT> struct RingDepth { static constexpr int value = 4; };
template <> struct RingDepth<XCT_F32> { static constexpr int value = 5; };
template <> struct RingDepth<XCT_F64> { static constexpr int value = 3; };  // 10 registers a group

// LDS reads issued together: the whole group, or half of it where the
// registers are needed elsewhere (the deeper FP32 ring, two FP32 accumulator
// sets of 16 slices, 32 slices, FP64 rows).
template <int FMT, int F, int RT> struct ReadBatch { static constexpr int value = 4; };
template <> struct ReadBatch<XCT_F32, 16, 1> { static constexpr int value = 2; };
template <> struct ReadBatch<XCT_F32, 16, 2> { static constexpr int value = 2; };
template <> struct ReadBatch<XCT_F16, 32, 1> { static constexpr int value = 2; };
template <int F> struct ReadBatch<XCT_F64, F, 1> { static constexpr int value = 2; };
template <int F> struct ReadBatch<XCT_F64, F, 2> { static constexpr int value = 1; };
template <> struct ReadBatch<XCT_BF16, 32, 1> { static constexpr int value = 2; };

// RT: row tiles per wavefront (a.W / RT wavefronts per block); H16: FP16
// arithmetic on an FP16 matrix (F >= 2); POISON: the debug build option that
// NaN-fills the stage buffer before each stage copy.
template <int FMT, int F, int RT, bool H16, bool POISON>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(4, 4))) k_spmm(SpmmArgs a) {
    typedef RowShape<FMT, F> R;
    constexpr int D = RingDepth<FMT>::value;
    constexpr int KB = ReadBatch<FMT, F, RT>::value;
    extern __shared__ __align__(16) char smem[];
    const int tid = threadIdx.x, nthr = blockDim.x, P = nthr >> 6, W = a.W;
    // wave-uniform: keeps the slab bounds and loop control in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    // Workgroup i runs on XCD i mod 8 (the dispatcher deals workgroups to
    // the XCDs in turn); its k-th workgroup takes block (chunk * 8 + xcd) * G
    // + k mod G with chunk = k / G: each XCD works through runs of G
    // consecutive blocks (sharing their input tiles in its L2) while the
    // eight XCDs advance through the Hilbert order together (their staged
    // tiles shared in the memory-side cache).
    int b = blockIdx.x;
    if (a.remap > 0) {
        const int G = a.remap, xcd = blockIdx.x & 7, k = blockIdx.x >> 3;
        b = ((k / G) * 8 + xcd) * G + k % G;
    }
    if (b >= a.n_blocks) return;  // whole workgroup, before any barrier

    // Lane l reads chunk (j + l) mod CH of a row at sub-step j, so the lanes
    // of one LDS cycle spread over the chunks; accumulator block j holds the
    // slices of that rotated chunk.
    int coff[R::CH];
    uint32_t cb[R::CH];  // LDS address of this lane's chunk j of row 0
#pragma unroll
    for (int j = 0; j < R::CH; ++j) {
        coff[j] = ((j + lane) & (R::CH - 1)) * 16;
        cb[j] = lds_addr(smem) + coff[j];
    }
    static_assert(!H16 || (FMT == XCT_F16 && F >= 2), "FP16 arithmetic needs an FP16 matrix and F >= 2");
    typedef typename Acc<FMT>::T AT;
    AT acc[RT][H16 ? 1 : F];
    h2 acc2[RT][H16 ? F / 2 : 1];
#pragma unroll
    for (int h = 0; h < RT; ++h) {
#pragma unroll
        for (int f = 0; f < (H16 ? 1 : F); ++f) acc[h][f] = (AT)0;
#pragma unroll
        for (int f = 0; f < (H16 ? F / 2 : 1); ++f) acc2[h][f] = h2{(_Float16)0, (_Float16)0};
    }

    constexpr int kVecPerTile = kTileSlots * R::RB / 16;  // 16-byte vectors per staged tile
    // stages of rows of 16 bytes or more are copied straight into LDS
    constexpr bool kDma = R::RB >= 16;
    const int s0 = a.blk_stage[b], s1 = a.blk_stage[b + 1];
    const int t0 = a.blk_tile[b], t1 = a.blk_tile[b + 1];
    const u32x4 *xin = (const u32x4 *)a.xin;

    // The wave's entries are one contiguous stream of groups [gw, ge); its
    // row tile h uses slab[p0 + (s - s0) * RT + h] .. [+1] in stage s.
    const int nst = s1 - s0;
    const int64_t p0 = (int64_t)s0 * W + (int64_t)wave * nst * RT;
    const int64_t gw = a.slab[p0], ge = a.slab[p0 + nst * RT];
    // Group indices below are relative to the wave's first group (a wave's
    // stream is far below 2^31 bytes).  Past the end of the stream the last
    // group is re-read; an empty stream re-reads the group before it, or
    // group 0 (the builder allocates at least one group).
    constexpr int GB = GroupBytes<FMT>::value;
    const int ne = (int)(ge - gw);
    const int64_t gfirst = ne > 0 ? gw : (gw > 0 ? gw - 1 : 0);
    const char *ent_w =
        (const char *)(FMT == XCT_F32 || FMT == XCT_F64 ? (const void *)a.slot : (const void *)a.packed) + gfirst * GB;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)ent_w, (short)0, (ne > 0 ? ne : 1) * GB, kRsrcWord3);
    const int rlast = ne > 0 ? ne - 1 : 0;
    int lg = 0;  // next group to load
    // Slot d of the ring holds group sg[d] and is only ever the direct target
    // of its own load (no register copies, no waits beyond the oldest load).
    // The flat loop (FP32) consumes the slots strictly in turn and reloads
    // each once consumed; the stage-by-stage loop (16-bit) reloads every slot
    // on every pass, a slot that was not consumed re-reading its group (a
    // conditional reload would make the compiler wait for the whole ring).
    auto take = [&]() -> int {
        const int g = lg < ne ? lg : rlast;
        ++lg;
        return g;
    };
    constexpr bool kFlat = FMT == XCT_F32 || FMT == XCT_F64;
    Group<FMT> e[D];
    int sg[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        sg[d] = take();
        e[d] = load_group<FMT>(rs, sg[d], lane);
    }

    // Copy of one stage into LDS.  Vector c (16 bytes) of a stage that starts
    // at tile-list position q0 comes from tile tile_list[q0 + c / kVecPerTile]
    // and goes to the placed row of its slot (rows of 16 bytes or more are
    // placed plainly, so whole tiles land contiguously).
    auto copy_static = [&](int q0, int nt) {
        if constexpr (POISON) {
            // debug build option: every byte of the stage buffer NaN (all-ones
            // is a NaN in each value format) before the stage lands, so that
            // an entry reading a slot this stage did not stage yields NaN
            for (int i = tid; i < a.T * kVecPerTile; i += nthr)
                ((u32x4 *)smem)[i] = u32x4{~0u, ~0u, ~0u, ~0u};
            __syncthreads();  // the fill is in LDS before any copy writes
        }
        if constexpr (kDma) {
            // Rows placed plainly: a tile's rows are contiguous in LDS, so each
            // 1 KB piece (64 vectors) is copied straight into LDS with no
            // registers, the whole stage in flight at once.  Wave w copies
            // the consecutive pieces [c0, c1); their tiles' indices come four
            // at a time (the tile list is padded by 4 entries).
            constexpr int kPiece = kVecPerTile >= 64 ? kVecPerTile / 64 : 1;
            const int pieces = nt * kPiece, per = (pieces + P - 1) / P;
            const int c0 = min(pieces, wave * per), c1 = min(pieces, c0 + per);
            if (c0 < c1) {
                int base = c0 / kPiece;
                i32x4 tl = sload_x4(a.tile_list + q0 + base);
                for (int c = c0; c < c1; ++c) {
                    const int q = c / kPiece, part = c - q * kPiece;
                    if (q - base >= 4) {
                        base = q;
                        tl = sload_x4(a.tile_list + q0 + base);
                    }
                    const int j = q - base;
                    const int tile = j == 0 ? tl.x : j == 1 ? tl.y : j == 2 ? tl.z : tl.w;
                    __builtin_amdgcn_global_load_lds(
                        (const void *)(xin + (int64_t)tile * kVecPerTile + part * 64 + lane),
                        (__attribute__((address_space(3))) void *)(smem + (size_t)(q * kVecPerTile + part * 64) * 16),
                        16, 0, 0);
                }
            }
            __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): this wave's pieces are in LDS
        } else {
            for (int e2 = tid; e2 < nt * kVecPerTile; e2 += nthr) {
                const int q = e2 / kVecPerTile, r = e2 % kVecPerTile;
                const u32x4 v = xin[(int64_t)a.tile_list[q0 + q] * kVecPerTile + r];
                constexpr int per = 16 / R::RB;  // rows per 16-byte vector
                const uint32_t u[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int k = 0; k < per; ++k) {
                    const uint32_t slot = (uint32_t)(q * kTileSlots + r * per + k);
                    char *dst = smem + slot * R::RB;
                    if constexpr (R::RB == 8) {
                        *(u32x2 *)dst = u32x2{u[2 * k], u[2 * k + 1]};
                    } else if constexpr (R::RB == 4) {
                        *(uint32_t *)dst = u[k];
                    } else {
                        *(uint16_t *)dst = (uint16_t)((k & 1) ? (u[k >> 1] >> 16) : (u[k >> 1] & 0xffffu));
                    }
                }
            }
        }
    };

    if (s0 < s1) copy_static(t0, min(a.T, t1 - t0));
    __syncthreads();
    int ph = 0;  // ring slot holding the next group (stage-by-stage loop)

    // FP32 matrices consume the stream in one flat loop; 16-bit matrices,
    // whose groups carry fewer FMAs, stage by stage (measured: the flat loop
    // is 3% faster than the best stage-by-stage ring at FP32, 4% slower at
    // FP16).
    if constexpr (kFlat) {
        // The wave's stream is a sequence of slab segments (stage s, row tile
        // h) consumed in one flat loop: the ring's slots are used in turn and
        // each is reloaded only after being consumed, rounds running across
        // segment and stage boundaries (so no group is fetched twice); the
        // stage transition (barrier, copy, barrier) happens where the stream
        // crosses into the next stage.  Every wave makes every transition.
        int nh[RT];  // group counts of stage s's RT slabs (far fewer than 2^31)
        auto stage_counts = [&](int st) {
            const int64_t ps = p0 + (int64_t)(st - s0) * RT;
            if constexpr (kDma) {
                const i32x4 sb = sload_x4(a.slab + ps);  // two int64 bounds
                nh[0] = sb.z - sb.x;
                if constexpr (RT == 2) {
                    const i32x4 sb1 = sload_x4(a.slab + ps + 1);
                    nh[1] = sb1.z - sb1.x;
                }
            } else {
#pragma unroll
                for (int hh = 0; hh < RT; ++hh) nh[hh] = (int)(a.slab[ps + hh + 1] - a.slab[ps + hh]);
            }
        };
        int st = s0, h = 0, left = 0;
        // Move to the next segment with groups left, crossing stage boundaries;
        // false once the stream and every remaining transition are done.
        auto advance = [&]() -> bool {
            while (left == 0) {
                if (h + 1 < RT) {
                    ++h;
                    left = nh[h];
                    continue;
                }
                __builtin_amdgcn_s_setprio(0);
                if (st + 1 >= s1) return false;
                const int q0n = t0 + (st + 1 - s0) * a.T;
                const int ntn = min(a.T, t1 - q0n);
                __syncthreads();  // every wave is done with this stage's data
                copy_static(q0n, ntn);
                __syncthreads();  // next stage in place
                ++st;
                stage_counts(st);
                h = 0;
                left = nh[0];
            }
            return true;
        };
        if (s0 < s1) {
            stage_counts(st);
            left = nh[0];
            bool more = advance();
            while (more) {
                prio_for_remaining(left + (h + 1 < RT ? nh[RT - 1] : 0));
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    if (more) {
                        if (RT == 1 || h == 0) {
                            if constexpr (H16)
                                use_group_h16<F, KB>(e[d], cb, acc2[0]);
                            else
                                use_group<FMT, F, KB>(e[d], cb, acc[0]);
                        } else {
                            if constexpr (H16)
                                use_group_h16<F, KB>(e[d], cb, acc2[RT - 1]);
                            else
                                use_group<FMT, F, KB>(e[d], cb, acc[RT - 1]);
                        }
                        sg[d] = take();
                        e[d] = load_group<FMT>(rs, sg[d], lane);
                        --left;
                        more = advance();
                    }
                }
            }
        }
    } else {
        for (int s = s0; s < s1; ++s) {
            // group counts of this stage's RT slabs (a slab holds far fewer
            // than 2^31 groups)
            int nh[RT];
            {
                const int64_t ps = p0 + (int64_t)(s - s0) * RT;
                if constexpr (kDma) {
                    const i32x4 sb = sload_x4(a.slab + ps);  // two int64 bounds
                    nh[0] = sb.z - sb.x;
                    if constexpr (RT == 2) {
                        const i32x4 sb1 = sload_x4(a.slab + ps + 1);
                        nh[1] = sb1.z - sb1.x;
                    }
                } else {
#pragma unroll
                    for (int h = 0; h < RT; ++h) nh[h] = (int)(a.slab[ps + h + 1] - a.slab[ps + h]);
                }
            }
#pragma unroll
            for (int h = 0; h < RT; ++h) {
                const int n = nh[h];
                const int later = h + 1 < RT ? nh[RT - 1] : 0;  // groups of the stage after this slab
                // consume this slab's n groups, the first one in slot ph; every
                // consumed slot is refilled from the cursor, possibly with a
                // later slab's group
                for (int i = -ph; i < n; i += D) {
                    prio_for_remaining(n - i + later);
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        const int k = i + d;
                        if (k >= 0 && k < n) {
                            if constexpr (H16)
                                use_group_h16<F, KB>(e[d], cb, acc2[h]);
                            else
                                use_group<FMT, F, KB>(e[d], cb, acc[h]);
                            sg[d] = take();
                        }
                        e[d] = load_group<FMT>(rs, sg[d], lane);
                    }
                }
                ph = (ph + n) % D;
            }
            __builtin_amdgcn_s_setprio(0);

            if (s + 1 < s1) {
                const int q0n = t0 + (s + 1 - s0) * a.T;
                const int ntn = min(a.T, t1 - q0n);
                __syncthreads();  // every wave is done with this stage's data
                copy_static(q0n, ntn);
                __syncthreads();  // next stage in place
            }
        }
    }

    // Undo the chunk rotation: slice c*SPC + t of this lane's row is in
    // accumulator block j = (c - lane) mod CH.
    double sq[F];  // this lane's per-slice sum of squares over its RT rows
#pragma unroll
    for (int f = 0; f < F; ++f) sq[f] = 0.0;
#pragma unroll
    for (int h = 0; h < RT; ++h) {
        AT af[F];  // the row's sums in accumulator order
#pragma unroll
        for (int f = 0; f < F; ++f) {
            if constexpr (H16)
                af[f] = (float)((f & 1) ? acc2[h][f >> 1].y : acc2[h][f >> 1].x);
            else
                af[f] = acc[h][f];
        }
        AT y[F];
#pragma unroll
        for (int c = 0; c < R::CH; ++c) {
#pragma unroll
            for (int t = 0; t < R::SPC; ++t) {
                AT v = af[t];
#pragma unroll
                for (int j = 1; j < R::CH; ++j) v = (coff[j] == c * 16) ? af[j * R::SPC + t] : v;
                y[c * R::SPC + t] = v;
            }
        }
        if (a.scale) {
#pragma unroll
            for (int f = 0; f < F; ++f) y[f] *= a.scale[f];
        }
        const int64_t rt = (int64_t)b * W + h * P + wave;
        bool natural = false;  // (16-bit matrices only: see spmm_call_f)
        if constexpr (FMT == XCT_F16 || FMT == XCT_BF16) natural = a.nat != nullptr;
        if (natural) {
            // the natural output directly (no conversion pass): each of the
            // F planes gets this wavefront's 8 x 8 tile as 8 runs of 8
            if (rt < a.n_row_tiles) {
                const int coord = a.row_coord[rt];
                const int o = lane_slot(lane, a.lanes);
                const int row = (coord / a.rowTW) * kTile + (o >> 3), col = (coord % a.rowTW) * kTile + (o & 7);
                if (row < a.H && col < a.Wd) {
                    const int64_t pix = (int64_t)row * a.Wd + col;
#pragma unroll
                    for (int f = 0; f < F; ++f) {
                        const int sl = a.s0 + f;
                        const int64_t i = (int64_t)sl * a.plane + pix;
                        if (sl < a.batch) store_io(a.nat, i, a.sub ? (float)y[f] - a.sub[i] : (float)y[f], a.io);
                    }
                }
            }
        } else if (rt < a.n_row_tiles) {
            AT *out = (AT *)a.yout + (rt * kTileSlots + lane_slot(lane, a.lanes)) * F;
            if constexpr (FMT == XCT_F64 && F >= 2) {
#pragma unroll
                for (int q = 0; q < F / 2; ++q) ((f64x2 *)out)[q] = f64x2{y[2 * q], y[2 * q + 1]};
            } else if constexpr (FMT != XCT_F64 && F >= 4) {
#pragma unroll
                for (int q = 0; q < F / 4; ++q)
                    ((f32x4 *)out)[q] = f32x4{y[4 * q], y[4 * q + 1], y[4 * q + 2], y[4 * q + 3]};
            } else {
#pragma unroll
                for (int f = 0; f < F; ++f) out[f] = y[f];
            }
        }
#pragma unroll
        for (int f = 0; f < F; ++f) sq[f] += (double)y[f] * (double)y[f];
    }
    if (a.sq_partial) {
        // per-slice sum of squares of this block's outputs, in FP64, fixed order
        __syncthreads();
        double *red = (double *)smem;  // [P][F]
#pragma unroll
        for (int f = 0; f < F; ++f) {
            double q = sq[f];
            for (int o = 32; o > 0; o >>= 1) q += __shfl_xor(q, o, 64);
            if (lane == 0) red[wave * F + f] = q;
        }
        __syncthreads();
        if (tid < F) {
            double q = 0.0;
            for (int w = 0; w < P; ++w) q += red[w * F + tid];
            a.sq_partial[(int64_t)b * F + tid] = q;
        }
    }
}

// ---- kernel timing for measurement tools -----------------------------------

// Blocks per XCD run for the launch (see k_spmm): option -1 plain order; 1
// one contiguous run of the Hilbert order per XCD; n >= 2 runs of n blocks;
// 0 (default) runs of 4.  Measured (projection + backprojection step):
// contiguous runs keep an XCD's blocks far from the other XCDs', so the
// eight staged regions overflow the memory-side cache once a pass stages
// more than ~128 MB (64 x 2048^2 FP16: 56.8 ms, 128 x 2816^2 FP16: 333 ms);
// runs of 4 keep the XCDs in one region (52.6 ms, 287 ms; plain order 53.5,
// 293 ms) and match contiguous runs where the input fits (16 x 1024^2:
// 4.81 vs 4.82 ms FP32, 3.34 vs 3.38 ms FP16).
constexpr int kDefaultRun = 4;
static int remap_chunk(int opt, const OpPlan &op) {
    if (opt < 0) return 0;
    if (opt == 1) return (op.n_blocks + 7) / 8;
    return opt >= 2 ? opt : kDefaultRun;
}

struct ProfileRec {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[2];
};
static ProfileRec g_prof;

template <int FMT, int F, int RT, bool H16>
static int launch_one(const SpmmLaunch &L, hipStream_t st) {
    const OpPlan &op = *L.op;
    SpmmArgs a;
    a.blk_stage = op.blk_stage;
    a.blk_tile = op.blk_tile;
    a.tile_list = op.tile_list;
    a.slab = op.slab;
    a.slot = op.slot;
    a.val = op.val;
    a.packed = op.packed;
    a.xin = L.xin;
    a.yout = L.yout;
    a.scale = L.scale;
    a.sq_partial = L.sq_partial;
    a.n_row_tiles = op.n_row_tiles;
    a.n_blocks = op.n_blocks;
    a.T = op.T;

    a.lanes = op.lanes;
    a.W = op.W;
    a.nat = L.nat;
    a.sub = L.sub;
    a.row_coord = L.gout ? L.gout->coord_of : nullptr;
    a.plane = L.gout ? (int64_t)L.gout->H * L.gout->Wd : 0;
    a.H = L.gout ? L.gout->H : 0;
    a.Wd = L.gout ? L.gout->Wd : 0;
    a.rowTW = L.gout ? L.gout->TW : 0;
    a.io = L.io;
    a.batch = L.batch;
    a.s0 = L.s0;
    typedef typename Stor<FMT>::T XT;
    size_t smem = (size_t)op.T * kTileSlots * F * sizeof(XT);
    const size_t red = sizeof(double) * (size_t)op.W * F;
    if (smem < red) smem = red;
    // the debug build option (NaN-filled stage buffers) has its own instantiation
    const void *kern = op.poison ? (const void *)k_spmm<FMT, F, RT, H16, true>
                                 : (const void *)k_spmm<FMT, F, RT, H16, false>;
    static int attr_bytes[2] = {0, 0};  // per instantiation: largest dynamic LDS size enabled so far
    if ((int)smem > attr_bytes[op.poison]) {
        XCT_HIP_TRY(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem));
        attr_bytes[op.poison] = (int)smem;
    }
    a.remap = remap_chunk(L.remap, op);
    const int grid = a.remap ? 8 * a.remap * ((op.n_blocks + 8 * a.remap - 1) / (8 * a.remap)) : op.n_blocks;
    if (grid == 0) return XCT_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (g_prof.on) {
        XCT_HIP_TRY(hipEventCreate(&e0));
        XCT_HIP_TRY(hipEventCreate(&e1));
        XCT_HIP_TRY(hipEventRecord(e0, st));
    }
    if (op.poison)
        hipLaunchKernelGGL((k_spmm<FMT, F, RT, H16, true>), dim3(grid), dim3(op.W / RT * kTileSlots), smem, st, a);
    else
        hipLaunchKernelGGL((k_spmm<FMT, F, RT, H16, false>), dim3(grid), dim3(op.W / RT * kTileSlots), smem, st, a);
    XCT_HIP_TRY(hipGetLastError());
    if (g_prof.on) {
        XCT_HIP_TRY(hipEventRecord(e1, st));
        g_prof.ev[op.which & 1].push_back({e0, e1});
    }
    return XCT_OK;
}

// FP16 arithmetic where the operator asks for it (FP16 matrices, F >= 2;
// a single fused slice keeps FP32 arithmetic).
template <int FMT, int F, int RT>
static int launch_arith(const SpmmLaunch &L, hipStream_t st) {
    if constexpr (FMT == XCT_F16 && F >= 2) {
        if (L.op->arith16) return launch_one<FMT, F, RT, true>(L, st);
    }
    return launch_one<FMT, F, RT, false>(L, st);
}

template <int FMT, int RT>
static int launch_rt(const SpmmLaunch &L, hipStream_t st) {
    switch (L.F) {
        case 1: return launch_arith<FMT, 1, RT>(L, st);
        case 2: return launch_arith<FMT, 2, RT>(L, st);
        case 4: return launch_arith<FMT, 4, RT>(L, st);
        case 8: return launch_arith<FMT, 8, RT>(L, st);
        case 16:
            // FP64 rows of 16 slices would be 128 bytes: FP64 fuses at most 8
            if constexpr (FMT != XCT_F64) return launch_arith<FMT, 16, RT>(L, st);
            return fail(XCT_ERR_UNSUPPORTED, "FP64 matrices fuse at most 8 slices");
        case 32:
            // 32 fused slices: 16-bit operands only (64-byte staged rows, as
            // FP32 at 16) and one row tile per wavefront (32 accumulators)
            if constexpr ((FMT == XCT_F16 || FMT == XCT_BF16) && RT == 1) return launch_arith<FMT, 32, RT>(L, st);
            return fail(XCT_ERR_UNSUPPORTED, "32 fused slices need a 16-bit matrix and one row tile per wavefront");
        default: return fail(XCT_ERR_INVALID, "unsupported fused slice count");
    }
}

template <int FMT>
static int launch_fmt(const SpmmLaunch &L, hipStream_t st) {
    switch (L.op->R) {
        case 1: return launch_rt<FMT, 1>(L, st);
        case 2: return launch_rt<FMT, 2>(L, st);
        default: return fail(XCT_ERR_INTERNAL, "unsupported row tiles per wavefront");
    }
}

int launch_spmm(const SpmmLaunch &L, hipStream_t st) {
    switch (L.vdt) {
        case XCT_F32: return launch_fmt<XCT_F32>(L, st);
        case XCT_F16: return launch_fmt<XCT_F16>(L, st);
        case XCT_BF16: return launch_fmt<XCT_BF16>(L, st);
        case XCT_F64: return launch_fmt<XCT_F64>(L, st);
        default: return fail(XCT_ERR_INVALID, "bad value dtype");
    }
}

// ---- layout conversions -----------------------------------------------------

struct ConvArgs {
    const int32_t *rank_of;  // raster tile -> Hilbert rank
    int H, Wd, TH, TW;
    int strips;  // runs of kConvTiles tiles per tile row
    int batch, s0, F;
    int io, storage;
    const float *sub;  // from_internal: natural-layout FP32 values to subtract, or null
};

// Natural [B][H][Wd] <-> internal [tile][64][F].  One thread per slot: the F
// loads (or stores) of the natural side are issued together.  A
// workgroup of 256 threads takes kConvTiles = 4 horizontally adjacent tiles
// (8 rows x 32 columns), each wavefront two of its rows, so that a natural
// access of a wavefront is two whole 128-byte row pieces and its internal
// rows are four runs of 16 consecutive slots (1 KB each at 16 FP32 slices).
constexpr int kConvTiles = 4;
__device__ __forceinline__ bool conv_slot(const ConvArgs &c, int64_t &t, int &row, int &col) {
    const int b = blockIdx.x;
    const int ty = b / c.strips, sx = b - ty * c.strips;
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = 2 * w + (l >> 5), cs = l & 31;
    const int tx = sx * kConvTiles + (cs >> 3), cc = cs & 7;
    if (ty >= c.TH || tx >= c.TW) return false;
    t = (int64_t)c.rank_of[ty * c.TW + tx] * kTileSlots + r * kTile + cc;
    row = ty * kTile + r;
    col = tx * kTile + cc;
    return true;
}
// Rows of 16 bytes or more go through LDS: each thread puts its row there,
// then the workgroup writes (or, the other way, reads) the internal rows of
// its tiles as consecutive 16-byte pieces, every wavefront access one
// contiguous run.  Row r of the workgroup's LDS rows (stride RB + 16 bytes)
// belongs to thread r; conv_src gives the thread holding slot o of tile
// tile of the workgroup.
__device__ __forceinline__ int conv_src(int tile, int o) {
    const int r = o >> 3;
    return (r >> 1) * 64 + ((r & 1) << 5) + (tile << 3) + (o & 7);
}
inline size_t conv_lds_bytes(int row_bytes) { return row_bytes >= 16 ? (size_t)256 * (row_bytes + 16) : 0; }

template <int F>
__global__ void k_to_internal(ConvArgs c, const void *nat, void *internal, const float *inv) {
    int64_t t = 0;
    int row = 0, col = 0;
    const bool valid = conv_slot(c, t, row, col);
    const bool in = valid && row < c.H && col < c.Wd;
    const int64_t plane = (int64_t)c.H * c.Wd;
    const int64_t pix = (int64_t)row * c.Wd + col;
    float v[F];
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const int s = c.s0 + f;
        v[f] = (in && s < c.batch) ? load_io(nat, (int64_t)s * plane + pix, c.io) : 0.f;
    }
    if (inv) {
#pragma unroll
        for (int f = 0; f < F; ++f) v[f] *= inv[f];
    }
    const bool f32 = c.storage == XCT_F32;
    // the row as 32-bit words (FP32 values or pairs of 16-bit ones)
    constexpr int NW = F;  // enough for either form
    uint32_t wd[NW];
    int nw;
    if (f32) {
#pragma unroll
        for (int f = 0; f < F; ++f) wd[f] = __float_as_uint(v[f]);
        nw = F;
    } else {
        uint16_t h[F];
#pragma unroll
        for (int f = 0; f < F; ++f) h[f] = (uint16_t)(c.storage == XCT_F16 ? f32_to_h16(v[f]) : f32_to_bf16(v[f]));
#pragma unroll
        for (int f = 0; f < F; f += 2) wd[f / 2] = h[f] | (F > 1 ? ((uint32_t)h[f + 1 < F ? f + 1 : f] << 16) : 0u);
        nw = (F + 1) / 2;
    }
    const int RB = f32 ? F * 4 : F * 2;
    if (RB < 16) {  // narrow rows: written directly
        if (!valid) return;
        if (f32) {
            float *dst = (float *)internal + t * F;
#pragma unroll
            for (int f = 0; f < F; ++f) dst[f] = v[f];
        } else {
            uint16_t *dst = (uint16_t *)internal + t * F;
#pragma unroll
            for (int f = 0; f < F; ++f) dst[f] = (uint16_t)((f & 1) ? (wd[f / 2] >> 16) : (wd[f / 2] & 0xffffu));
        }
        return;
    }
    extern __shared__ __align__(16) char cbuf[];
    const int RBp = RB + 16;
    {
        char *mine = cbuf + (size_t)threadIdx.x * RBp;
#pragma unroll
        for (int q = 0; q < NW / 4; ++q)
            if (4 * q < nw) *(u32x4 *)(mine + 16 * q) = u32x4{wd[4 * q], wd[4 * q + 1], wd[4 * q + 2], wd[4 * q + 3]};
    }
    __syncthreads();
    const int cpr = RB / 16, per_tile = kTileSlots * cpr;
    const int ty = blockIdx.x / c.strips, sx = blockIdx.x - ty * c.strips;
    for (int k = threadIdx.x; k < kConvTiles * per_tile; k += blockDim.x) {
        const int tile = k / per_tile, rem = k - tile * per_tile, o = rem / cpr, q = rem - o * cpr;
        const int tx = sx * kConvTiles + tile;
        if (tx >= c.TW) continue;
        const u32x4 w = *(const u32x4 *)(cbuf + (size_t)conv_src(tile, o) * RBp + 16 * q);
        const int64_t rank = c.rank_of[ty * c.TW + tx];
        *(u32x4 *)((char *)internal + (rank * kTileSlots + o) * RB + 16 * q) = w;
    }
}

// FP64 matrices: the same conversions with FP64 rows (any io dtype; FP64 io
// keeps every bit, narrower io is rounded once, nearest-even).
__device__ __forceinline__ double load_io64(const void *p, int64_t i, int io) {
    if (io == XCT_F64) return ((const double *)p)[i];
    return (double)load_io(p, i, io);
}

__device__ __forceinline__ void store_io64(void *p, int64_t i, double v, int io) {
    if (io == XCT_F64)
        ((double *)p)[i] = v;
    else
        store_io(p, i, (float)v, io);
}

template <int F>
__global__ void k_to_internal64(ConvArgs c, const void *nat, double *internal) {
    int64_t t;
    int row, col;
    if (!conv_slot(c, t, row, col)) return;
    const bool in = row < c.H && col < c.Wd;
    const int64_t plane = (int64_t)c.H * c.Wd;
    const int64_t pix = (int64_t)row * c.Wd + col;
    double v[F];
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const int s = c.s0 + f;
        v[f] = (in && s < c.batch) ? load_io64(nat, (int64_t)s * plane + pix, c.io) : 0.0;
    }
    double *dst = internal + t * F;
    if constexpr (F >= 2) {
#pragma unroll
        for (int q = 0; q < F / 2; ++q) ((f64x2 *)dst)[q] = f64x2{v[2 * q], v[2 * q + 1]};
    } else {
        dst[0] = v[0];
    }
}

template <int F>
__global__ void k_from_internal64(ConvArgs c, const double *internal, void *nat) {
    int64_t t;
    int row, col;
    if (!conv_slot(c, t, row, col)) return;
    if (row >= c.H || col >= c.Wd) return;
    const int64_t plane = (int64_t)c.H * c.Wd;
    const int64_t pix = (int64_t)row * c.Wd + col;
    double v[F];
    const double *src = internal + t * F;
    if constexpr (F >= 2) {
#pragma unroll
        for (int q = 0; q < F / 2; ++q) {
            const f64x2 w = ((const f64x2 *)src)[q];
            v[2 * q] = w.x;
            v[2 * q + 1] = w.y;
        }
    } else {
        v[0] = src[0];
    }
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const int s = c.s0 + f;
        if (s < c.batch) store_io64(nat, (int64_t)s * plane + pix, v[f], c.io);
    }
}

template <int F>
__global__ void k_from_internal(ConvArgs c, const float *internal, void *nat) {
    int64_t t = 0;
    int row = 0, col = 0;
    const bool valid = conv_slot(c, t, row, col);
    float v[F];
    constexpr int RB = F * 4;
    if constexpr (RB >= 16) {
        // the workgroup's internal rows into LDS as consecutive 16-byte
        // pieces, then each thread takes its own row
        extern __shared__ __align__(16) char cbuf[];
        constexpr int RBp = RB + 16, cpr = RB / 16, per_tile = kTileSlots * cpr;
        const int ty = blockIdx.x / c.strips, sx = blockIdx.x - ty * c.strips;
        for (int k = threadIdx.x; k < kConvTiles * per_tile; k += blockDim.x) {
            const int tile = k / per_tile, rem = k - tile * per_tile, o = rem / cpr, q = rem - o * cpr;
            const int tx = sx * kConvTiles + tile;
            if (tx >= c.TW) continue;
            const int64_t rank = c.rank_of[ty * c.TW + tx];
            *(u32x4 *)(cbuf + (size_t)conv_src(tile, o) * RBp + 16 * q) =
                *(const u32x4 *)((const char *)internal + (rank * kTileSlots + o) * RB + 16 * q);
        }
        __syncthreads();
        if (!valid) return;
        const char *mine = cbuf + (size_t)threadIdx.x * RBp;
#pragma unroll
        for (int q = 0; q < F / 4; ++q) {
            const u32x4 w = *(const u32x4 *)(mine + 16 * q);
            v[4 * q] = __uint_as_float(w.x);
            v[4 * q + 1] = __uint_as_float(w.y);
            v[4 * q + 2] = __uint_as_float(w.z);
            v[4 * q + 3] = __uint_as_float(w.w);
        }
    } else {
        if (!valid) return;
        const float *src = internal + t * F;
#pragma unroll
        for (int f = 0; f < F; ++f) v[f] = src[f];
    }
    if (row >= c.H || col >= c.Wd) return;
    const int64_t plane = (int64_t)c.H * c.Wd;
    const int64_t pix = (int64_t)row * c.Wd + col;
#pragma unroll
    for (int f = 0; f < F; ++f) {
        const int s = c.s0 + f;
        const int64_t i = (int64_t)s * plane + pix;
        if (s < c.batch) store_io(nat, i, c.sub ? v[f] - c.sub[i] : v[f], c.io);
    }
}

// Per-slice max |v| over the natural layout of one fused group (grid.y =
// slice of the group).  FP32 planes whose length is a multiple of 4 (in a
// 16-byte aligned array) are read as 16-byte vectors, several per thread.
__global__ void k_absmax(const void *nat, int io, int64_t plane, int batch, int s0, int F, uint32_t *amax) {
    const int f = blockIdx.y;
    const int s = s0 + f;
    if (s >= batch) return;
    float m = 0.f;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (io == XCT_F32 && (plane & 3) == 0 && ((uintptr_t)nat & 15) == 0) {
        const f32x4 *p = (const f32x4 *)((const float *)nat + (int64_t)s * plane);
        const int64_t n4 = plane / 4;
        auto vmax = [](f32x4 v) { return fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))); };
        int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
        for (; i + 3 * stride < n4; i += 4 * stride) {  // four loads in flight
            const f32x4 v0 = p[i], v1 = p[i + stride], v2 = p[i + 2 * stride], v3 = p[i + 3 * stride];
            m = fmaxf(m, fmaxf(fmaxf(vmax(v0), vmax(v1)), fmaxf(vmax(v2), vmax(v3))));
        }
        for (; i < n4; i += stride) m = fmaxf(m, vmax(p[i]));
    } else {
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < plane; i += stride)
            m = fmaxf(m, fabsf(load_io(nat, (int64_t)s * plane + i, io)));
    }
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    __shared__ float wm[16];
    if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = fmaxf(m, wm[w]);
        atomicMax(&amax[f], __float_as_uint(m));  // non-negative floats order like their bits
    }
}

// Clear the per-slice maxima before the first group (a kernel, not a memset
// node, so that a caller may capture the call into a graph).
__global__ void k_clear_amax(uint32_t *amax, int n) {
    if ((int)threadIdx.x < n) amax[threadIdx.x] = 0u;
}

// m = 2^ceil(log2 max) (1 for a zero or non-finite max), scale = m, inv = 1/m.
// amax is cleared after it is read so the next group can reuse it.
__global__ void k_pow2_scale(uint32_t *amax, int F, float *scale, float *inv) {
    const int f = threadIdx.x;
    if (f >= F) return;
    const float m = pow2_at_least(__uint_as_float(amax[f]));
    amax[f] = 0u;
    scale[f] = m;
    inv[f] = 1.f / m;  // exact: m is a power of two
}

static ConvArgs conv_args(const Grid &g, int batch, int s0, int F, int io, int storage) {
    ConvArgs c;
    c.rank_of = g.rank_of;
    c.H = g.H;
    c.Wd = g.Wd;
    c.TH = g.TH;
    c.TW = g.TW;
    c.strips = (g.TW + kConvTiles - 1) / kConvTiles;
    c.batch = batch;
    c.s0 = s0;
    c.F = F;
    c.io = io;
    c.storage = storage;
    c.sub = nullptr;
    return c;
}

int launch_to_internal(const Grid &g, const void *nat, xct_dtype io, int batch, int s0, int F, void *internal,
                       xct_dtype storage, const float *inv_scale, hipStream_t st) {
    const ConvArgs c = conv_args(g, batch, s0, F, io, storage);
    const dim3 grid((unsigned)((int64_t)g.TH * c.strips)), blk(256);
    if (storage == XCT_F64) {
        double *d = (double *)internal;
        switch (F) {
            case 1: hipLaunchKernelGGL(k_to_internal64<1>, grid, blk, 0, st, c, nat, d); break;
            case 2: hipLaunchKernelGGL(k_to_internal64<2>, grid, blk, 0, st, c, nat, d); break;
            case 4: hipLaunchKernelGGL(k_to_internal64<4>, grid, blk, 0, st, c, nat, d); break;
            case 8: hipLaunchKernelGGL(k_to_internal64<8>, grid, blk, 0, st, c, nat, d); break;
            default: return fail(XCT_ERR_INVALID, "unsupported fused slice count for FP64");
        }
        XCT_HIP_TRY(hipGetLastError());
        return XCT_OK;
    }
    const size_t sm = conv_lds_bytes(F * (storage == XCT_F32 ? 4 : 2));
    switch (F) {
        case 1: hipLaunchKernelGGL(k_to_internal<1>, grid, blk, sm, st, c, nat, internal, inv_scale); break;
        case 2: hipLaunchKernelGGL(k_to_internal<2>, grid, blk, sm, st, c, nat, internal, inv_scale); break;
        case 4: hipLaunchKernelGGL(k_to_internal<4>, grid, blk, sm, st, c, nat, internal, inv_scale); break;
        case 8: hipLaunchKernelGGL(k_to_internal<8>, grid, blk, sm, st, c, nat, internal, inv_scale); break;
        case 16: hipLaunchKernelGGL(k_to_internal<16>, grid, blk, sm, st, c, nat, internal, inv_scale); break;
        case 32: hipLaunchKernelGGL(k_to_internal<32>, grid, blk, sm, st, c, nat, internal, inv_scale); break;
        default: return fail(XCT_ERR_INVALID, "unsupported fused slice count");
    }
    XCT_HIP_TRY(hipGetLastError());
    return XCT_OK;
}

// FP64 sums (FP64 matrices) to the natural layout
int launch_from_internal64(const Grid &g, const double *internal, int batch, int s0, int F, void *nat, xct_dtype io,
                           hipStream_t st) {
    const ConvArgs c = conv_args(g, batch, s0, F, io, XCT_F64);
    const dim3 grid((unsigned)((int64_t)g.TH * c.strips)), blk(256);
    switch (F) {
        case 1: hipLaunchKernelGGL(k_from_internal64<1>, grid, blk, 0, st, c, internal, nat); break;
        case 2: hipLaunchKernelGGL(k_from_internal64<2>, grid, blk, 0, st, c, internal, nat); break;
        case 4: hipLaunchKernelGGL(k_from_internal64<4>, grid, blk, 0, st, c, internal, nat); break;
        case 8: hipLaunchKernelGGL(k_from_internal64<8>, grid, blk, 0, st, c, internal, nat); break;
        default: return fail(XCT_ERR_INVALID, "unsupported fused slice count for FP64");
    }
    XCT_HIP_TRY(hipGetLastError());
    return XCT_OK;
}

int launch_from_internal(const Grid &g, const float *internal, int batch, int s0, int F, void *nat, xct_dtype io,
                         hipStream_t st, const float *sub) {
    ConvArgs c = conv_args(g, batch, s0, F, io, XCT_F32);
    c.sub = sub;
    const dim3 grid((unsigned)((int64_t)g.TH * c.strips)), blk(256);
    const size_t sm = conv_lds_bytes(F * 4);
    switch (F) {
        case 1: hipLaunchKernelGGL(k_from_internal<1>, grid, blk, sm, st, c, internal, nat); break;
        case 2: hipLaunchKernelGGL(k_from_internal<2>, grid, blk, sm, st, c, internal, nat); break;
        case 4: hipLaunchKernelGGL(k_from_internal<4>, grid, blk, sm, st, c, internal, nat); break;
        case 8: hipLaunchKernelGGL(k_from_internal<8>, grid, blk, sm, st, c, internal, nat); break;
        case 16: hipLaunchKernelGGL(k_from_internal<16>, grid, blk, sm, st, c, internal, nat); break;
        case 32: hipLaunchKernelGGL(k_from_internal<32>, grid, blk, sm, st, c, internal, nat); break;
        default: return fail(XCT_ERR_INVALID, "unsupported fused slice count");
    }
    XCT_HIP_TRY(hipGetLastError());
    return XCT_OK;
}

int launch_pow2_scale(uint32_t *amax, int F, float *scale, float *inv, hipStream_t st) {
    hipLaunchKernelGGL(k_pow2_scale, dim3(1), dim3(64), 0, st, amax, F, scale, inv);
    XCT_HIP_TRY(hipGetLastError());
    return XCT_OK;
}

int launch_natural_scale(const Grid &g, const void *nat, xct_dtype io, int batch, int s0, int F, uint32_t *amax,
                         float *scale, float *inv, hipStream_t st) {
    const int64_t plane = (int64_t)g.H * g.Wd;
    // 256 threads a workgroup, about 8 vectors (or 32 elements) a thread, at
    // most 128 workgroups a slice
    int blocks = (int)std::min<int64_t>(128, (plane + 256 * 32 - 1) / (256 * 32));
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_absmax, dim3(blocks, F), dim3(256), 0, st, nat, (int)io, plane, batch, s0, F, amax);
    XCT_HIP_TRY(hipGetLastError());
    return launch_pow2_scale(amax, F, scale, inv, st);
}

// ---- boundary entry points ---------------------------------------------------

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct SpmmWs {
    void *in;
    void *out;  // FP32 sums, FP64 for FP64 matrices
    uint32_t *amax;
    float *scale, *inv;
};

// Workspace of one fused group of F slices: the staged operand in the
// storage dtype, the FP32 sums, and the per-slice max, scale and inverse.
static size_t spmm_ws_layout_f(const xct_matrix *m, int F, char *base, SpmmWs *w) {
    const int64_t tiles = std::max(m->vol.n_tiles, m->sino.n_tiles);
    const size_t in_b = align256((size_t)tiles * kTileSlots * F * elem_bytes(m->vdt));
    const size_t out_b = align256((size_t)tiles * kTileSlots * F * (m->vdt == XCT_F64 ? sizeof(double) : sizeof(float)));
    const size_t small = align256(sizeof(uint32_t) * kMaxFuse) * 3;
    if (w) {
        w->in = base;
        w->out = base + in_b;
        char *p = base + in_b + out_b;
        w->amax = (uint32_t *)p;
        w->scale = (float *)(p + align256(sizeof(uint32_t) * kMaxFuse));
        w->inv = (float *)(p + 2 * align256(sizeof(uint32_t) * kMaxFuse));
    }
    return in_b + out_b + small;
}

static size_t spmm_ws_layout(const xct_matrix *m, int batch, char *base, SpmmWs *w) {
    return spmm_ws_layout_f(m, run_fuse(batch, m->fuse), base, w);
}

// The product of spmm_call with F slices fused per matrix pass (any power of
// two up to the matrix's fuse: the plan's stages fit the LDS at any smaller
// F) and a workspace of spmm_ws_layout_f(m, F) bytes.
static int spmm_call_f(const xct_matrix *m, int dir, const void *src, void *dst, int batch, xct_dtype io,
                       void *workspace, int F, hipStream_t st, const float *sub = nullptr) {
    const OpPlan &op = dir ? m->AT : m->A;
    const Grid &gin = dir ? m->sino : m->vol;
    const Grid &gout = dir ? m->vol : m->sino;
    SpmmWs w;
    spmm_ws_layout_f(m, F, (char *)workspace, &w);
    const bool norm = m->vdt == XCT_F16 || m->vdt == XCT_BF16;
    if (norm) {
        hipLaunchKernelGGL(k_clear_amax, dim3(1), dim3(64), 0, st, w.amax, kMaxFuse);
        XCT_HIP_TRY(hipGetLastError());
    }
    for (int s0 = 0; s0 < batch; s0 += F) {
        int rc;
        if (norm) {
            rc = launch_natural_scale(gin, src, io, batch, s0, F, w.amax, w.scale, w.inv, st);
            if (rc) return rc;
        }
        rc = launch_to_internal(gin, src, io, batch, s0, F, w.in, m->vdt, norm ? w.inv : nullptr, st);
        if (rc) return rc;
        SpmmLaunch L{&op, w.in, w.out, norm ? w.scale : nullptr, nullptr, F, m->vdt, m->remap};
        if (norm) {
            // 16-bit matrices: the sums go straight to the natural output.
            // (Measured at 16 x 1024^2 x 1500: the FP16 step 2% shorter with
            // unchanged launches; the FP32 kernel's launches grew 1.2% from
            // the scattered 32-byte output runs at every block's end, for
            // 0.4% on the step, so FP32 sums keep the conversion pass.)
            L.nat = dst;
            L.sub = sub;
            L.gout = &gout;
            L.io = io;
            L.batch = batch;
            L.s0 = s0;
        }
        rc = launch_spmm(L, st);
        if (rc) return rc;
        if (!norm) {
            rc = m->vdt == XCT_F64 ? launch_from_internal64(gout, (const double *)w.out, batch, s0, F, dst, io, st)
                                   : launch_from_internal(gout, (const float *)w.out, batch, s0, F, dst, io, st, sub);
            if (rc) return rc;
        }
    }
    return XCT_OK;
}

int spmm_call(const xct_matrix *m, int dir, const void *src, void *dst, int batch, xct_dtype io,
                     void *workspace, void *stream) {
    if (!m || !src || !dst || !workspace) return fail(XCT_ERR_INVALID, "NULL argument");
    if (batch < 1) return fail(XCT_ERR_INVALID, "batch must be >= 1");
    if (!valid_dtype(io)) return fail(XCT_ERR_INVALID, "bad io dtype");
    if (((uintptr_t)workspace & 255) != 0) return fail(XCT_ERR_INVALID, "workspace must be 256-byte aligned");
    return spmm_call_f(m, dir, src, dst, batch, io, workspace, run_fuse(batch, m->fuse), (hipStream_t)stream);
}

int spmm_residual(const xct_matrix *m, const float *x, const float *y, float *r, int batch, void *workspace,
                  hipStream_t st) {
    if (m->vdt == XCT_F64) return fail(XCT_ERR_INTERNAL, "the fused residual takes FP32 or 16-bit matrices");
    return spmm_call_f(m, 0, x, r, batch, XCT_F32, workspace, run_fuse(batch, m->fuse), st, y);
}

// ---- the allocation-free form of the products --------------------------------
//
// For callers that cannot allocate device memory (graph capture, serving
// loops): the staging workspace is a fixed array of device memory that the
// code object carries, one copy per GPU, held until the process ends.  Its
// device address is looked up once per device (a host-side reference to the
// array names no device memory).  Every call on a GPU uses that GPU's one
// array: calls that overlap on one GPU race, whatever their streams.  The
// array's leftovers from an earlier call are harmless: the conversion writes
// every staged element and the product every sum before they are read, and
// the per-slice maxima are cleared first.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static void *g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

static int scratch_for_current_device(void **out) {
    int dev = -1;
    XCT_HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(XCT_ERR_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        XCT_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(XCT_ERR_HIP, "no device address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return XCT_OK;
}

size_t spmm_workspace(const xct_matrix *m, int batch) { return spmm_ws_layout(m, batch, nullptr, nullptr); }

}  // namespace xct

using namespace xct;

extern "C" size_t xct_spmm_workspace_bytes(const xct_matrix *m, int batch) {
    if (!m || batch < 1) return 0;
    return spmm_workspace(m, batch);
}

extern "C" int xct_project(const xct_matrix *m, const void *x, void *y, int batch, xct_dtype io, void *workspace,
                           void *stream) {
    return spmm_call(m, 0, x, y, batch, io, workspace, stream);
}

extern "C" int xct_backproject(const xct_matrix *m, const void *y, void *x, int batch, xct_dtype io, void *workspace,
                               void *stream) {
    return spmm_call(m, 1, y, x, batch, io, workspace, stream);
}

extern "C" size_t xct_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int xct_apply_noalloc(const xct_matrix *m, int which, const void *in, void *out, int batch,
                                 xct_dtype io, void *stream) {
    if (!m || !in || !out) return fail(XCT_ERR_INVALID, "NULL argument");
    if (which != 0 && which != 1) return fail(XCT_ERR_INVALID, "which must be 0 (A x) or 1 (A^T y)");
    if (batch < 1) return fail(XCT_ERR_INVALID, "batch must be >= 1");
    if (!valid_dtype(io)) return fail(XCT_ERR_INVALID, "bad io dtype");
    // the most slices per matrix pass whose staging fits the array
    int F = run_fuse(batch, m->fuse);
    while (F > 1 && spmm_ws_layout_f(m, F, nullptr, nullptr) > kScratchBytes) F >>= 1;
    const size_t need = spmm_ws_layout_f(m, F, nullptr, nullptr);
    if (need > kScratchBytes)
        return fail(XCT_ERR_UNSUPPORTED, "one slice of this geometry needs " + std::to_string(need) +
                                             " bytes of staging, beyond the " + std::to_string(kScratchBytes) +
                                             "-byte allocation-free scratch; use xct_project / xct_backproject "
                                             "with a workspace");
    void *ws = nullptr;
    int rc = scratch_for_current_device(&ws);
    if (rc) return rc;
    return spmm_call_f(m, which, in, out, batch, io, ws, F, (hipStream_t)stream);
}

extern "C" int xct_profile_enable(int on) {
    g_prof.on = on != 0;
    return XCT_OK;
}

extern "C" int xct_profile_read(int64_t *launches, double *ms) {
    if (!launches || !ms) return fail(XCT_ERR_INVALID, "NULL argument");
    int rc = XCT_OK;
    for (int w = 0; w < 2; ++w) {
        launches[w] = (int64_t)g_prof.ev[w].size();
        ms[w] = 0.0;
        for (auto &pr : g_prof.ev[w]) {
            float t = 0.f;
            hipError_t e = hipEventSynchronize(pr.second);
            if (e == hipSuccess) e = hipEventElapsedTime(&t, pr.first, pr.second);
            if (e != hipSuccess && rc == XCT_OK)
                rc = fail(XCT_ERR_HIP, std::string("profile events: ") + hipGetErrorString(e));
            ms[w] += t;
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        g_prof.ev[w].clear();
    }
    return rc;
}
