// GPU construction of the staged-ELL forms of A and A^T.
//
// The paper memoises the Siddon matrix once (Sec. II-B) and reorders both
// the tomogram and the sinogram by pseudo-Hilbert tiles (Sec. III-A.1,
// Fig. 3): row tiles in Hilbert order are grouped into thread blocks, and
// the input footprint of a block is staged through on-chip memory in
// rounds that each fit the buffer (Sec. III-B "multi-stage 3D buffering";
// the stage maps of Listing 1).  Here every block builds its own plan:
//   k_footprint  marks the input tiles its rows touch in an LDS bitmap
//                indexed by Hilbert rank, and counts them and the entries;
//   k_plan       writes the touched tiles in Hilbert order (the tile list),
//                cuts it into stages of T tiles and records, per stage and
//                wavefront, the longest lane's entry count (the ELL slab);
//   k_fill       writes every entry at its slab position as a 16-bit
//                stage-local slot plus the length, rounded to nearest-even
//                once from FP64 (Sec. III-C "data packing").
// The three kernels generate the entries of a row with the same code, so
// they see the same entry set; k_fill still checks every write against the
// slab bounds and reports a violation instead of writing past it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <numeric>
#include <unordered_map>
#include <type_traits>
#include <string>
#include <vector>

#include "common.hpp"
#include "geometry.hpp"

namespace xct {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

// ---- the library's device allocations ---------------------------------------
//
// Every device buffer the library takes goes through dev_alloc and dev_free,
// which keep the live buffers and their sizes (xct_device_memory reports
// them, for leak checks).  Failure injection for the tests of error paths:
// with XCT_FAULT_ALLOC=n in the environment, the n-th allocation counted
// from when the variable took its current value fails as out of memory.
static std::mutex g_alloc_mu;
static std::unordered_map<void *, size_t> g_alloc_live;
static int64_t g_alloc_count = 0;
static std::string g_fault_value;

hipError_t dev_alloc(void **p, size_t bytes) {
    std::lock_guard<std::mutex> lock(g_alloc_mu);
    const char *env = std::getenv("XCT_FAULT_ALLOC");
    const std::string cur = env ? env : "";
    if (cur != g_fault_value) {
        g_fault_value = cur;
        g_alloc_count = 0;
    }
    ++g_alloc_count;
    if (!cur.empty() && std::atoll(cur.c_str()) == g_alloc_count) {
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    const hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess)
        g_alloc_live[*p] = bytes;
    else
        (void)hipGetLastError();  // the failure is returned here; later calls must not see it again
    return e;
}

void dev_free(void *p) {
    if (!p) return;
    {
        std::lock_guard<std::mutex> lock(g_alloc_mu);
        g_alloc_live.erase(p);
    }
    (void)hipFree(p);
}

// ---- rounding FP64 -> 16-bit, nearest-even, single rounding -------------

__host__ __device__ inline uint16_t dbl_to_half_bits(double v) {
    // v >= 0 and finite (lengths); scale is bounded by sqrt(2) so no overflow.
    if (!(v > 0.0)) return 0;
    union { double d; uint64_t u; } b;
    b.d = v;
    int e = (int)((b.u >> 52) & 0x7ff) - 1023;
    uint64_t m = (b.u & 0xfffffffffffffull) | (1ull << 52);  // 53-bit significand
    // half: normal exponent range [-14, 15], 10 fraction bits
    int shift;            // bits of m to drop
    int ebias;            // biased exponent of the result before rounding carry
    if (e >= -14) {
        shift = 52 - 10;
        ebias = e + 15;
    } else {
        shift = 52 - 10 + (-14 - e);
        ebias = 0;
        if (shift > 63) return 0;
    }
    uint64_t q = m >> shift;
    uint64_t rem = m & ((1ull << shift) - 1);
    uint64_t halfway = 1ull << (shift - 1);
    if (rem > halfway || (rem == halfway && (q & 1))) ++q;
    if (ebias == 0) return (uint16_t)q;  // subnormal (q may carry into the normal range: still correct)
    // q has 11 bits (implicit one) unless rounding carried to 12 bits
    if (q >> 11) { q >>= 1; ++ebias; }
    if (ebias >= 31) return 0x7c00;
    return (uint16_t)((ebias << 10) | (q & 0x3ff));
}

__host__ __device__ inline uint16_t dbl_to_bf16_bits(double v) {
    if (!(v > 0.0)) return 0;
    union { double d; uint64_t u; } b;
    b.d = v;
    int e = (int)((b.u >> 52) & 0x7ff) - 1023;
    if (e < -126) return 0;  // below the normal range: not reachable for lengths >= 1e-9
    uint64_t m = (b.u & 0xfffffffffffffull) | (1ull << 52);
    const int shift = 52 - 7;
    uint64_t q = m >> shift;
    uint64_t rem = m & ((1ull << shift) - 1);
    uint64_t halfway = 1ull << (shift - 1);
    if (rem > halfway || (rem == halfway && (q & 1))) ++q;
    int ebias = e + 127;
    if (q >> 8) { q >>= 1; ++ebias; }
    return (uint16_t)((ebias << 7) | (q & 0x7f));
}

// ---- pseudo-Hilbert ordering of a tile grid ------------------------------

// Distance of (x, y) along the Hilbert curve filling a side x side square
// (side a power of two): at each scale pick the quadrant, add the cells of
// the quadrants before it, and rotate/reflect into the quadrant's frame.
static uint64_t hilbert_index(uint32_t side, uint32_t x, uint32_t y) {
    uint64_t d = 0;
    for (uint32_t s = side >> 1; s > 0; s >>= 1) {
        uint32_t rx = (x & s) ? 1u : 0u, ry = (y & s) ? 1u : 0u;
        d += (uint64_t)s * s * ((3u * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = side - 1 - x;
                y = side - 1 - y;
            }
            std::swap(x, y);
        }
    }
    return d;
}

// Tiles of a TH x TW grid ordered along the Hilbert curve of the enclosing
// power-of-two square, skipping cells outside the grid (pseudo-Hilbert).
static void hilbert_ranks(int TH, int TW, std::vector<int32_t> &rank_of, std::vector<int32_t> &coord_of) {
    uint32_t side = 1;
    while (side < (uint32_t)std::max(TH, TW)) side <<= 1;
    const int64_t n = (int64_t)TH * TW;
    std::vector<std::pair<uint64_t, int32_t>> key(n);
    for (int ty = 0; ty < TH; ++ty)
        for (int tx = 0; tx < TW; ++tx)
            key[(int64_t)ty * TW + tx] = {hilbert_index(side, (uint32_t)tx, (uint32_t)ty), ty * TW + tx};
    std::sort(key.begin(), key.end());
    rank_of.assign(n, 0);
    coord_of.assign(n, 0);
    for (int64_t r = 0; r < n; ++r) {
        coord_of[r] = key[r].second;
        rank_of[key[r].second] = (int32_t)r;
    }
}

// ---- row generators -------------------------------------------------------

// Rows of A: row tile = sinogram tile (8 angles x 8 channels); inputs are
// voxel tiles.
// Each generator visits the entries of one row as (key, offset, length):
// key = key_of[raster index of the input tile], the input tile's place in
// the block's staging order; offset = slot within the 8 x 8 tile.
struct ProjRows {
    int N, M, C;
    const int32_t *row_coord;  // sinogram rank -> raster tile
    int rowTW;                 // sinogram tiles per tile row
    int inTW;                  // voxel tiles per tile row
    int lanes;                 // lane_slot order
    double zero_below;         // lengths at or below this round to zero in the stored format: not entries
    template <class V>
    __device__ __forceinline__ void run(int64_t rt, int lane, const int32_t *key_of, V &&v) const {
        const int coord = row_coord[rt];
        const int o = lane_slot(lane, lanes);
        const int k = (coord / rowTW) * kTile + (o >> 3);
        const int c = (coord % rowTW) * kTile + (o & 7);
        if (k >= M || c >= C) return;
        trace_ray(N, M, C, k, c, [&](int i, int j, double len) {
            if (len > zero_below) v(key_of[(i >> 3) * inTW + (j >> 3)], ((i & 7) << 3) | (j & 7), len);
        });
    }
};

// Rows of A^T: row tile = voxel tile; inputs are sinogram tiles.
struct BackRows {
    int N, M, C;
    const int32_t *row_coord;  // voxel rank -> raster tile
    int rowTW;
    int inTW;                  // sinogram tiles per tile row
    int lanes;                 // lane_slot order
    double zero_below;         // as ProjRows
    template <class V>
    __device__ __forceinline__ void run(int64_t rt, int lane, const int32_t *key_of, V &&v) const {
        const int coord = row_coord[rt];
        const int o = lane_slot(lane, lanes);
        const int i = (coord / rowTW) * kTile + (o >> 3);
        const int j = (coord % rowTW) * kTile + (o & 7);
        if (i >= N || j >= N) return;
        trace_voxel(N, M, C, i, j, [&](int k, int c, double len) {
            if (len > zero_below) v(key_of[(k >> 3) * inTW + (c >> 3)], ((k & 7) << 3) | (c & 7), len);
        });
    }
};

// Staging order of the input tiles of a block.  Class q of the block selects
// a permutation of the input tiles: key_of[q][raster] is a tile's place in
// the order and tile_of[q][key] its internal (Hilbert-rank) index.  A block
// stages the tiles it touches in increasing key.
struct StageOrder {
    const int32_t *key_of;
    const int32_t *tile_of;
    const int32_t *blk_class;  // [n_blocks] or nullptr (class 0 everywhere)
    int64_t n_in;
    __device__ __forceinline__ int64_t base(int b) const { return blk_class ? (int64_t)blk_class[b] * n_in : 0; }
};

// ---- builder kernels --------------------------------------------------------

// Slab of (stage s, row tile h * P + w) in a block whose stages start at sb:
// wavefront w's slabs are contiguous, stage by stage, its R row tiles
// interleaved within each stage, so a wavefront's entries are one stream.
__host__ __device__ __forceinline__ int64_t slab_index(int64_t sb, int nst, int W, int R, int w, int h, int s) {
    return sb * W + ((int64_t)w * nst + s) * R + h;
}

struct BuildLds {
    uint32_t *bits;    // [nwords] touched input tiles, by rank
    uint32_t *prefix;  // [nwords] set bits before each word
    int64_t *red;      // [nthr + 1] scratch for reductions / scans
    uint16_t *cnt;     // [SW][nthr] per-lane entry counters of a stage window
};

__device__ __forceinline__ BuildLds carve(void *smem, int nwords, int nthr) {
    BuildLds L;
    char *p = (char *)smem;
    L.red = (int64_t *)p;
    p += sizeof(int64_t) * (size_t)(nthr + 1);
    L.bits = (uint32_t *)p;
    p += sizeof(uint32_t) * (size_t)nwords;
    L.prefix = (uint32_t *)p;
    p += sizeof(uint32_t) * (size_t)nwords;
    L.cnt = (uint16_t *)p;
    return L;
}

// A block has W row tiles; its P = blockDim / 64 wavefronts take R = W / P
// each: wavefront w holds row tiles h * P + w, h < R.
template <class Rows>
__device__ void mark_tiles(const Rows &rows, const int32_t *key_of, int64_t n_row_tiles, const BuildLds &L,
                           int nwords, int64_t *entries, int W) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int w = tid; w < nwords; w += nthr) L.bits[w] = 0u;
    __syncthreads();
    const int P = nthr >> 6, R = W / P;
    int64_t n = 0;
    for (int h = 0; h < R; ++h) {
        const int64_t rt = (int64_t)blockIdx.x * W + h * P + (tid >> 6);
        if (rt >= n_row_tiles) continue;
        int last = -1;
        rows.run(rt, tid & 63, key_of, [&](int key, int, double) {
            ++n;
            if (key == last) return;
            last = key;
            const uint32_t m = 1u << (key & 31);
            if (!(L.bits[key >> 5] & m)) atomicOr(&L.bits[key >> 5], m);
        });
    }
    if (entries) *entries = n;
    __syncthreads();
}

// Sum of one value per thread; result valid in every thread.
__device__ int64_t block_sum(const BuildLds &L, int64_t v) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    L.red[tid] = v;
    __syncthreads();
    if (tid == 0) {
        int64_t s = 0;
        for (int t = 0; t < nthr; ++t) s += L.red[t];
        L.red[nthr] = s;
    }
    __syncthreads();
    const int64_t s = L.red[nthr];
    __syncthreads();
    return s;
}

__device__ void build_prefix(const BuildLds &L, int nwords) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int per = (nwords + nthr - 1) / nthr;
    const int w0 = min(nwords, tid * per), w1 = min(nwords, w0 + per);
    int64_t s = 0;
    for (int w = w0; w < w1; ++w) s += __popc(L.bits[w]);
    L.red[tid] = s;
    __syncthreads();
    if (tid == 0) {
        int64_t acc = 0;
        for (int t = 0; t < nthr; ++t) {
            const int64_t x = L.red[t];
            L.red[t] = acc;
            acc += x;
        }
        L.red[nthr] = acc;
    }
    __syncthreads();
    uint32_t p = (uint32_t)L.red[tid];
    for (int w = w0; w < w1; ++w) {
        L.prefix[w] = p;
        p += __popc(L.bits[w]);
    }
    __syncthreads();
}

__device__ __forceinline__ int tile_pos(const BuildLds &L, int rank) {
    const uint32_t below = (1u << (rank & 31)) - 1u;
    return (int)(L.prefix[rank >> 5] + __popc(L.bits[rank >> 5] & below));
}

template <class Rows>
__global__ void k_footprint(Rows rows, StageOrder ord, int64_t n_row_tiles, int nwords, int W, int32_t *ntiles,
                            int64_t *nnz) {
    extern __shared__ __align__(16) char smem[];
    const BuildLds L = carve(smem, nwords, blockDim.x);
    int64_t e = 0;
    mark_tiles(rows, ord.key_of + ord.base(blockIdx.x), n_row_tiles, L, nwords, &e, W);
    int64_t t = 0;
    for (int w = threadIdx.x; w < nwords; w += blockDim.x) t += __popc(L.bits[w]);
    const int64_t tiles = block_sum(L, t);
    const int64_t ent = block_sum(L, e);
    if (threadIdx.x == 0) {
        ntiles[blockIdx.x] = (int32_t)tiles;
        nnz[blockIdx.x] = ent;
    }
}

__device__ __forceinline__ int wave_max(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

template <class Rows>
__global__ void k_plan(Rows rows, StageOrder ord, int64_t n_row_tiles, int nwords, int W, int T, int SW,
                       const int32_t *blk_tile, const int32_t *blk_stage, int32_t *tile_list, int32_t *stage_len,
                       int *err) {
    extern __shared__ __align__(16) char smem[];
    const int tid = threadIdx.x, nthr = blockDim.x, P = nthr >> 6, R = W / P, wave = tid >> 6;
    const int NV = W * kTileSlots;  // row lanes of the block (counters per stage)
    const BuildLds L = carve(smem, nwords, nthr);
    const int b = blockIdx.x;
    const int32_t *key_of = ord.key_of + ord.base(b);
    const int32_t *tile_of = ord.tile_of + ord.base(b);
    mark_tiles(rows, key_of, n_row_tiles, L, nwords, nullptr, W);
    build_prefix(L, nwords);
    const int base = blk_tile[b];
    const int ntl = blk_tile[b + 1] - base;
    for (int w = tid; w < nwords; w += nthr) {
        uint32_t m = L.bits[w];
        int p = (int)L.prefix[w];
        while (m) {
            const int bit = __ffs(m) - 1;
            if (p >= ntl) {  // footprint differs from the counting pass
                atomicOr(err, 2);
                break;
            }
            tile_list[base + p++] = tile_of[w * 32 + bit];
            m &= m - 1u;
        }
    }
    const int nst = blk_stage[b + 1] - blk_stage[b];
    for (int s0 = 0; s0 < nst; s0 += SW) {
        for (int q = tid; q < SW * NV; q += nthr) L.cnt[q] = 0;
        __syncthreads();
        for (int h = 0; h < R; ++h) {
            const int64_t rt = (int64_t)b * W + h * P + wave;
            const int vt = h * nthr + tid;
            if (rt >= n_row_tiles) continue;
            rows.run(rt, tid & 63, key_of, [&](int key, int, double) {
                const int st = tile_pos(L, key) / T - s0;
                if (st >= 0 && st < SW && s0 + st < nst) L.cnt[st * NV + vt] += 1;
            });
        }
        __syncthreads();
        const int lim = min(SW, nst - s0);
        for (int st = 0; st < lim; ++st)
            for (int h = 0; h < R; ++h) {
                const int v = wave_max((int)L.cnt[st * NV + h * nthr + tid]);
                if ((tid & 63) == 0)
                    stage_len[(int64_t)(blk_stage[b] + s0 + st) * W + h * P + wave] = (v + kGroup - 1) / kGroup;
            }
        __syncthreads();
    }
}

template <class Rows, int FMT>
__global__ void k_fill(Rows rows, StageOrder ord, int64_t n_row_tiles, int nwords, int W, int T, int SW,
                       const int32_t *blk_stage, const int64_t *slab, uint16_t *slot, float *val, double *val64,
                       uint32_t *packed, int *err) {
    extern __shared__ __align__(16) char smem[];
    const int tid = threadIdx.x, nthr = blockDim.x, P = nthr >> 6, R = W / P, wave = tid >> 6, lane = tid & 63;
    const int NV = W * kTileSlots;
    const BuildLds L = carve(smem, nwords, nthr);
    const int b = blockIdx.x;
    const int32_t *key_of = ord.key_of + ord.base(b);
    mark_tiles(rows, key_of, n_row_tiles, L, nwords, nullptr, W);
    build_prefix(L, nwords);
    const int nst = blk_stage[b + 1] - blk_stage[b];
    for (int s0 = 0; s0 < nst; s0 += SW) {
        for (int q = tid; q < SW * NV; q += nthr) L.cnt[q] = 0;
        __syncthreads();
        for (int h = 0; h < R; ++h) {
            const int64_t rt = (int64_t)b * W + h * P + wave;
            const int vt = h * nthr + tid;
            if (rt >= n_row_tiles) continue;
            rows.run(rt, lane, key_of, [&](int key, int off, double len) {
                const int pos = tile_pos(L, key);
                const int st = pos / T;
                const int sl = st - s0;
                if (sl < 0 || sl >= SW) return;
                if (st >= nst) {
                    atomicOr(err, 4);
                    return;
                }
                const int n = L.cnt[sl * NV + vt]++;
                const int64_t gs = slab_index(blk_stage[b], nst, W, R, wave, h, st);
                const int64_t g = slab[gs] + n / kGroup;
                if (g >= slab[gs + 1]) {
                    atomicOr(err, 1);
                    return;
                }
                const int64_t idx = (g * kTileSlots + lane) * kGroup + (n % kGroup);
                const uint32_t s = (uint32_t)((pos % T) * kTileSlots + off);
                if (FMT == XCT_F32) {
                    const int64_t li = (int64_t)lane * kGroup + (n % kGroup);
                    slot[g * 768 + li] = (uint16_t)s;
                    val[g * 384 + 128 + li] = (float)len;
                } else if (FMT == XCT_F64) {
                    const int64_t li = (int64_t)lane * kGroup + (n % kGroup);
                    slot[g * 1280 + li] = (uint16_t)s;
                    val64[g * 320 + 64 + li] = len;
                } else if (FMT == XCT_F16) {
                    packed[idx] = (s << 16) | dbl_to_half_bits(len);
                } else {
                    packed[idx] = (s << 16) | dbl_to_bf16_bits(len);
                }
            });
        }
        __syncthreads();
    }
}

// ---- step order of the slabs against LDS bank conflicts --------------------
//
// The SpMM reads a staged row of RB bytes as CH = RB / 16 chunks of 16 bytes,
// lane l taking chunk (j + l) mod CH at sub-step j.  A wavefront's 16-byte
// LDS read on gfx950 is served in four phases of 16 lanes, lane l being in
// phase (bit 2 ^ bit 3 ^ bit 4 of l) + 2 * (bit 5 of l), and within a phase
// each group of four banks (the 16 B at a given offset mod 256 B) delivers
// one distinct address per cycle (measured with lane/address permutations).
// Chunk c of placed row r lies in group (r * CH + c) mod 16, so the lanes of
// one phase that share l mod CH read without conflict when their rows differ
// mod Q = 16 / CH.  Each such set of Q lanes (a unit) is scheduled step by
// step: the entries of a lane within a slab may be taken in any order (the
// sum is the same up to rounding) and its padding steps may point at any row
// (their length is 0), so at every step the unit's lanes take entries of Q
// different row classes wherever their remaining entries allow.  Lanes whose
// remaining entries fill all remaining steps go first, the most constrained
// of them first; then lanes with the most entries left; the rest pad.

// The quads (4 consecutive lanes) of a 32-lane half in phase parity p.
__device__ __forceinline__ int phase_quad(int p, int a) {
    const int q0[4] = {0, 3, 5, 6}, q1[4] = {1, 2, 4, 7};
    return p ? q1[a] : q0[a];
}

// LDS bytes per step of a slab and fixed part, for a launch of k_balance.
inline size_t balance_lds_step(xct_dtype vdt) {
    return (size_t)kTileSlots * (vdt == XCT_F64 ? 14 : vdt == XCT_F32 ? 10 : 8);
}
inline size_t balance_lds_fixed(int Q) { return (size_t)2 * kTileSlots * Q * sizeof(uint16_t); }

template <int FMT, int Q>
__global__ void __launch_bounds__(64) k_balance(const int64_t *slab, const int32_t *ids, int L_cap, uint16_t *slot,
                                                float *val, double *val64, uint32_t *packed,
                                                unsigned long long *n_done, int *err) {
    constexpr int CH = 16 / Q;  // chunks per staged row
    constexpr int NU = 64 / Q;  // units per wavefront
    constexpr bool kSplit = FMT == XCT_F32 || FMT == XCT_F64;  // slots and lengths stored apart
    typedef typename std::conditional<FMT == XCT_F64, uint64_t, uint32_t>::type EntT;
    extern __shared__ __align__(16) char smem[];
    const int lane = threadIdx.x;
    const int64_t sid = ids[blockIdx.x];
    const int64_t g0 = slab[sid];
    const int L = (int)(slab[sid + 1] - g0) * kGroup;
    if (L == 0 || L > L_cap) return;  // whole workgroup (the host sorts slabs by length)
    char *p = smem;
    EntT *ent = (EntT *)p;  // F32 / F64: length bits; 16-bit: packed entry
    p += sizeof(EntT) * (size_t)L * 64;
    uint16_t *eslot = (uint16_t *)p;  // F32 / F64 only
    if (kSplit) p += sizeof(uint16_t) * (size_t)L * 64;
    uint16_t *order = (uint16_t *)p;  // per lane: its steps sorted by row class
    p += sizeof(uint16_t) * (size_t)L * 64;
    uint16_t *src = (uint16_t *)p;  // new step -> old step, or 0x8000 | class for padding
    p += sizeof(uint16_t) * (size_t)L * 64;
    uint16_t *nxt = (uint16_t *)p;  // [64][Q] next position in order[] per class
    p += sizeof(uint16_t) * 64 * Q;
    uint16_t *lim = (uint16_t *)p;  // [64][Q] end of each class in order[]

    for (int t = 0; t < L; t += kGroup) {
        const int64_t g = g0 + t / kGroup;
        if constexpr (FMT == XCT_F32) {
            const uint16_t *sp = slot + g * 768 + lane * kGroup;
            const float *vp = val + g * 384 + 128 + lane * kGroup;
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                ent[(t + q) * 64 + lane] = __float_as_uint(vp[q]);
                eslot[(t + q) * 64 + lane] = sp[q];
            }
        } else if constexpr (FMT == XCT_F64) {
            const uint16_t *sp = slot + g * 1280 + lane * kGroup;
            const double *vp = val64 + g * 320 + 64 + lane * kGroup;
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                ent[(t + q) * 64 + lane] = (EntT)__double_as_longlong(vp[q]);
                eslot[(t + q) * 64 + lane] = sp[q];
            }
        } else {
            const uint32_t *pp = packed + (g * kTileSlots + lane) * kGroup;
#pragma unroll
            for (int q = 0; q < kGroup; ++q) ent[(t + q) * 64 + lane] = pp[q];
        }
    }
    auto real_cls = [&](int t, int l, int &cls) -> bool {
        const EntT e = ent[t * 64 + l];
        if constexpr (kSplit) {
            cls = eslot[t * 64 + l] & (Q - 1);
            return e != 0u;
        } else {
            cls = (int)(e >> 16) & (Q - 1);
            return (e & 0xffffu) != 0u;
        }
    };
    // counting sort of this lane's steps by class
    {
        int c[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) c[q] = 0;
        for (int t = 0; t < L; ++t) {
            int cls;
            const bool r = real_cls(t, lane, cls);
#pragma unroll
            for (int q = 0; q < Q; ++q) c[q] += (r && cls == q) ? 1 : 0;
        }
        int acc = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            nxt[lane * Q + q] = (uint16_t)acc;
            acc += c[q];
            lim[lane * Q + q] = (uint16_t)acc;
            c[q] = acc - c[q];  // running position
        }
        for (int t = 0; t < L; ++t) {
            int cls;
            if (!real_cls(t, lane, cls)) continue;
            int k = 0;
#pragma unroll
            for (int q = 0; q < Q; ++q)
                if (cls == q) k = c[q]++;
            order[k * 64 + lane] = (uint16_t)t;
        }
    }
    __syncthreads();

    if (lane < NU) {
        const int ph = lane / CH, m = lane % CH;
        int ul[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) ul[i] = 32 * (ph >> 1) + 4 * phase_quad(ph & 1, i & 3) + m + CH * (i >> 2);
        // per lane and class: entries left (cnt) and the end of the class in
        // order[] (end); the next entry of the class is order[end - cnt]
        int cnt[Q][Q], end[Q][Q], rem[Q];
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            rem[i] = 0;
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                end[i][q] = lim[ul[i] * Q + q];
                cnt[i][q] = end[i][q] - (int)nxt[ul[i] * Q + q];
                rem[i] += cnt[i][q];
            }
        }
        constexpr int kUnset = -1, kPadPending = 0x200, kPad = 0x100;
        for (int t = 0; t < L; ++t) {
            const int rs = L - t;
            uint32_t used = 0;
            int pick[Q];
#pragma unroll
            for (int i = 0; i < Q; ++i) pick[i] = kUnset;
            // lanes whose entries fill every remaining step, fewest classes first
            for (int it = 0; it < Q; ++it) {
                int best = -1, bk = 1 << 30;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    int nz = 0;
#pragma unroll
                    for (int q = 0; q < Q; ++q) nz += cnt[i][q] > 0 ? 1 : 0;
                    if (pick[i] == kUnset && rem[i] >= rs && nz < bk) {
                        bk = nz;
                        best = i;
                    }
                }
                if (best < 0) break;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    if (i != best) continue;
                    int bq = 0, bkey = -1;
#pragma unroll
                    for (int q = 0; q < Q; ++q) {
                        const int key = cnt[i][q] > 0 ? (((used >> q) & 1u) ? 0 : (1 << 16)) + cnt[i][q] : -1;
                        if (key > bkey) {
                            bkey = key;
                            bq = q;
                        }
                    }
                    pick[i] = bq;
                    used |= 1u << bq;
                }
            }
            // then lanes with the most entries left, on a free class
            for (int it = 0; it < Q; ++it) {
                int best = -1, bk = 0;
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    if (pick[i] == kUnset && rem[i] > bk) {
                        bk = rem[i];
                        best = i;
                    }
                if (best < 0) break;
#pragma unroll
                for (int i = 0; i < Q; ++i) {
                    if (i != best) continue;
                    int bq = -1, bkey = 0;
#pragma unroll
                    for (int q = 0; q < Q; ++q)
                        if (!((used >> q) & 1u) && cnt[i][q] > bkey) {
                            bkey = cnt[i][q];
                            bq = q;
                        }
                    if (bq >= 0) {
                        pick[i] = bq;
                        used |= 1u << bq;
                    } else {
                        pick[i] = kPadPending;
                    }
                }
            }
            // padding on the classes left over
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                if (pick[i] != kUnset && pick[i] != kPadPending) continue;
                const uint32_t freeb = ~used & ((1u << Q) - 1u);
                const int q = freeb ? __builtin_ctz(freeb) : 0;
                used |= 1u << q;
                pick[i] = kPad | q;
            }
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                const int l = ul[i];
                if (pick[i] & kPad) {
                    src[t * 64 + l] = (uint16_t)(0x8000 | (pick[i] & 0xff));
                    continue;
                }
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    if (q != pick[i]) continue;
                    const int k = end[i][q] - cnt[i][q];
                    if (cnt[i][q] <= 0) atomicOr(err, 8);  // cannot happen: a class is picked with entries left
                    src[t * 64 + l] = order[min(max(k, 0), L - 1) * 64 + l];
                    cnt[i][q] -= 1;
                    rem[i] -= 1;
                }
            }
        }
    }
    __syncthreads();

    for (int t = 0; t < L; t += kGroup) {
        const int64_t g = g0 + t / kGroup;
        EntT e[kGroup];
        uint16_t sl[kGroup];
#pragma unroll
        for (int q = 0; q < kGroup; ++q) {
            const int sidx = src[(t + q) * 64 + lane];
            if (sidx & 0x8000) {
                e[q] = kSplit ? (EntT)0 : (EntT)(sidx & 0xff) << 16;
                sl[q] = (uint16_t)(sidx & 0xff);
            } else {
                e[q] = ent[sidx * 64 + lane];
                sl[q] = kSplit ? eslot[sidx * 64 + lane] : 0;
            }
        }
        if constexpr (FMT == XCT_F32) {
            uint16_t *sp = slot + g * 768 + lane * kGroup;
            float *vp = val + g * 384 + 128 + lane * kGroup;
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                sp[q] = sl[q];
                vp[q] = __uint_as_float((uint32_t)e[q]);
            }
        } else if constexpr (FMT == XCT_F64) {
            uint16_t *sp = slot + g * 1280 + lane * kGroup;
            double *vp = val64 + g * 320 + 64 + lane * kGroup;
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                sp[q] = sl[q];
                vp[q] = __longlong_as_double((long long)e[q]);
            }
        } else {
            uint32_t *pp = packed + (g * kTileSlots + lane) * kGroup;
#pragma unroll
            for (int q = 0; q < kGroup; ++q) pp[q] = (uint32_t)e[q];
        }
    }
    if (lane == 0) atomicAdd(n_done, 1ull);
}

// ---- host orchestration ---------------------------------------------------

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        dev_free(p);
    }
};

template <class T>
static int upload(T **dst, const std::vector<T> &src) {
    XCT_HIP_TRY(dev_alloc((void **)dst, sizeof(T) * std::max<size_t>(1, src.size())));
    if (!src.empty()) XCT_HIP_TRY(hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
    return XCT_OK;
}

static int make_grid(Grid &g, int H, int Wd) {
    g.H = H;
    g.Wd = Wd;
    g.TH = (H + kTile - 1) / kTile;
    g.TW = (Wd + kTile - 1) / kTile;
    g.n_tiles = (int64_t)g.TH * g.TW;
    hilbert_ranks(g.TH, g.TW, g.h_rank_of, g.h_coord_of);
    int rc = upload(&g.rank_of, g.h_rank_of);
    if (rc) return rc;
    return upload(&g.coord_of, g.h_coord_of);
}

// ---- staging orders -------------------------------------------------------

constexpr int kSweepClasses = 64;  // direction classes of the projection sweep order

struct HostOrder {
    std::vector<int32_t> key_of, tile_of, blk_class;
    int n_class = 1;
};

// Hilbert order: the key is the tile's Hilbert rank, which is also its
// internal index.
static void order_hilbert(const Grid &in, HostOrder &o) {
    o.n_class = 1;
    o.key_of = in.h_rank_of;
    o.tile_of.resize(in.n_tiles);
    for (int64_t r = 0; r < in.n_tiles; ++r) o.tile_of[r] = (int32_t)r;
}

// Raster order of the input grid (for A^T: sinogram tiles angle-major, so a
// stage covers whole channel ranges of consecutive angles and every voxel of
// a wavefront finds about the same number of entries in it).
static void order_raster(const Grid &in, HostOrder &o) {
    o.n_class = 1;
    o.key_of.resize(in.n_tiles);
    o.tile_of.resize(in.n_tiles);
    for (int64_t t = 0; t < in.n_tiles; ++t) {
        o.key_of[t] = (int32_t)t;
        o.tile_of[t] = in.h_rank_of[t];
    }
}

// Sweep order for A: voxel tiles sorted by the distance of their centre
// along a ray direction, one order per direction class; a block uses the
// class of its rays' mean angle.  A stage is then a band across the block's
// (nearly parallel) rays and every ray of a wavefront crosses it with about
// the same number of voxels, which keeps the ELL slabs short.
static void order_sweep_proj(const xct_matrix *m, int W, int n_blocks, HostOrder &o) {
    const Grid &in = m->vol, &rows = m->sino;
    const int Q = kSweepClasses;
    o.n_class = Q;
    const int64_t n = in.n_tiles;
    o.key_of.resize((size_t)Q * n);
    o.tile_of.resize((size_t)Q * n);
    std::vector<std::pair<double, int32_t>> key(n);
    for (int q = 0; q < Q; ++q) {
        const double th = M_PI * (q + 0.5) / Q;
        const double dx = -std::sin(th), dy = std::cos(th);
        for (int64_t t = 0; t < n; ++t) {
            const int ty = (int)(t / in.TW), tx = (int)(t % in.TW);
            key[t] = {(tx + 0.5) * dx + (ty + 0.5) * dy, in.h_rank_of[t]};
        }
        std::sort(key.begin(), key.end());
        for (int64_t p = 0; p < n; ++p) {
            const int32_t rank = key[p].second;
            const int32_t raster = in.h_coord_of[rank];
            o.key_of[(size_t)q * n + raster] = (int32_t)p;
            o.tile_of[(size_t)q * n + p] = rank;
        }
    }
    o.blk_class.resize(n_blocks);
    for (int b = 0; b < n_blocks; ++b) {
        double sc = 0.0, ss = 0.0;
        for (int w = 0; w < W; ++w) {
            const int64_t rt = (int64_t)b * W + w;
            if (rt >= rows.n_tiles) break;
            const int ta = rows.h_coord_of[rt] / rows.TW;
            for (int k = ta * kTile; k < std::min(m->M, ta * kTile + kTile); ++k) {
                const double th = M_PI * k / m->M;
                sc += std::cos(2.0 * th);
                ss += std::sin(2.0 * th);
            }
        }
        double th = 0.5 * std::atan2(ss, sc);
        if (th < 0) th += M_PI;
        int q = (int)(th / M_PI * Q);
        o.blk_class[b] = q < 0 ? 0 : (q >= Q ? Q - 1 : q);
    }
}

struct DevOrder {
    StageOrder d{};
    void *bufs[3] = {nullptr, nullptr, nullptr};
    ~DevOrder() {
        for (void *p : bufs)
            dev_free(p);
    }
};

static int upload_order(const HostOrder &h, int64_t n_in, DevOrder &d) {
    int32_t *k = nullptr, *t = nullptr, *c = nullptr;
    int rc = upload(&k, h.key_of);
    d.bufs[0] = k;
    if (!rc) rc = upload(&t, h.tile_of);
    d.bufs[1] = t;
    if (!rc && !h.blk_class.empty()) {
        rc = upload(&c, h.blk_class);
        d.bufs[2] = c;
    }
    d.d.key_of = k;
    d.d.tile_of = t;
    d.d.blk_class = c;
    d.d.n_in = n_in;
    return rc;
}

static void free_op(OpPlan &op) {
    void *ps[] = {op.blk_stage, op.blk_tile, op.tile_list, op.slab, op.ent};
    for (void *p : ps)
        dev_free(p);
    op = OpPlan();
}

template <class Rows>
static int build_op(OpPlan &op, const Rows &rows, const StageOrder &ord, int64_t n_row_tiles, int64_t n_in_tiles,
                    int W, int T, xct_dtype vdt, int row_bytes, int balance, hipStream_t st) {
    op.which = std::is_same<Rows, BackRows>::value ? 1 : 0;
    op.lanes = rows.lanes;
    op.n_row_tiles = n_row_tiles;
    op.n_in_tiles = n_in_tiles;
    op.W = W;
    op.R = W > 16 ? W / 16 : 1;  // row tiles per wavefront
    op.T = T;
    op.n_blocks = (int)((n_row_tiles + W - 1) / W);
    const int R = op.R, P = W / R;
    const int nthr = P * kTileSlots;  // threads of the builder kernels: one per lane of a wavefront
    const int NV = W * kTileSlots;    // row lanes of a block
    const int nwords = (int)((n_in_tiles + 31) / 32);
    int dev = 0;
    XCT_HIP_TRY(hipGetDevice(&dev));
    int lds_max = 0;
    XCT_HIP_TRY(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    const size_t fixed = sizeof(int64_t) * (size_t)(nthr + 1) + sizeof(uint32_t) * 2 * (size_t)nwords;
    if ((size_t)lds_max < fixed + sizeof(uint16_t) * (size_t)NV)
        return fail(XCT_ERR_UNSUPPORTED, "grid too large for the builder's LDS tile bitmap");
    int SW = (int)std::min<size_t>(64, ((size_t)lds_max - fixed) / (sizeof(uint16_t) * (size_t)NV));
    const size_t smem_mark = fixed;
    const size_t smem_win = fixed + sizeof(uint16_t) * (size_t)SW * NV;

    const int nb = op.n_blocks;
    DevBuf d_nt, d_nnz, d_len, d_err;
    XCT_HIP_TRY(dev_alloc(&d_nt.p, sizeof(int32_t) * nb));
    XCT_HIP_TRY(dev_alloc(&d_nnz.p, sizeof(int64_t) * nb));
    XCT_HIP_TRY(hipFuncSetAttribute((const void *)k_footprint<Rows>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem_mark));
    hipLaunchKernelGGL(k_footprint<Rows>, dim3(nb), dim3(nthr), smem_mark, st, rows, ord, n_row_tiles, nwords, W,
                       (int32_t *)d_nt.p, (int64_t *)d_nnz.p);
    XCT_HIP_TRY(hipGetLastError());
    std::vector<int32_t> nt(nb);
    std::vector<int64_t> nnzb(nb);
    XCT_HIP_TRY(hipMemcpyAsync(nt.data(), d_nt.p, sizeof(int32_t) * nb, hipMemcpyDeviceToHost, st));
    XCT_HIP_TRY(hipMemcpyAsync(nnzb.data(), d_nnz.p, sizeof(int64_t) * nb, hipMemcpyDeviceToHost, st));
    XCT_HIP_TRY(hipStreamSynchronize(st));

    std::vector<int32_t> blk_tile(nb + 1, 0), blk_stage(nb + 1, 0);
    int64_t nnz = 0;
    for (int b = 0; b < nb; ++b) {
        const int64_t tiles = blk_tile[b] + (int64_t)nt[b];
        const int64_t stages = blk_stage[b] + (int64_t)(nt[b] + T - 1) / T;
        if (tiles > INT32_MAX || stages > INT32_MAX) return fail(XCT_ERR_UNSUPPORTED, "tile list too long");
        blk_tile[b + 1] = (int32_t)tiles;
        blk_stage[b + 1] = (int32_t)stages;
        nnz += nnzb[b];
    }
    op.n_list = blk_tile[nb];
    op.n_stages = blk_stage[nb];
    op.nnz = nnz;
    op.staged_slots = op.n_list * kTileSlots;
    int rc = upload(&op.blk_tile, blk_tile);
    if (!rc) rc = upload(&op.blk_stage, blk_stage);
    if (rc) return rc;
    // 4 entries of padding: the SpMM reads the list four entries at a time
    XCT_HIP_TRY(dev_alloc((void **)&op.tile_list, sizeof(int32_t) * (op.n_list + 4)));
    XCT_HIP_TRY(hipMemsetAsync(op.tile_list, 0, sizeof(int32_t) * (op.n_list + 4), st));
    const int64_t nlen = op.n_stages * W;
    XCT_HIP_TRY(dev_alloc(&d_len.p, sizeof(int32_t) * std::max<int64_t>(1, nlen)));
    XCT_HIP_TRY(dev_alloc(&d_err.p, sizeof(int)));
    XCT_HIP_TRY(hipMemsetAsync(d_err.p, 0, sizeof(int), st));
    XCT_HIP_TRY(hipFuncSetAttribute((const void *)k_plan<Rows>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)smem_win));
    hipLaunchKernelGGL(k_plan<Rows>, dim3(nb), dim3(nthr), smem_win, st, rows, ord, n_row_tiles, nwords, W, T, SW,
                       op.blk_tile, op.blk_stage, op.tile_list, (int32_t *)d_len.p, (int *)d_err.p);
    XCT_HIP_TRY(hipGetLastError());
    std::vector<int32_t> len(nlen);
    if (nlen) XCT_HIP_TRY(hipMemcpyAsync(len.data(), d_len.p, sizeof(int32_t) * nlen, hipMemcpyDeviceToHost, st));
    XCT_HIP_TRY(hipStreamSynchronize(st));
    // Slabs are laid out wavefront by wavefront within a block (slab_index),
    // so a wavefront's entries form one contiguous stream; len is indexed
    // [stage][row tile of the block].
    std::vector<int64_t> slab(nlen + 1, 0);
    {
        int64_t acc = 0;
        for (int b = 0; b < nb; ++b) {
            const int sb = blk_stage[b], nst = blk_stage[b + 1] - blk_stage[b];
            for (int w = 0; w < P; ++w)
                for (int sl = 0; sl < nst; ++sl)
                    for (int h = 0; h < R; ++h) {
                        const int64_t i = slab_index(sb, nst, W, R, w, h, sl);
                        slab[i] = acc;
                        acc += len[(int64_t)(sb + sl) * W + h * P + w];
                    }
        }
        slab[nlen] = acc;
    }
    op.n_groups = slab[nlen];
    op.padded = op.n_groups * kTileSlots * kGroup;
    rc = upload(&op.slab, slab);
    if (rc) return rc;
    // at least one group: the kernel's prefetch may re-read group 0
    const size_t nent = (size_t)std::max<int64_t>(1, op.n_groups) * kTileSlots * kGroup;
    const size_t ent_bytes = nent * entry_bytes(vdt);
    XCT_HIP_TRY(dev_alloc(&op.ent, ent_bytes));
    XCT_HIP_TRY(hipMemsetAsync(op.ent, 0, ent_bytes, st));
    if (vdt == XCT_F32) {
        op.slot = (uint16_t *)op.ent;
        op.val = (float *)op.ent;
    } else if (vdt == XCT_F64) {
        op.slot = (uint16_t *)op.ent;
        op.val64 = (double *)op.ent;
    } else {
        op.packed = (uint32_t *)op.ent;
    }
    auto fill = [&](auto kern) -> int {
        XCT_HIP_TRY(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)smem_win));
        hipLaunchKernelGGL(kern, dim3(nb), dim3(nthr), smem_win, st, rows, ord, n_row_tiles, nwords, W, T, SW,
                           op.blk_stage, op.slab, op.slot, op.val, op.val64, op.packed, (int *)d_err.p);
        XCT_HIP_TRY(hipGetLastError());
        return XCT_OK;
    };
    if (vdt == XCT_F32)
        rc = fill(k_fill<Rows, XCT_F32>);
    else if (vdt == XCT_F64)
        rc = fill(k_fill<Rows, XCT_F64>);
    else if (vdt == XCT_F16)
        rc = fill(k_fill<Rows, XCT_F16>);
    else
        rc = fill(k_fill<Rows, XCT_BF16>);
    if (rc) return rc;
    int err = 0;
    XCT_HIP_TRY(hipMemcpyAsync(&err, d_err.p, sizeof(int), hipMemcpyDeviceToHost, st));
    XCT_HIP_TRY(hipStreamSynchronize(st));
    if (err) return fail(XCT_ERR_INTERNAL, "builder passes disagree on the entry set (code " + std::to_string(err) + ")");
    op.n_slabs = nlen;
    op.balanced = 0;
    // reorder the slabs' steps against LDS bank conflicts (rows of 32 or 64 bytes)
    const int Q = row_bytes == 64 ? 4 : row_bytes == 32 ? 8 : 0;
    if (balance && Q && nlen) {
        const size_t step = balance_lds_step(vdt), fixed_b = balance_lds_fixed(Q);
        const int64_t cap = ((int64_t)(((size_t)lds_max - fixed_b) / step) / kGroup) * kGroup;
        // slabs by length: each launch sizes its LDS for its longest slab, so
        // the many short slabs run many workgroups per CU
        const int64_t bucket_cap[4] = {32, 64, 128, cap};
        std::vector<int32_t> ids[4];
        int64_t empty = 0;
        for (int64_t i = 0; i < nlen; ++i) {
            const int64_t L = (slab[i + 1] - slab[i]) * kGroup;  // slab i in slab (wave-major) order
            if (L == 0) {
                ++empty;
                continue;
            }
            for (int k = 0; k < 4; ++k)
                if (L <= bucket_cap[k] && L <= cap) {
                    ids[k].push_back((int32_t)i);
                    break;
                }
        }
        DevBuf d_done;
        XCT_HIP_TRY(dev_alloc(&d_done.p, sizeof(unsigned long long)));
        XCT_HIP_TRY(hipMemsetAsync(d_done.p, 0, sizeof(unsigned long long), st));
        std::vector<DevBuf> d_ids(4);
        for (int k = 0; k < 4; ++k) {
            if (ids[k].empty()) continue;
            const int64_t bc = std::min(bucket_cap[k], cap);
            const size_t smem_b = fixed_b + step * (size_t)bc;
            XCT_HIP_TRY(dev_alloc(&d_ids[k].p, sizeof(int32_t) * ids[k].size()));
            XCT_HIP_TRY(hipMemcpyAsync(d_ids[k].p, ids[k].data(), sizeof(int32_t) * ids[k].size(),
                                       hipMemcpyHostToDevice, st));
            auto bal = [&](auto kern) -> int {
                XCT_HIP_TRY(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                (int)smem_b));
                hipLaunchKernelGGL(kern, dim3((unsigned)ids[k].size()), dim3(64), smem_b, st, op.slab,
                                   (const int32_t *)d_ids[k].p, (int)bc, op.slot, op.val, op.val64, op.packed,
                                   (unsigned long long *)d_done.p, (int *)d_err.p);
                XCT_HIP_TRY(hipGetLastError());
                return XCT_OK;
            };
            if (vdt == XCT_F32)
                rc = Q == 4 ? bal(k_balance<XCT_F32, 4>) : bal(k_balance<XCT_F32, 8>);
            else if (vdt == XCT_F64)
                rc = Q == 4 ? bal(k_balance<XCT_F64, 4>) : bal(k_balance<XCT_F64, 8>);
            else if (vdt == XCT_F16)
                rc = Q == 4 ? bal(k_balance<XCT_F16, 4>) : bal(k_balance<XCT_F16, 8>);
            else
                rc = Q == 4 ? bal(k_balance<XCT_BF16, 4>) : bal(k_balance<XCT_BF16, 8>);
            if (rc) return rc;
        }
        unsigned long long done = 0;
        XCT_HIP_TRY(hipMemcpyAsync(&done, d_done.p, sizeof(done), hipMemcpyDeviceToHost, st));
        XCT_HIP_TRY(hipMemcpyAsync(&err, d_err.p, sizeof(int), hipMemcpyDeviceToHost, st));
        XCT_HIP_TRY(hipStreamSynchronize(st));
        if (err) return fail(XCT_ERR_INTERNAL, "slab reordering lost an entry (code " + std::to_string(err) + ")");
        op.balanced = (int64_t)done + empty;  // empty slabs are trivially conflict-free
    }
    const int64_t eb = (int64_t)entry_bytes(vdt);
    op.bytes = op.padded * eb + (int64_t)sizeof(int64_t) * (nlen + 1) + (int64_t)sizeof(int32_t) * op.n_list +
               (int64_t)sizeof(int32_t) * 2 * (nb + 1);
    return XCT_OK;
}

}  // namespace xct

using namespace xct;

extern "C" const char *xct_last_error(void) { return g_last_error.c_str(); }

extern "C" int xct_device_memory(int64_t *buffers, int64_t *bytes) {
    if (!buffers || !bytes) return fail(XCT_ERR_INVALID, "NULL argument");
    std::lock_guard<std::mutex> lock(g_alloc_mu);
    int64_t b = 0;
    for (const auto &kv : g_alloc_live) b += (int64_t)kv.second;
    *buffers = (int64_t)g_alloc_live.size();
    *bytes = b;
    return XCT_OK;
}

extern "C" void xct_free_matrix(xct_matrix *m) {
    if (!m) return;
    free_op(m->A);
    free_op(m->AT);
    void *ps[] = {m->vol.rank_of, m->vol.coord_of, m->sino.rank_of, m->sino.coord_of};
    for (void *p : ps)
        dev_free(p);
    for (hipEvent_t e : m->stream_ev)
        if (e) (void)hipEventDestroy(e);
    delete m;
}

extern "C" int xct_build_matrix(int n, int n_angles, int n_channels, xct_dtype value_dtype,
                                const xct_build_opts *opts, void *stream, xct_matrix **out) {
    if (!out) return fail(XCT_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (n < 1 || n > 8192) return fail(XCT_ERR_INVALID, "n must be in [1, 8192]");
    if (n_angles < 1 || n_angles > 30000) return fail(XCT_ERR_INVALID, "n_angles must be in [1, 30000]");
    if (n_channels < 1 || n_channels > 16384) return fail(XCT_ERR_INVALID, "n_channels must be in [1, 16384]");
    if (!valid_dtype(value_dtype)) return fail(XCT_ERR_INVALID, "bad value dtype");
    if (opts && (opts->stage_order < 0 || opts->stage_order > 1))
        return fail(XCT_ERR_INVALID, "stage_order must be 0 (sweep) or 1 (Hilbert)");
    xct_build_opts o = {};
    if (opts) o = *opts;
    const int W = o.tile_waves ? o.tile_waves : 16;
    const int F = o.fuse ? o.fuse : (value_dtype == XCT_F64 ? 8 : 16);
    int lds = o.lds_bytes;
    if (W < 1 || (W > 16 && W != 32)) return fail(XCT_ERR_INVALID, "tile_waves must be in [1, 16] or 32");
    if (F != 1 && F != 2 && F != 4 && F != 8 && F != 16 && F != 32)
        return fail(XCT_ERR_INVALID, "fuse must be 1, 2, 4, 8, 16 or 32");
    if (F == 32 && (value_dtype == XCT_F32 || value_dtype == XCT_F64 || W > 16))
        return fail(XCT_ERR_UNSUPPORTED, "32 fused slices need a 16-bit matrix and at most 16 row tiles per workgroup");
    if (F == 16 && value_dtype == XCT_F64)
        return fail(XCT_ERR_UNSUPPORTED, "FP64 matrices fuse at most 8 slices (64-byte staged rows)");
    const int per_tile = kTileSlots * F * elem_bytes(value_dtype);
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return fail(XCT_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(he));
    int lds_max = 0;
    he = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (he != hipSuccess) return fail(XCT_ERR_HIP, std::string("hipDeviceGetAttribute: ") + hipGetErrorString(he));
    if (!lds) lds = lds_max;  // one workgroup of 16 waves per CU with the whole LDS
    if (lds < per_tile || lds > lds_max)
        return fail(XCT_ERR_INVALID, "lds_bytes must hold one tile and fit the device LDS");
    int T = lds / per_tile;
    if (T > 1024) T = 1024;  // stage-local slots must fit 16 bits
    if (o.lane_order < 0 || o.lane_order > 1) return fail(XCT_ERR_INVALID, "lane_order must be 0 or 1");
    if (o.xcd_remap < -1) return fail(XCT_ERR_INVALID, "xcd_remap must be -1, 0, 1 or a run length >= 2");
    if (o.slab_order < 0 || o.slab_order > 1) return fail(XCT_ERR_INVALID, "slab_order must be 0 or 1");
    if (o.arith < 0 || o.arith > 1) return fail(XCT_ERR_INVALID, "arith must be 0 or 1");
    if (o.arith == 1 && value_dtype != XCT_F16)
        return fail(XCT_ERR_UNSUPPORTED, "FP16 arithmetic needs an FP16 matrix");
    if (o.debug_poison_lds < 0 || o.debug_poison_lds > 1)
        return fail(XCT_ERR_INVALID, "debug_poison_lds must be 0 or 1");
    const int row_bytes = F * elem_bytes(value_dtype);
    const int lanes = o.lane_order;
    // A length that rounds to zero in the stored format contributes nothing
    // and is not an entry (FP16: lengths up to 2^-25, the half-way point to
    // the smallest subnormal, round to zero; BF16 and FP32 keep every length
    // above the geometric cut-off).
    const double zero_below = value_dtype == XCT_F16 ? 0x1p-25 : 0.0;
    auto t0 = std::chrono::steady_clock::now();
    xct_matrix *m = new (std::nothrow) xct_matrix();
    if (!m) return fail(XCT_ERR_OOM, "host allocation failed");
    m->n = n;
    m->M = n_angles;
    m->C = n_channels;
    m->vdt = value_dtype;
    m->fuse = F;
    m->remap = o.xcd_remap;  // resolved per launch (remap_chunk)
    hipStream_t st = (hipStream_t)stream;
    // host containers may throw; the C ABI returns a status instead
    int rc = XCT_OK;
    try {
        rc = make_grid(m->vol, n, n);
        if (!rc) rc = make_grid(m->sino, n_angles, n_channels);
        if (!rc) {
            ProjRows pr{n, n_angles, n_channels, m->sino.coord_of, m->sino.TW, m->vol.TW, lanes, zero_below};
            HostOrder ho;
            const int nb = (int)((m->sino.n_tiles + W - 1) / W);
            if (o.stage_order == 1)
                order_hilbert(m->vol, ho);
            else
                order_sweep_proj(m, W, nb, ho);
            DevOrder dord;
            rc = upload_order(ho, m->vol.n_tiles, dord);
            if (!rc)
                rc = build_op(m->A, pr, dord.d, m->sino.n_tiles, m->vol.n_tiles, W, T, value_dtype, row_bytes,
                              o.slab_order == 0, st);
        }
        if (!rc) {
            BackRows br{n, n_angles, n_channels, m->vol.coord_of, m->vol.TW, m->sino.TW, lanes, zero_below};
            HostOrder ho;
            if (o.stage_order == 1)
                order_hilbert(m->sino, ho);
            else
                order_raster(m->sino, ho);
            DevOrder dord;
            rc = upload_order(ho, m->sino.n_tiles, dord);
            if (!rc)
                rc = build_op(m->AT, br, dord.d, m->vol.n_tiles, m->sino.n_tiles, W, T, value_dtype, row_bytes,
                              o.slab_order == 0, st);
        }
    } catch (const std::bad_alloc &) {
        rc = fail(XCT_ERR_OOM, "host allocation failed during the build");
    } catch (const std::exception &e) {
        rc = fail(XCT_ERR_INTERNAL, std::string("build: ") + e.what());
    }
    m->A.arith16 = m->AT.arith16 = o.arith == 1 ? 1 : 0;
    m->A.poison = m->AT.poison = o.debug_poison_lds;
    if (rc) {
        std::string msg = g_last_error;
        xct_free_matrix(m);
        g_last_error = msg;
        return rc;
    }
    m->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = m;
    return XCT_OK;
}

static void fill_stats(const OpPlan &op, xct_op_stats &s) {
    s.nnz = op.nnz;
    s.padded = op.padded;
    s.bytes = op.bytes;
    s.stages = op.n_stages;
    s.staged_slots = op.staged_slots;
    s.blocks = op.n_blocks;
    s.tiles_per_stage = op.T;
    s.slabs = op.n_slabs;
    s.balanced_slabs = op.balanced;
}

extern "C" int xct_matrix_info(const xct_matrix *m, xct_matrix_info_t *info) {
    if (!m || !info) return fail(XCT_ERR_INVALID, "NULL argument");
    info->n = m->n;
    info->n_angles = m->M;
    info->n_channels = m->C;
    info->value_dtype = m->vdt;
    info->fuse = m->fuse;
    fill_stats(m->A, info->A);
    fill_stats(m->AT, info->AT);
    info->build_seconds = m->build_seconds;
    return XCT_OK;
}

template <class T>
static int download(std::vector<T> &dst, const T *src, int64_t n) {
    dst.resize((size_t)std::max<int64_t>(n, 0));
    if (n > 0) XCT_HIP_TRY(hipMemcpy(dst.data(), src, sizeof(T) * (size_t)n, hipMemcpyDeviceToHost));
    return XCT_OK;
}

static float half_bits_to_float(uint16_t h) {
    const int e = (h >> 10) & 0x1f, f = h & 0x3ff;
    float v;
    if (e == 0)
        v = std::ldexp((float)f, -24);
    else if (e == 31)
        v = f ? NAN : INFINITY;
    else
        v = std::ldexp((float)(f | 0x400), e - 25);
    return (h & 0x8000) ? -v : v;
}

static float bf16_bits_to_float(uint16_t h) {
    uint32_t u = (uint32_t)h << 16;
    float v;
    std::memcpy(&v, &u, 4);
    return v;
}

static int matrix_to_coo(const xct_matrix *m, int which, int32_t *rows, int32_t *cols, float *vals, int64_t cap,
                         int64_t *count);

extern "C" int xct_matrix_to_coo(const xct_matrix *m, int which, int32_t *rows, int32_t *cols, float *vals,
                                 int64_t cap, int64_t *count) {
    try {  // host copies of the operator may not fit: a status, never an exception
        return matrix_to_coo(m, which, rows, cols, vals, cap, count);
    } catch (const std::bad_alloc &) {
        return fail(XCT_ERR_OOM, "host allocation failed while decoding the operator");
    }
}

static int matrix_to_coo(const xct_matrix *m, int which, int32_t *rows, int32_t *cols, float *vals, int64_t cap,
                         int64_t *count) {
    if (!m || !rows || !cols || !vals || !count) return fail(XCT_ERR_INVALID, "NULL argument");
    if (which != 0 && which != 1) return fail(XCT_ERR_INVALID, "which must be 0 (A) or 1 (A^T)");
    const OpPlan &op = which ? m->AT : m->A;
    const Grid &rg = which ? m->vol : m->sino;
    const Grid &ig = which ? m->sino : m->vol;
    std::vector<int32_t> blk_stage, blk_tile, tile_list, rcoord, icoord;
    std::vector<int64_t> slab;
    std::vector<uint16_t> slot;
    std::vector<float> val;
    std::vector<double> val64;
    std::vector<uint32_t> packed;
    int rc = download(blk_stage, op.blk_stage, op.n_blocks + 1);
    if (!rc) rc = download(blk_tile, op.blk_tile, op.n_blocks + 1);
    if (!rc) rc = download(tile_list, op.tile_list, op.n_list);
    if (!rc) rc = download(slab, op.slab, op.n_stages * op.W + 1);
    if (!rc) rc = download(rcoord, rg.coord_of, rg.n_tiles);
    if (!rc) rc = download(icoord, ig.coord_of, ig.n_tiles);
    if (!rc && m->vdt == XCT_F32) {
        rc = download(slot, op.slot, op.padded * 3);  // the whole buffer, 6 B per entry
        if (!rc) val.assign((float *)slot.data(), (float *)slot.data() + op.padded * 3 / 2);
    } else if (!rc && m->vdt == XCT_F64) {
        rc = download(slot, op.slot, op.padded * 5);  // the whole buffer, 10 B per entry
        if (!rc) val64.assign((double *)slot.data(), (double *)slot.data() + op.padded * 5 / 4);
    } else if (!rc) {
        rc = download(packed, op.packed, op.padded);
    }
    if (rc) return rc;
    int64_t n = 0;
    const int W = op.W, T = op.T;
    for (int b = 0; b < op.n_blocks; ++b) {
        for (int s = blk_stage[b]; s < blk_stage[b + 1]; ++s) {
            const int sl = s - blk_stage[b];
            const int q0 = blk_tile[b] + sl * T;
            const int nt = std::min(T, blk_tile[b + 1] - q0);
            const int nst = blk_stage[b + 1] - blk_stage[b];
            for (int w = 0; w < W; ++w) {
                const int64_t rt = (int64_t)b * W + w;
                const int P = W / op.R;
                const int64_t p = slab_index(blk_stage[b], nst, W, op.R, w % P, w / P, sl);
                for (int64_t g = slab[p]; g < slab[p + 1]; ++g) {
                    for (int lane = 0; lane < kTileSlots; ++lane) {
                        for (int q = 0; q < kGroup; ++q) {
                            const int64_t idx = (g * kTileSlots + lane) * kGroup + q;
                            uint32_t sidx;
                            float v;
                            if (m->vdt == XCT_F32) {
                                const int64_t li = (int64_t)lane * kGroup + q;
                                sidx = slot[g * 768 + li];
                                v = val[g * 384 + 128 + li];
                            } else if (m->vdt == XCT_F64) {
                                const int64_t li = (int64_t)lane * kGroup + q;
                                sidx = slot[g * 1280 + li];
                                v = (float)val64[g * 320 + 64 + li];  // decoded lengths are FP32
                            } else {
                                sidx = packed[idx] >> 16;
                                const uint16_t bits = (uint16_t)(packed[idx] & 0xffff);
                                v = m->vdt == XCT_F16 ? half_bits_to_float(bits) : bf16_bits_to_float(bits);
                            }
                            if (v == 0.0f) {
                                // padding points at one of the first 16 rows (its bank class)
                                if (sidx >= 16) return fail(XCT_ERR_INTERNAL, "padding entry outside rows 0..15");
                                continue;
                            }
                            if (rt >= op.n_row_tiles)
                                return fail(XCT_ERR_INTERNAL, "entry in a padding row tile");
                            const uint32_t logical = sidx;
                            const int pos = (int)(logical / kTileSlots), off = (int)(logical % kTileSlots);
                            if (pos >= nt) return fail(XCT_ERR_INTERNAL, "slot outside its stage");
                            const int rco = rcoord[rt];
                            const int ro = lane_slot(lane, op.lanes);
                            const int r_row = (rco / rg.TW) * kTile + (ro >> 3);
                            const int r_col = (rco % rg.TW) * kTile + (ro & 7);
                            const int ico = icoord[tile_list[q0 + pos]];
                            const int i_row = (ico / ig.TW) * kTile + (off >> 3);
                            const int i_col = (ico % ig.TW) * kTile + (off & 7);
                            if (r_row >= rg.H || r_col >= rg.Wd || i_row >= ig.H || i_col >= ig.Wd)
                                return fail(XCT_ERR_INTERNAL, "entry outside the grid");
                            if (n >= cap) return fail(XCT_ERR_INVALID, "cap too small");
                            rows[n] = r_row * rg.Wd + r_col;
                            cols[n] = i_row * ig.Wd + i_col;
                            vals[n] = v;
                            ++n;
                        }
                    }
                }
            }
        }
    }
    *count = n;
    return XCT_OK;
}
