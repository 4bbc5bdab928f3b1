// GPU construction of the BVH: a linear BVH (Morton order) as the logical
// tree, then packing into one of the node layouts.  The paper fixes the
// topology first and specialises only the physical packing to a layout
// (Sec. 5, two-phase construction); the packing kernels here play the part of
// its generated constructors (count pass, then fill pass, App. F).
#include <algorithm>
#include <array>
#include <cmath>
#include <cstddef>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.h"

namespace bvhlib {
namespace {

constexpr int kBlock = 256;
constexpr int kWave = 64;

struct Box {
    float4 lo;  // w: unused, except in the node boxes (nbox): the node's triangle count
    float4 hi;  // w: unused, except in the node boxes (nbox): its first sorted triangle
};

// The node boxes carry the node's range in their spare words, so a reader of
// a node's box gets its range from the same 32-byte load.
__device__ inline Box with_range(Box b, uint32_t first, uint32_t count) {
    b.lo.w = __uint_as_float(count);
    b.hi.w = __uint_as_float(first);
    return b;
}
__device__ inline uint32_t range_count(const Box &b) { return __float_as_uint(b.lo.w); }
__device__ inline uint32_t range_first(const Box &b) { return __float_as_uint(b.hi.w); }

struct BuildInfo {
    float slo[3], shi[3];   // scene box
    float clo[3], chi[3];   // box of the primitive-box centres
    uint32_t err;           // bit 0: vertex index out of range; bit 1: non-finite extent
    uint32_t n_leaves;      // leaves of the collapsed binary tree
    uint32_t max_depth;     // nodes on the longest root-to-leaf path
    uint32_t max_stack;     // worst-case traversal stack entries
    uint32_t next_count;    // wide packing: size of the next frontier
    uint32_t pad[3];
};

inline unsigned grid_for(uint64_t n, int per_block = kBlock) {
    return (unsigned)((n + per_block - 1) / per_block);
}

// ---------------------------------------------------------------------------
// Wave / block reductions and scans (wave64)
// ---------------------------------------------------------------------------
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan of one value per thread over the block (THREADS threads,
// wsum THREADS / kWave words); *total = block sum.
template <int THREADS = kBlock>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t *total, uint32_t *wsum) {
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    uint32_t inc = wave_incl_scan(v);
    if (lane == kWave - 1) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < THREADS / kWave; i++) {
        uint32_t s = wsum[i];
        off += (i < w) ? s : 0u;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__device__ inline float readlane_t(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline uint32_t readlane_t(uint32_t v, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

// Cross-lane steps through DPP (data-parallel primitives of the VALU: one
// instruction each, no LDS traffic).  dpp<CTRL, ROWS>(old, v) gives each lane
// of the written rows the value v of its source lane, or `old` where the
// source is outside the row; GFX9 controls: row_shl:n = 0x100 + n, row_shr:n
// = 0x110 + n, wave_shl:1 = 0x130, row_bcast:15 = 0x142, row_bcast:31 = 0x143.
template <int CTRL, int ROWS, typename T>
__device__ inline T dpp(T old, T v) {
    static_assert(sizeof(T) == 4, "32-bit lanes");
    return __builtin_bit_cast(T, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, old),
                                                             __builtin_bit_cast(int, v), CTRL,
                                                             ROWS, 0xf, false));
}
// Inclusive scan within each 32-lane half (lanes 0-31 and 32-63): within the
// 16-lane rows, then the last lane of rows 0 and 2 into rows 1 and 3.
template <typename T, typename Op>
__device__ inline T half_scan(T v, T id, Op op) {
    v = op(v, dpp<0x111, 0xf>(id, v));
    v = op(v, dpp<0x112, 0xf>(id, v));
    v = op(v, dpp<0x114, 0xf>(id, v));
    v = op(v, dpp<0x118, 0xf>(id, v));
    return op(v, dpp<0x142, 0xa>(id, v));
}
// Inclusive suffix scan within each 32-lane half: within the rows, then the
// first lane of rows 1 and 3 (their row totals by then) into rows 0 and 2.
template <typename T, typename Op>
__device__ inline T half_suffix_scan(T v, T id, Op op, int lane) {
    v = op(v, dpp<0x101, 0xf>(id, v));
    v = op(v, dpp<0x102, 0xf>(id, v));
    v = op(v, dpp<0x104, 0xf>(id, v));
    v = op(v, dpp<0x108, 0xf>(id, v));
    const T r1 = readlane_t(v, 16), r3 = readlane_t(v, 48);
    if (lane < 16) v = op(v, r1);
    else if (lane >= 32 && lane < 48) v = op(v, r3);
    return v;
}
// Whole-wave reduction: the row scans, the two broadcasts, then lane 63.
template <typename T, typename Op>
__device__ inline T wave_reduce(T v, T id, Op op) {
    v = op(v, dpp<0x111, 0xf>(id, v));
    v = op(v, dpp<0x112, 0xf>(id, v));
    v = op(v, dpp<0x114, 0xf>(id, v));
    v = op(v, dpp<0x118, 0xf>(id, v));
    v = op(v, dpp<0x142, 0xa>(id, v));
    v = op(v, dpp<0x143, 0xc>(id, v));
    return readlane_t(v, 63);
}

__device__ inline float wave_min(float v) {
    return wave_reduce<float>(v, INFINITY, [](float a, float b) { return fminf(a, b); });
}
// Build-wide maxima (stack and depth bounds) without contention: one
// atomicMax per wave into one of kMaxSlots slots chosen by the wave's global
// index, each slot on a cache line of its own, folded by k_fold_max_slots at
// the end.  Device-scope atomics on one word (or one line) from every wave
// of a launch serialise across the XCDs (tens of microseconds per large
// launch); spread over 256 lines they do not.  Every lane of the wave must
// reach the call (lanes with nothing to report pass 0).
constexpr int kMaxSlots = 256;
constexpr int kSlotStride = 32;  // words between slots: one 128-byte line each

__device__ inline void wave_max_to_slots(uint32_t *slots, uint32_t v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, kWave));
    const uint32_t wave = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0 && v)
        atomicMax(&slots[(wave & (kMaxSlots - 1)) * kSlotStride], v);
}

__device__ inline float wave_max(float v) {
    return wave_reduce<float>(v, -INFINITY, [](float a, float b) { return fmaxf(a, b); });
}

// ---------------------------------------------------------------------------
// Exclusive scan of uint32 arrays: per-tile sums, a single-block scan of the
// tile sums, then per-tile scans.  Works in place.
// ---------------------------------------------------------------------------
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__global__ __launch_bounds__(kBlock) void k_scan_reduce(const uint32_t *in, uint32_t n,
                                                        uint32_t *tile_sums) {
    __shared__ uint32_t wsum[kBlock / kWave];
    const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++)
        if (base + k < n) s += in[base + k];
    uint32_t tot;
    block_excl_scan(s, &tot, wsum);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kBlock) void k_scan_tiles(uint32_t *tile_sums, uint32_t ntiles,
                                                       uint32_t *total_out) {
    __shared__ uint32_t wsum[kBlock / kWave];
    uint32_t carry = 0;
    for (uint32_t c = 0; c < ntiles; c += kBlock) {
        const uint32_t i = c + threadIdx.x;
        uint32_t v = i < ntiles ? tile_sums[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_excl_scan(v, &tot, wsum);
        if (i < ntiles) tile_sums[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total_out) {
        *total_out = carry;
        __threadfence_system();  // the total may live in host memory the host polls
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_final(const uint32_t *in, uint32_t *out,
                                                       uint32_t n, const uint32_t *tile_sums) {
    __shared__ uint32_t wsum[kBlock / kWave];
    const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        v[k] = base + k < n ? in[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(s, &tot, wsum) + tile_sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
}

// Short arrays (a few tiles) in one block: tile after tile with a carry.
constexpr uint32_t kScanSingleTiles = 8;

__global__ __launch_bounds__(kBlock) void k_scan_single(const uint32_t *in, uint32_t *out,
                                                        uint32_t n, uint32_t *total_out) {
    __shared__ uint32_t wsum[kBlock / kWave];
    uint32_t carry = 0;
    for (uint32_t c = 0; c < n; c += kScanTile) {
        const uint32_t base = c + threadIdx.x * kScanItems;
        uint32_t v[kScanItems];
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < kScanItems; k++) {
            v[k] = base + k < n ? in[base + k] : 0u;
            sum += v[k];
        }
        uint32_t tot;
        uint32_t run = carry + block_excl_scan(sum, &tot, wsum);
#pragma unroll
        for (int k = 0; k < kScanItems; k++) {
            if (base + k < n) out[base + k] = run;
            run += v[k];
        }
        carry += tot;
        __syncthreads();  // wsum is reused by the next tile
    }
    if (threadIdx.x == 0 && total_out) {
        *total_out = carry;
        __threadfence_system();  // the total may live in host memory the host polls
    }
}

// Middle-sized arrays: after k_scan_reduce, each block adds up the sums of
// the tiles before it itself (a few thousand at most), so no launch sits
// between the two passes; the last block writes the total.
constexpr uint32_t kScanFusedTiles = 4096;

__global__ __launch_bounds__(kBlock) void k_scan_final_fused(const uint32_t *in, uint32_t *out,
                                                             uint32_t n, const uint32_t *tile_sums,
                                                             uint32_t *total_out) {
    __shared__ uint32_t wsum[kBlock / kWave];
    uint32_t part = 0;
    for (uint32_t t = threadIdx.x; t < blockIdx.x; t += kBlock) part += tile_sums[t];
    uint32_t before;
    block_excl_scan(part, &before, wsum);
    const uint32_t base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        v[k] = base + k < n ? in[base + k] : 0u;
        sum += v[k];
    }
    uint32_t tot;
    uint32_t run = before + block_excl_scan(sum, &tot, wsum);
#pragma unroll
    for (int k = 0; k < kScanItems; k++) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0 && total_out) {
        *total_out = before + tot;
        __threadfence_system();  // the total may live in host memory the host polls
    }
}

// Exclusive scan of n values; total (device) receives the sum if non-null.
// tile_sums must hold ceil(n / kScanTile) entries.
void scan_u32(const uint32_t *in, uint32_t *out, uint32_t n, uint32_t *tile_sums,
              uint32_t *total, hipStream_t s) {
    const uint32_t ntiles = (n + kScanTile - 1) / kScanTile;
    if (ntiles <= kScanSingleTiles) {
        k_scan_single<<<1, kBlock, 0, s>>>(in, out, n, total);
        return;
    }
    if (ntiles <= kScanFusedTiles) {
        k_scan_reduce<<<ntiles, kBlock, 0, s>>>(in, n, tile_sums);
        k_scan_final_fused<<<ntiles, kBlock, 0, s>>>(in, out, n, tile_sums, total);
        return;
    }
    if (ntiles > 0) k_scan_reduce<<<ntiles, kBlock, 0, s>>>(in, n, tile_sums);
    k_scan_tiles<<<1, kBlock, 0, s>>>(tile_sums, ntiles, total);
    if (ntiles > 0) k_scan_final<<<ntiles, kBlock, 0, s>>>(in, out, n, tile_sums);
}

// The clears at the start of a build, in one launch: the build info and the
// slot words set to zero, the leaf marks to zero (layouts that mark leaves)
// and the parent links to -1 (where the topology builder does not write every
// one of them).
__global__ __launch_bounds__(kBlock) void k_build_init(BuildInfo *info, uint32_t *slots,
                                                       uint32_t nslots, uint32_t *mark,
                                                       uint32_t nmark, int32_t *parent,
                                                       uint64_t nparent) {
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < sizeof(BuildInfo) / sizeof(uint32_t)) reinterpret_cast<uint32_t *>(info)[i] = 0u;
    if (i < nslots) slots[i] = 0u;
    if (i < nmark) mark[i] = 0u;
    if (i < nparent) parent[i] = -1;
}

// ---------------------------------------------------------------------------
// a1: triangle boxes, scene box and centre box
// ---------------------------------------------------------------------------
// Each thread boxes kPrimItems triangles (block b covers kPrimItems * kBlock
// consecutive ones), so the single-block final reduction reads few partials.
constexpr int kPrimItems = 4;

__global__ __launch_bounds__(kBlock) void k_prim_bounds(const float *verts, int64_t n_verts,
                                                        const int32_t *tris, uint32_t n,
                                                        Box *pbox, float *partial,
                                                        BuildInfo *info) {
    __shared__ float red[12][kBlock / kWave];
    float v[12] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY,
                   INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int item = 0; item < kPrimItems; item++) {
        const uint32_t i = (blockIdx.x * kPrimItems + item) * kBlock + threadIdx.x;
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        float c[3] = {INFINITY, INFINITY, INFINITY}, cm[3] = {-INFINITY, -INFINITY, -INFINITY};
        if (i < n) {
            int32_t idx[3] = {tris[3 * (size_t)i], tris[3 * (size_t)i + 1], tris[3 * (size_t)i + 2]};
            bool ok = true;
            for (int k = 0; k < 3; k++) ok = ok && idx[k] >= 0 && (int64_t)idx[k] < n_verts;
            if (!ok) {
                atomicOr(&info->err, 1u);
                for (int a = 0; a < 3; a++) lo[a] = hi[a] = 0.0f;
            } else {
                for (int k = 0; k < 3; k++) {
                    const float *p = verts + 3 * (size_t)idx[k];
                    for (int a = 0; a < 3; a++) {
                        lo[a] = fminf(lo[a], p[a]);
                        hi[a] = fmaxf(hi[a], p[a]);
                    }
                }
            }
            Box b;
            b.lo = make_float4(lo[0], lo[1], lo[2], 0.0f);
            b.hi = make_float4(hi[0], hi[1], hi[2], 0.0f);
            pbox[i] = b;
            for (int a = 0; a < 3; a++) c[a] = cm[a] = 0.5f * lo[a] + 0.5f * hi[a];
        }
        for (int a = 0; a < 3; a++) {
            v[a] = fminf(v[a], lo[a]);
            v[3 + a] = fmaxf(v[3 + a], hi[a]);
            v[6 + a] = fminf(v[6 + a], c[a]);
            v[9 + a] = fmaxf(v[9 + a], cm[a]);
        }
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int k = 0; k < 12; k++) {
        bool is_min = (k < 3) || (k >= 6 && k < 9);
        float r = is_min ? wave_min(v[k]) : wave_max(v[k]);
        if (lane == 0) red[k][w] = r;
    }
    __syncthreads();
    if (threadIdx.x < 12) {
        const int k = threadIdx.x;
        bool is_min = (k < 3) || (k >= 6 && k < 9);
        float r = red[k][0];
        for (int j = 1; j < kBlock / kWave; j++) r = is_min ? fminf(r, red[k][j]) : fmaxf(r, red[k][j]);
        partial[12 * (size_t)blockIdx.x + k] = r;
    }
}

__global__ __launch_bounds__(kBlock) void k_bounds_final(const float *partial, uint32_t nparts,
                                                         BuildInfo *info) {
    __shared__ float red[12][kBlock / kWave];
    float v[12];
    for (int k = 0; k < 12; k++) {
        bool is_min = (k < 3) || (k >= 6 && k < 9);
        v[k] = is_min ? INFINITY : -INFINITY;
    }
    for (uint32_t p = threadIdx.x; p < nparts; p += kBlock)
        for (int k = 0; k < 12; k++) {
            bool is_min = (k < 3) || (k >= 6 && k < 9);
            float x = partial[12 * (size_t)p + k];
            v[k] = is_min ? fminf(v[k], x) : fmaxf(v[k], x);
        }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int k = 0; k < 12; k++) {
        bool is_min = (k < 3) || (k >= 6 && k < 9);
        float r = is_min ? wave_min(v[k]) : wave_max(v[k]);
        if (lane == 0) red[k][w] = r;
    }
    __syncthreads();
    if (threadIdx.x < 12) {
        const int k = threadIdx.x;
        bool is_min = (k < 3) || (k >= 6 && k < 9);
        float r = red[k][0];
        for (int j = 1; j < kBlock / kWave; j++) r = is_min ? fminf(r, red[k][j]) : fmaxf(r, red[k][j]);
        if (k < 3) info->slo[k] = r;
        else if (k < 6) info->shi[k - 3] = r;
        else if (k < 9) info->clo[k - 6] = r;
        else info->chi[k - 9] = r;
    }
}

// ---------------------------------------------------------------------------
// a2: Morton codes of the box centres, `bits` bits per axis (at most 21).
// The builder uses ceil(log2(n)/3) + 4 bits (one less where that saves a
// sort pass): 2^9 to 2^12 grid cells per triangle, so equal codes are rare,
// and the radix sort only sorts 3*bits bits (four 8-bit passes for two
// million triangles instead of eight).
// ---------------------------------------------------------------------------
__device__ inline uint32_t quantize_axis_bits(float x, float lo, float inv_ext, int bits) {
    const float cells = (float)(1u << bits);
    float u = (x - lo) * inv_ext * cells;
    u = fminf(fmaxf(u, 0.0f), cells - 1.0f);
    return (uint32_t)u;
}

template <typename KeyT>
__global__ __launch_bounds__(kBlock) void k_morton(const Box *pbox, uint32_t n,
                                                   const BuildInfo *info, int bits,
                                                   KeyT *keys, uint32_t *vals) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    Box b = pbox[i];
    float c[3] = {0.5f * b.lo.x + 0.5f * b.hi.x, 0.5f * b.lo.y + 0.5f * b.hi.y,
                  0.5f * b.lo.z + 0.5f * b.hi.z};
    uint32_t q[3];
    for (int a = 0; a < 3; a++) {
        float ext = info->chi[a] - info->clo[a];
        float inv = ext > 0.0f ? 1.0f / ext : 0.0f;
        q[a] = quantize_axis_bits(c[a], info->clo[a], inv, bits);
    }
    // bit k of x, y, z goes to key bit 3k+2, 3k+1, 3k
    uint64_t key = 0;
    for (int bit = 0; bit < bits; bit++) {
        key |= (uint64_t)((q[0] >> bit) & 1u) << (3 * bit + 2);
        key |= (uint64_t)((q[1] >> bit) & 1u) << (3 * bit + 1);
        key |= (uint64_t)((q[2] >> bit) & 1u) << (3 * bit);
    }
    keys[i] = (KeyT)key;  // 3 * bits <= the key width (checked by the caller)
    vals[i] = i;
}

inline int morton_bits(int n) {
    int lg = 0;
    while ((1ll << lg) < (long long)std::max(n, 2)) lg++;
    const int b = std::min(21, std::max(4, (lg + 2) / 3 + 4));
    // one bit per axis less when the last 8-bit sort pass would only sort
    // 1-3 bits (33 bits for two million triangles: 4 passes instead of 5;
    // still 2^9 grid cells per triangle, and the traversal times measured the same)
    const int r = (3 * b) % 8;
    return (r >= 1 && r <= 3 && b > 4) ? b - 1 : b;
}

// ---------------------------------------------------------------------------
// a3: stable LSD radix sort of (u64 key, u32 value), 8 bits per pass.
// Per pass three launches: per-tile digit counts (digit-major matrix), one
// block per digit turning its row into exclusive prefixes over the tiles
// plus the digit's total, and the scatter.  The scatter ranks its tile's
// keys stably in LDS (each wave a contiguous quarter of the tile, equal
// digits found with ballots, no block barrier per round), then writes the
// tile out in local digit order, so consecutive lanes store consecutive
// addresses of a digit's run.
// ---------------------------------------------------------------------------
constexpr int kSortItems = 8;
constexpr int kSortTile = kBlock * kSortItems;
constexpr int kSortWaves = kBlock / kWave;
constexpr int kRadix = 256;
static_assert(kRadix == kBlock, "one digit per thread in the per-digit steps");

template <typename KeyT>
__global__ __launch_bounds__(kBlock) void k_radix_hist(const KeyT *keys, uint32_t n, int shift,
                                                       uint32_t *hist, uint32_t ntiles) {
    __shared__ uint32_t h[kRadix];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * kSortTile;
    for (int k = 0; k < kSortItems; k++) {
        uint32_t i = base + k * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Block d: row d of the count matrix -> exclusive prefix over tiles, in
// place; total[d] = the row's sum.
__global__ __launch_bounds__(kBlock) void k_radix_offsets(uint32_t *hist, uint32_t ntiles,
                                                          uint32_t *total) {
    __shared__ uint32_t wsum[kBlock / kWave];
    uint32_t *row = hist + (size_t)blockIdx.x * ntiles;
    uint32_t carry = 0;
    for (uint32_t c = 0; c < ntiles; c += kBlock) {
        const uint32_t t = c + threadIdx.x;
        const uint32_t v = t < ntiles ? row[t] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, &tot, wsum);
        if (t < ntiles) row[t] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) total[blockIdx.x] = carry;
}

template <typename KeyT>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(const KeyT *keys_in,
                                                          const uint32_t *vals_in,
                                                          KeyT *keys_out, uint32_t *vals_out,
                                                          uint32_t n, int shift,
                                                          const uint32_t *prefix,
                                                          const uint32_t *total,
                                                          uint32_t ntiles) {
    __shared__ KeyT skey[kSortTile];
    __shared__ uint32_t sval[kSortTile];
    __shared__ uint32_t wcount[kSortWaves][kRadix];  // digit counts per wave, then run positions
    __shared__ uint32_t gdst[kRadix];                 // output index of local position 0 of digit d
    __shared__ uint32_t wsum[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    const uint32_t tile = blockIdx.x;
    const uint32_t base = tile * kSortTile;
    const uint32_t wbase = base + (uint32_t)w * (kSortItems * kWave);
#pragma unroll
    for (int k = 0; k < kSortWaves; k++) wcount[k][threadIdx.x] = 0;
    __syncthreads();
    // this wave's quarter of the tile, item r of a lane at wbase + r*64 + lane
    KeyT key[kSortItems];
    uint32_t val[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const uint32_t i = wbase + r * kWave + lane;
        key[r] = i < n ? keys_in[i] : (KeyT)0;
        val[r] = i < n ? vals_in[i] : 0u;
        if (i < n) atomicAdd(&wcount[w][(uint32_t)(key[r] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    {   // thread d: local start of digit d per wave, and its output offset
        const uint32_t d = threadIdx.x;
        uint32_t c[kSortWaves], sum = 0;
#pragma unroll
        for (int k = 0; k < kSortWaves; k++) {
            c[k] = wcount[k][d];
            sum += c[k];
        }
        uint32_t tot_local;
        const uint32_t lstart = block_excl_scan(sum, &tot_local, wsum);
        uint32_t tot_all;
        const uint32_t gstart = block_excl_scan(total[d], &tot_all, wsum);
        gdst[d] = gstart + prefix[(size_t)d * ntiles + tile] - lstart;
        uint32_t run = lstart;
#pragma unroll
        for (int k = 0; k < kSortWaves; k++) {
            wcount[k][d] = run;
            run += c[k];
        }
    }
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    uint32_t *wrun = wcount[w];
#pragma unroll
    for (int r = 0; r < kSortItems; r++) {
        const bool valid = wbase + r * kWave + lane < n;
        const uint32_t d = (uint32_t)(key[r] >> shift) & (kRadix - 1);
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t start = valid ? wrun[d] : 0u;
        __builtin_amdgcn_wave_barrier();
        if (valid) {
            const uint32_t pos = start + (uint32_t)__popcll(peers & lt_mask);
            skey[pos] = key[r];
            sval[pos] = val[r];
            if ((peers & lt_mask) == 0) wrun[d] = start + (uint32_t)__popcll(peers);
        }
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    const uint32_t m = min((uint32_t)kSortTile, n - base);
    for (uint32_t p = threadIdx.x; p < m; p += kBlock) {
        const KeyT k = skey[p];
        const uint32_t o = gdst[(uint32_t)(k >> shift) & (kRadix - 1)] + p;
        if (o < n) {  // always true for a consistent histogram; guards the write
            keys_out[o] = k;
            vals_out[o] = sval[p];
        }
    }
}

// ---------------------------------------------------------------------------
// a4: hierarchy of the sorted codes (Karras 2012).  Internal node i covers a
// key range [first, last] and splits it at the highest differing bit; equal
// keys are separated by their positions.  Node ids: internal i -> i, sorted
// leaf j -> (n - 1) + j; the root is id 0.
// ---------------------------------------------------------------------------
// Sorted keys as seen by one block: keys [w0, w0 + kKarrasWindow) staged in
// LDS (the block's own nodes and a halo on either side, where nearly all of
// the searches land), the rest read from global memory.
constexpr int kKarrasHalo = 512;
constexpr int kKarrasWindow = kBlock + 2 * kKarrasHalo;

template <typename KeyT>
struct KeyWindow {
    const KeyT *g;
    const KeyT *lds;
    int w0;
    __device__ KeyT at(int j) const {
        const unsigned k = (unsigned)(j - w0);
        return k < (unsigned)kKarrasWindow ? lds[k] : g[j];
    }
};

// Length of the common prefix of sorted keys i and j (positions i and j
// appended as tie-breaks), -1 when j is out of range.
__device__ inline int prefix_len(uint64_t a, uint64_t b, int i, int j) {
    if (a != b) return __clzll((long long)(a ^ b));
    return 64 + __clz((int)((uint32_t)i ^ (uint32_t)j));
}
__device__ inline int prefix_len(uint32_t a, uint32_t b, int i, int j) {
    if (a != b) return __clz((int)(a ^ b));
    return 32 + __clz((int)((uint32_t)i ^ (uint32_t)j));
}
template <typename KeyT>
__device__ inline int common_prefix(const KeyWindow<KeyT> &kw, KeyT ki, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    return prefix_len(ki, kw.at(j), i, j);
}

// Node i of the hierarchy; returns how many leaves of the collapsed tree it
// accounts for (see k_karras).
template <typename KeyT>
__device__ inline uint32_t karras_node(const KeyWindow<KeyT> &kw, int n, int i, int32_t *ileft,
                                       int32_t *iright, uint32_t *ifirst, uint32_t *icount,
                                       uint8_t *iaxis, int32_t *parent, int L) {
    const KeyT ki = kw.at(i);
    const int d = (common_prefix(kw, ki, n, i, i + 1) - common_prefix(kw, ki, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = common_prefix(kw, ki, n, i, i - d);
    int lmax = 2;
    while (common_prefix(kw, ki, n, i, i + lmax * d) > dmin) lmax *= 2;
    int l = 0;
    for (int t = lmax / 2; t >= 1; t /= 2)
        if (common_prefix(kw, ki, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = common_prefix(kw, ki, n, i, j);
    int s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (common_prefix(kw, ki, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int gamma = i + s * d + (d < 0 ? -1 : 0);
    const int first = min(i, j), last = max(i, j);
    const int lc = (first == gamma) ? (n - 1) + gamma : gamma;
    const int rc = (last == gamma + 1) ? (n - 1) + gamma + 1 : gamma + 1;
    ileft[i] = lc;
    iright[i] = rc;
    parent[lc] = i;
    parent[rc] = i;
    ifirst[i] = (uint32_t)first;
    icount[i] = (uint32_t)(last - first + 1);
    // split axis: key bit (width - 1) - dnode (bit 3b+2 is x, 3b+1 is y, 3b is z)
    constexpr int kKeyBits = 8 * (int)sizeof(KeyT);
    uint8_t axis = 0;
    if (dnode < kKeyBits) {
        const int p = (kKeyBits - 1) - dnode;
        axis = (p % 3 == 2) ? 0 : (p % 3 == 1 ? 1 : 2);
    }
    iaxis[i] = axis;
    if (i == 0) parent[0] = -1;
    const int cnt = last - first + 1, cl = gamma - first + 1, cr = last - gamma;
    if (cnt > L) return (uint32_t)(cl <= L) + (uint32_t)(cr <= L);
    return (i == 0) ? 1u : 0u;  // the root of at most L primitives is the only leaf
}

// With leaf_slots (the wide layouts): also counts the collapsed tree's leaves
// (leaf size L), which are the children of at most L primitives of the nodes
// of more than L, or the root alone when it holds at most L; per-wave counts
// are added into the kMaxSlots slots a line apart, as in k_count_leaves.
template <typename KeyT>
__global__ __launch_bounds__(kBlock) void k_karras(const KeyT *keys, int n, int32_t *ileft,
                                                   int32_t *iright, uint32_t *ifirst,
                                                   uint32_t *icount, uint8_t *iaxis,
                                                   int32_t *parent, int L, uint32_t *leaf_slots) {
    __shared__ KeyT sk[kKarrasWindow];
    const int w0 = (int)(blockIdx.x * kBlock) - kKarrasHalo;
    for (int k = threadIdx.x; k < kKarrasWindow; k += kBlock) {
        const int j = w0 + k;
        if (j >= 0 && j < n) sk[k] = keys[j];
    }
    __syncthreads();
    const KeyWindow<KeyT> kw{keys, sk, w0};
    const int i = blockIdx.x * kBlock + threadIdx.x;
    uint32_t leaves = 0;
    if (i < n - 1) leaves = karras_node(kw, n, i, ileft, iright, ifirst, icount, iaxis, parent, L);
    if (leaf_slots) {  // every lane of the wave arrives here
        const uint32_t c = (uint32_t)__popcll(__ballot(leaves >= 1)) + (uint32_t)__popcll(__ballot(leaves >= 2));
        const uint32_t wave = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
        if ((threadIdx.x & (kWave - 1)) == 0 && c)
            atomicAdd(&leaf_slots[(wave & (kMaxSlots - 1)) * kSlotStride], c);
    }
}


// ---------------------------------------------------------------------------
// a5: node boxes.  Every node of the hierarchy covers a contiguous range of
// the sorted primitives, so its box is the union of the primitive boxes in
// that range: a range query, answered without any inter-thread
// synchronisation.  Sorted primitive boxes are grouped in blocks of kRangeBlock;
// a sparse table holds the union of 2^k consecutive blocks, so a range is
// its partial blocks (read directly) plus at most two overlapping table
// entries (min/max are idempotent).
// ---------------------------------------------------------------------------
constexpr int kRangeBlock = 64;

__device__ inline Box box_union(const Box &a, const Box &b) {
    Box u;
    u.lo = make_float4(fminf(a.lo.x, b.lo.x), fminf(a.lo.y, b.lo.y), fminf(a.lo.z, b.lo.z), 0.0f);
    u.hi = make_float4(fmaxf(a.hi.x, b.hi.x), fmaxf(a.hi.y, b.hi.y), fmaxf(a.hi.z, b.hi.z), 0.0f);
    return u;
}

__device__ inline Box box_empty() {
    Box e;
    e.lo = make_float4(INFINITY, INFINITY, INFINITY, 0.0f);
    e.hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.0f);
    return e;
}

// Leaf boxes in sorted order (node ids n-1 .. 2n-2) and, one wave per block
// of kRangeBlock: the block union (sparse-table level 0) and the in-block
// prefix and suffix unions (inclusive wave scans).
__device__ inline void wave_scan_box(float *v, bool reverse) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const float t = reverse ? __shfl_down(v[k], o, kWave) : __shfl_up(v[k], o, kWave);
            const bool take = reverse ? (lane + o < kWave) : (lane >= o);
            if (take) v[k] = k < 3 ? fminf(v[k], t) : fmaxf(v[k], t);
        }
    }
}

__device__ inline Box box_of(const float *v) {
    Box u;
    u.lo = make_float4(v[0], v[1], v[2], 0.0f);
    u.hi = make_float4(v[3], v[4], v[5], 0.0f);
    return u;
}

__global__ __launch_bounds__(kBlock) void k_leaf_boxes(const Box *pbox, const uint32_t *perm, int n,
                                                       Box *nbox, Box *table, Box *pre, Box *suf) {
    const int j = blockIdx.x * kBlock + threadIdx.x;
    Box b = box_empty();
    if (j < n) {
        b = pbox[perm[j]];
        nbox[(n - 1) + j] = with_range(b, (uint32_t)j, 1u);
    }
    const float v0[6] = {b.lo.x, b.lo.y, b.lo.z, b.hi.x, b.hi.y, b.hi.z};
    float p[6], q[6];
    for (int k = 0; k < 6; k++) p[k] = q[k] = v0[k];
    wave_scan_box(p, false);
    wave_scan_box(q, true);
    if (j < n) {
        pre[j] = box_of(p);
        suf[j] = box_of(q);
    }
    const int blk = j / kRangeBlock;
    if ((threadIdx.x & (kWave - 1)) == kWave - 1 && blk * kRangeBlock < n) table[blk] = box_of(p);
}

// Sparse-table levels k0 .. k0+m-1 (m <= 3) from level k0-1 in one launch:
// T_{k0-1+d}[i] = union over j < 2^d of T_{k0-1}[i + j 2^(k0-1)], written
// where the entry's 2^(k0-1+d) blocks lie inside the table.
__global__ __launch_bounds__(kBlock) void k_table_levels(Box *table, int nblocks, int k0, int m) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int half = 1 << (k0 - 1);
    const Box *base = table + (size_t)(k0 - 1) * nblocks;
    Box u = box_empty();
    for (int d = 1; d <= m; d++) {
        if (i + (half << d) > nblocks) return;
        // fold in the entries j in [2^(d-1), 2^d)
        for (int j = (d == 1 ? 0 : 1 << (d - 1)); j < (1 << d); j++) u = box_union(u, base[i + j * half]);
        table[(size_t)(k0 - 1 + d) * nblocks + i] = u;
    }
}

// Internal node i's range has i as one end (Karras order) or contains it
// (the SAH ids), so a range inside one 64-block lies within 64 leaves of i:
// the workgroup stages the leaf boxes around its nodes in LDS (coalesced,
// about 1.5 boxes per node) and unions in-block ranges from there; a range
// outside the window (the SAH root's remapped id) reads global memory.
constexpr int kBoxWindow = kBlock + 2 * kRangeBlock;

__global__ __launch_bounds__(kBlock) void k_internal_boxes(const uint32_t *ifirst,
                                                           const uint32_t *icount, int n,
                                                           const Box *table, int nblocks,
                                                           const Box *pre, const Box *suf,
                                                           Box *nbox, float *area) {
    __shared__ float wb[6][kBoxWindow];
    const int i0 = blockIdx.x * kBlock;
    const int wlo = max(0, i0 - kRangeBlock), whi = min(n, i0 + kBlock + kRangeBlock);
    const Box *leaf = nbox + (n - 1);
    for (int j = wlo + (int)threadIdx.x; j < whi; j += kBlock) {
        const Box x = leaf[j];
        wb[0][j - wlo] = x.lo.x;
        wb[1][j - wlo] = x.lo.y;
        wb[2][j - wlo] = x.lo.z;
        wb[3][j - wlo] = x.hi.x;
        wb[4][j - wlo] = x.hi.y;
        wb[5][j - wlo] = x.hi.z;
    }
    __syncthreads();
    const int i = i0 + (int)threadIdx.x;
    if (i >= n - 1) return;
    const int a = (int)ifirst[i], b = a + (int)icount[i] - 1;
    if (a < 0 || b >= n || b < a) {  // malformed range: empty box, the range as given
        nbox[i] = with_range(box_empty(), ifirst[i], icount[i]);
        return;
    }
    const int ba = a / kRangeBlock, bb = b / kRangeBlock;
    Box u = box_empty();
    if (ba == bb && a >= wlo && b < whi) {
        float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
        for (int j = a - wlo; j <= b - wlo; j++) {
#pragma unroll
            for (int c = 0; c < 3; c++) {
                v[c] = fminf(v[c], wb[c][j]);
                v[3 + c] = fmaxf(v[3 + c], wb[3 + c][j]);
            }
        }
        u.lo = make_float4(v[0], v[1], v[2], 0.0f);
        u.hi = make_float4(v[3], v[4], v[5], 0.0f);
    } else if (ba == bb) {
        int j = a;
        for (; j + 3 <= b; j += 4) {
            const Box x0 = leaf[j], x1 = leaf[j + 1], x2 = leaf[j + 2], x3 = leaf[j + 3];
            u = box_union(u, box_union(box_union(x0, x1), box_union(x2, x3)));
        }
        for (; j <= b; j++) u = box_union(u, leaf[j]);
    } else {
        // suffix of a's block, prefix of b's block, whole blocks in between
        u = box_union(suf[a], pre[b]);
        const int lo = ba + 1, hi = bb - 1;
        if (lo <= hi) {
            const int len = hi - lo + 1;
            const int k = 31 - __clz(len);
            const Box *lvl = table + (size_t)k * nblocks;
            u = box_union(u, box_union(lvl[lo], lvl[hi - (1 << k) + 1]));
        }
    }
    nbox[i] = with_range(u, (uint32_t)a, (uint32_t)(b - a + 1));
    const float dx = u.hi.x - u.lo.x, dy = u.hi.y - u.lo.y, dz = u.hi.z - u.lo.z;
    area[i] = dx * dy + dy * dz + dz * dx;
}

// ---------------------------------------------------------------------------
// a6: collapse.  A node is kept ("alive") if it is the root or its parent
// holds more than L triangles; an alive node with at most L triangles is a
// leaf covering its sorted range.  mark[first] = 1 for every leaf.
// ---------------------------------------------------------------------------
struct TreeView {
    int n;                 // triangles
    int leaf_size;
    const int32_t *ileft, *iright, *parent;
    const uint32_t *ifirst, *icount;
    const uint8_t *iaxis;
    const Box *nbox;
    const float *area;     // surface-area measure of internal nodes
    uint32_t *stack_slots;  // kMaxSlots slots each, kSlotStride words apart (zeroed at build start): see wave_max_to_slots
    uint32_t *depth_slots;
    __device__ bool is_prim(int x) const { return x >= n - 1; }
    __device__ uint32_t count(int x) const { return is_prim(x) ? 1u : icount[x]; }
    __device__ uint32_t first(int x) const { return is_prim(x) ? (uint32_t)(x - (n - 1)) : ifirst[x]; }
    __device__ bool alive(int x) const {
        if (x == 0) return true;
        const int p = parent[x];
        return p >= 0 && p < n - 1 && icount[p] > (uint32_t)leaf_size;
    }
    __device__ bool is_leaf(int x) const { return count(x) <= (uint32_t)leaf_size; }
};

__global__ __launch_bounds__(kBlock) void k_mark_leaves(TreeView tv, uint32_t *mark) {
    const int x = blockIdx.x * kBlock + threadIdx.x;
    if (x >= 2 * tv.n - 1) return;
    if (tv.alive(x) && tv.is_leaf(x)) mark[tv.first(x)] = 1u;
}

// The wide layouts need only the number of leaves: per-wave counts added
// into kMaxSlots slots a line apart, then folded into a host-mapped word.
__global__ __launch_bounds__(kBlock) void k_count_leaves(TreeView tv, uint32_t *slots) {
    const int x = blockIdx.x * kBlock + threadIdx.x;
    const bool leaf = x < 2 * tv.n - 1 && tv.alive(x) && tv.is_leaf(x);
    const uint64_t b = __ballot(leaf);
    const uint32_t wave = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if ((threadIdx.x & (kWave - 1)) == 0 && b)
        atomicAdd(&slots[(wave & (kMaxSlots - 1)) * kSlotStride], (uint32_t)__popcll(b));
}

__global__ __launch_bounds__(kBlock) void k_fold_leaf_count(const uint32_t *slots, uint32_t *host_word) {
    __shared__ uint32_t wsum[kBlock / kWave];
    uint32_t v = 0;
    for (int i = threadIdx.x; i < kMaxSlots; i += kBlock) v += slots[i * kSlotStride];
    uint32_t total;
    block_excl_scan(v, &total, wsum);
    if (threadIdx.x == 0) {
        *host_word = total;
        __threadfence_system();  // the host polls the word
    }
}

// ---------------------------------------------------------------------------
// a7 (AABB2): preorder packing.  With leaf_before(x) = number of leaves that
// precede x's range (exclusive scan of mark) and lturns(x) = number of
// left-child steps on the root-to-x path, the preorder index of x in the
// collapsed tree is lturns(x) + 2 * leaf_before(x), and the right child of
// interior x sits 2 * (leaf_before(right) - leaf_before(x)) after x.
// ---------------------------------------------------------------------------
// Writes node x's record; reports its depth and, for a leaf, its stack need.
__device__ inline void emit_aabb2_item(const TreeView &tv, int x, const uint32_t *lbefore,
                                       bvh_node_aabb2 *nodes, uint32_t n_nodes, BuildInfo *info,
                                       uint32_t *depth_out, uint32_t *stack_out) {
    uint32_t lturns = 0, depth = 1;
    for (int y = x; y != 0; depth++) {
        const int p = tv.parent[y];
        if (p < 0 || p >= tv.n - 1 || depth >= 1024) {
            atomicOr(&info->err, 4u);
            return;
        }
        lturns += (tv.ileft[p] == y) ? 1u : 0u;
        y = p;
    }
    const uint32_t f = tv.first(x);
    const uint32_t idx = lturns + 2u * lbefore[f];
    if (idx >= n_nodes) {
        atomicOr(&info->err, 4u);
        return;
    }
    bvh_node_aabb2 nd;
    const Box b = tv.nbox[x];
    nd.lo[0] = b.lo.x; nd.lo[1] = b.lo.y; nd.lo[2] = b.lo.z;
    nd.hi[0] = b.hi.x; nd.hi[1] = b.hi.y; nd.hi[2] = b.hi.z;
    if (tv.is_leaf(x)) {
        nd.offset = f;
        nd.meta = tv.count(x);
    } else {
        const int r = tv.iright[x];
        nd.offset = 2u * (lbefore[tv.first(r)] - lbefore[f]);
        nd.meta = (uint32_t)tv.iaxis[x] << 16;
    }
    nodes[idx] = nd;
    *depth_out = depth;
    if (tv.is_leaf(x)) *stack_out = depth - 1;
}

__global__ __launch_bounds__(kBlock) void k_emit_aabb2(TreeView tv, const uint32_t *lbefore,
                                                       bvh_node_aabb2 *nodes, uint32_t n_nodes,
                                                       BuildInfo *info) {
    const int x = blockIdx.x * kBlock + threadIdx.x;
    uint32_t depth = 0, stack = 0;
    if (x < 2 * tv.n - 1 && tv.alive(x))
        emit_aabb2_item(tv, x, lbefore, nodes, n_nodes, info, &depth, &stack);
    wave_max_to_slots(tv.depth_slots, depth);
    wave_max_to_slots(tv.stack_slots, stack);
}

// ---------------------------------------------------------------------------
// a7 (pbrt-q16): the AABB2 nodes re-encoded with u16 boxes in one frame for
// the whole scene (App. D.3).  The plane value of q is fmaf(q, s, o); each
// box gets the tightest q that still encloses it (as quantize_axis does for
// the wide layouts), and an interior node's split axis goes into the lowest
// bits of its lower x and y planes, lowering a plane by one step where the
// bit differs (which keeps the box enclosing).
// ---------------------------------------------------------------------------
__device__ inline uint32_t q16_lower(float x, float o, float s) {
    if (s == 0.0f) return 0u;
    float f = floorf((x - o) / s);
    f = fminf(fmaxf(f, 0.0f), 65535.0f);
    uint32_t a = (uint32_t)f;
    while (a > 0 && fmaf((float)a, s, o) > x) a--;
    while (a < 65535u && fmaf((float)(a + 1), s, o) <= x) a++;
    return a;
}
__device__ inline uint32_t q16_upper(float x, float o, float s) {
    if (s == 0.0f) return 0u;
    float f = ceilf((x - o) / s);
    f = fminf(fmaxf(f, 0.0f), 65535.0f);
    uint32_t b = (uint32_t)f;
    while (b < 65535u && fmaf((float)b, s, o) < x) b++;
    while (b > 0 && fmaf((float)(b - 1), s, o) >= x) b--;
    return b;
}

struct WorldFrame {
    float o[3], s[3], top[3];
};

// sg-eq (App. D.1): 10-bit steps up from the frame origin (lower planes) and
// down from the frame top (upper planes), tightest enclosing q per plane.
__device__ inline uint32_t q10_lower(float x, float o, float s) {
    if (s == 0.0f) return 0u;
    float f = floorf((x - o) / s);
    f = fminf(fmaxf(f, 0.0f), 1023.0f);
    uint32_t a = (uint32_t)f;
    while (a > 0 && fmaf((float)a, s, o) > x) a--;
    while (a < 1023u && fmaf((float)(a + 1), s, o) <= x) a++;
    return a;
}
__device__ inline uint32_t q10_upper(float x, float top, float s) {
    if (s == 0.0f) return 0u;
    float f = floorf((top - x) / s);
    f = fminf(fmaxf(f, 0.0f), 1023.0f);
    uint32_t b = (uint32_t)f;
    while (b > 0 && fmaf(-(float)b, s, top) < x) b--;
    while (b < 1023u && fmaf(-(float)(b + 1), s, top) >= x) b++;
    return b;
}

// A16: records padded with a zero word to 16 B (SG_EQ_A16).
template <bool A16>
__global__ __launch_bounds__(kBlock) void k_pack_sg_eq(const bvh_node_aabb2 *in, uint32_t n_nodes,
                                                       WorldFrame fr, void *out, BuildInfo *info) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_nodes) return;
    const bvh_node_aabb2 nd = in[i];
    uint32_t lo[3], hi[3];
    for (int a = 0; a < 3; a++) {
        lo[a] = q10_lower(nd.lo[a], fr.o[a], fr.s[a]);
        hi[a] = q10_upper(nd.hi[a], fr.top[a], fr.s[a]);
        if (fr.s[a] != 0.0f && (fmaf((float)lo[a], fr.s[a], fr.o[a]) > nd.lo[a] ||
                                fmaf(-(float)hi[a], fr.s[a], fr.top[a]) < nd.hi[a]))
            atomicOr(&info->err, 4u);
    }
    const uint32_t cnt = nd.meta & 0xFFFFu;
    bvh_node_sg_eq q;
    q.qlo = lo[0] << 20 | lo[1] << 10 | lo[2] | (cnt & 3u) << 30;
    q.qhi = hi[0] << 20 | hi[1] << 10 | hi[2] | (cnt >> 2) << 30;
    q.off = cnt > 0 ? nd.offset : (nd.offset | ((nd.meta >> 16) & 3u) << 30);
    if (A16)
        static_cast<bvh_node_sg_eq_a16 *>(out)[i] = bvh_node_sg_eq_a16{q.qlo, q.qhi, q.off, 0u};
    else
        static_cast<bvh_node_sg_eq *>(out)[i] = q;
}

// Split: boxes to out_box[i], meta words to out_meta[i] (PBRT_Q16_SOAOS);
// otherwise whole records to out[i].
template <bool Split>
__global__ __launch_bounds__(kBlock) void k_pack_pbrt_q16(const bvh_node_aabb2 *in, uint32_t n_nodes,
                                                          WorldFrame fr, bvh_node_pbrt_q16 *out,
                                                          bvh_node_box_q16 *out_box,
                                                          uint32_t *out_meta, BuildInfo *info) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_nodes) return;
    const bvh_node_aabb2 nd = in[i];
    uint32_t lo[3], hi[3];
    for (int a = 0; a < 3; a++) {
        lo[a] = q16_lower(nd.lo[a], fr.o[a], fr.s[a]);
        hi[a] = q16_upper(nd.hi[a], fr.o[a], fr.s[a]);
        // a plane outside the frame (never for a valid build) is reported
        if (fr.s[a] != 0.0f && (fmaf((float)lo[a], fr.s[a], fr.o[a]) > nd.lo[a] ||
                                fmaf((float)hi[a], fr.s[a], fr.o[a]) < nd.hi[a]))
            atomicOr(&info->err, 4u);
    }
    const uint32_t cnt = nd.meta & 0xFFFFu;
    uint32_t meta;
    if (cnt > 0) {
        meta = cnt | (nd.offset << 4);
    } else {
        const uint32_t axis = (nd.meta >> 16) & 3u;
        for (int k = 0; k < 2; k++) {
            const uint32_t bit = (axis >> k) & 1u;
            if ((lo[k] & 1u) != bit && lo[k] > 0) lo[k]--;
        }
        meta = nd.offset << 4;
    }
    if (Split) {
        bvh_node_box_q16 q;
        q.lo[0] = (uint16_t)lo[0]; q.lo[1] = (uint16_t)lo[1]; q.lo[2] = (uint16_t)lo[2];
        q.hi[0] = (uint16_t)hi[0]; q.hi[1] = (uint16_t)hi[1]; q.hi[2] = (uint16_t)hi[2];
        out_box[i] = q;
        out_meta[i] = meta;
    } else {
        bvh_node_pbrt_q16 q;
        q.lo[0] = (uint16_t)lo[0]; q.lo[1] = (uint16_t)lo[1]; q.lo[2] = (uint16_t)lo[2];
        q.hi[0] = (uint16_t)hi[0]; q.hi[1] = (uint16_t)hi[1]; q.hi[2] = (uint16_t)hi[2];
        q.meta = meta;
        out[i] = q;
    }
}

// SHARED_SLAB: node c keeps one slab, the exact extent of its box along the
// axis where that box is narrowest relative to its parent's box (the scene
// box for the root; lowest axis on ties), written by its parent's thread.
__device__ inline bvh_node_slab slab_record(const bvh_node_aabb2 &c, const float *plo,
                                            const float *phi) {
    int axis = 0;
    float best = INFINITY;
    for (int a = 0; a < 3; a++) {
        const float pe = phi[a] - plo[a], ce = c.hi[a] - c.lo[a];
        const float ratio = pe > 0.0f ? ce / pe : 1.0f;
        if (ratio < best) {
            best = ratio;
            axis = a;
        }
    }
    const uint32_t cnt = c.meta & 0xFFFFu, split = (c.meta >> 16) & 3u;
    return bvh_node_slab{c.lo[axis], c.hi[axis], c.offset,
                         cnt | ((uint32_t)axis << 16) | (split << 18)};
}

__global__ __launch_bounds__(kBlock) void k_pack_slab(const bvh_node_aabb2 *in, uint32_t n_nodes,
                                                      const BuildInfo *info, bvh_node_slab *out) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_nodes) return;
    const bvh_node_aabb2 nd = in[i];
    if (i == 0) out[0] = slab_record(nd, info->slo, info->shi);
    if ((nd.meta & 0xFFFFu) != 0u) return;
    const uint32_t kids[2] = {i + 1u, i + nd.offset};
    for (int k = 0; k < 2; k++)
        if (kids[k] < n_nodes) out[kids[k]] = slab_record(in[kids[k]], nd.lo, nd.hi);
}

// AABB2 records split into a box array and a topology array (PBRT_SOAOS).
__global__ __launch_bounds__(kBlock) void k_split_aabb2(const bvh_node_aabb2 *in, uint32_t n_nodes,
                                                        bvh_node_box_f32 *box, bvh_node_topo *topo) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n_nodes) return;
    const bvh_node_aabb2 nd = in[i];
    bvh_node_box_f32 b;
    for (int a = 0; a < 3; a++) {
        b.lo[a] = nd.lo[a];
        b.hi[a] = nd.hi[a];
    }
    box[i] = b;
    topo[i] = bvh_node_topo{nd.offset, nd.meta};
}

// ---------------------------------------------------------------------------
// a7 (wide): top-down, one frontier level per step.  Each frontier item is an
// alive interior binary node that becomes a wide node: its child list starts
// as its two children and repeatedly replaces the interior candidate of
// largest surface area by that candidate's two children, up to K children.
// The list depends only on the binary node, so one launch forms it for every
// alive interior node up front (a chain of dependent loads per node, hidden
// by running all of them at once); per level an exclusive scan of the
// interior-child counts places the children and one pass writes the nodes,
// the next frontier and its counts.
// ---------------------------------------------------------------------------
// Greedy opening of one wide node (binary node x): returns the number of
// interior candidates and writes K candidate ids (-1 for unused slots).
template <int K>
__device__ inline uint32_t wide_open_item(const TreeView &tv, int x, int32_t *cand_out) {
    int c[K];
#pragma unroll
    for (int k = 0; k < K; k++) c[k] = -1;
    int nc;
    if (tv.is_leaf(x)) {  // only for a root that is a single leaf
        c[0] = x;
        nc = 1;
    } else {
        c[0] = tv.ileft[x];
        c[1] = tv.iright[x];
        nc = 2;
        while (nc < K) {
            int best = -1;
            float best_a = -1.0f;
#pragma unroll
            for (int k = 0; k < K; k++) {
                if (k >= nc || tv.is_leaf(c[k])) continue;
                const float a = tv.area[c[k]];
                if (a > best_a) {
                    best_a = a;
                    best = k;
                }
            }
            if (best < 0) break;
            // replace c[best] by its two children, keeping left-to-right order
            int y = -1;
#pragma unroll
            for (int k = 0; k < K; k++)
                if (k == best) y = c[k];
            const int yl = tv.ileft[y], yr = tv.iright[y];
#pragma unroll
            for (int k = K - 1; k >= 1; k--)
                if (k > best + 1 && k <= nc) c[k] = c[k - 1];
#pragma unroll
            for (int k = 0; k < K; k++) {
                if (k == best) c[k] = yl;
                if (k == best + 1) c[k] = yr;
            }
            nc++;
        }
    }
    uint32_t ni = 0, mask = 0;
#pragma unroll
    for (int k = 0; k < K; k++) {
        cand_out[k] = c[k];
        if (c[k] >= 0 && !tv.is_leaf(c[k])) {
            ni++;
            mask |= 1u << k;
        }
    }
    return ni | (mask << 8);
}

// Binary nodes 0 .. m-1 (m = max(n-1, 1)): the root and every alive interior
// node get their child list (cand_all[x*K ..]) and a word with the number of
// interior children (low 8 bits) and which slots hold them (bit 8 + slot).
template <int K>
__global__ __launch_bounds__(kBlock) void k_wide_open_all(TreeView tv, uint32_t m, int32_t *cand_all,
                                                          uint32_t *ni_all) {
    const uint32_t x = blockIdx.x * kBlock + threadIdx.x;
    if (x >= m) return;
    if (x != 0 && !(tv.alive((int)x) && !tv.is_leaf((int)x))) return;
    ni_all[x] = wide_open_item<K>(tv, (int)x, cand_all + (size_t)x * K);
}

// Quantisation of one axis of K child intervals (the first nc valid) to QMAX
// steps of the parent interval [plo, phi].  Returns the scale; q values are
// the tightest with fmaf(qlo, s, plo) <= clo and fmaf(qhi, s, plo) >= chi.
template <int K, int QMAX>
__device__ inline float quantize_axis(float plo, float phi, const float *clo, const float *chi,
                                      int nc, uint32_t *qlo, uint32_t *qhi, uint32_t *err) {
    const float ext = phi - plo;
    float s = 0.0f;
    if (!(ext >= 0.0f) || !isfinite(ext)) {
        atomicOr(err, 2u);
    } else if (ext > 0.0f) {
        s = ext / (float)QMAX;
        for (int g = 0; g < 64 && fmaf((float)QMAX, s, plo) < phi; g++) s = nextafterf(s, INFINITY);
    }
#pragma unroll
    for (int k = 0; k < K; k++) {
        uint32_t a = QMAX, b = 0;  // empty slot: lo above hi
        if (k < nc) {
            if (s == 0.0f) {
                a = 0;
                b = 0;
            } else {
                float fl = floorf((clo[k] - plo) / s);
                fl = fminf(fmaxf(fl, 0.0f), (float)QMAX);
                a = (uint32_t)fl;
                while (a > 0 && fmaf((float)a, s, plo) > clo[k]) a--;
                while (a < (uint32_t)QMAX && fmaf((float)(a + 1), s, plo) <= clo[k]) a++;
                float fh = ceilf((chi[k] - plo) / s);
                fh = fminf(fmaxf(fh, 0.0f), (float)QMAX);
                b = (uint32_t)fh;
                while (b < (uint32_t)QMAX && fmaf((float)b, s, plo) < chi[k]) b++;
                while (b > 0 && fmaf((float)(b - 1), s, plo) >= chi[k]) b--;
            }
        }
        qlo[k] = a;
        qhi[k] = b;
    }
    return s;
}

__device__ inline float box_comp(const Box &b, int c) {
    return c == 0 ? b.lo.x : c == 1 ? b.lo.y : c == 2 ? b.lo.z : c == 3 ? b.hi.x : c == 4 ? b.hi.y : b.hi.z;
}

// Node writers: the record is assembled as 32-bit words in registers (every
// index is a compile-time constant after unrolling) and stored with 16-byte
// stores, so a wave writes whole records instead of one field at a time.
template <int Words>
__device__ inline void store_record(void *dst, const uint32_t *r) {
    static_assert(Words % 4 == 0, "records are whole 16-byte chunks");
    uint4 *d = static_cast<uint4 *>(dst);
#pragma unroll
    for (int i = 0; i < Words / 4; i++)
        d[i] = make_uint4(r[4 * i], r[4 * i + 1], r[4 * i + 2], r[4 * i + 3]);
}

template <int Layout>
struct WideOut;

template <>
struct WideOut<BVH_LAYOUT_BVH4> {
    static constexpr int K = 4;
    static constexpr int kWords = sizeof(bvh_node_bvh4) / 4;
    __device__ static void write(void *dst, const Box &pb, const Box *cb,
                                 const uint32_t *ref, int nc, uint32_t *err) {
        (void)pb;
        (void)err;
        uint32_t r[kWords];
#pragma unroll
        for (int k = 0; k < K; k++) {
            const bool v = k < nc;
            r[0 * K + k] = __float_as_uint(v ? cb[k].lo.x : INFINITY);
            r[1 * K + k] = __float_as_uint(v ? cb[k].lo.y : INFINITY);
            r[2 * K + k] = __float_as_uint(v ? cb[k].lo.z : INFINITY);
            r[3 * K + k] = __float_as_uint(v ? cb[k].hi.x : -INFINITY);
            r[4 * K + k] = __float_as_uint(v ? cb[k].hi.y : -INFINITY);
            r[5 * K + k] = __float_as_uint(v ? cb[k].hi.z : -INFINITY);
            r[6 * K + k] = v ? ref[k] : kRefEmpty;
        }
        r[7 * K] = (uint32_t)nc;
        r[7 * K + 1] = r[7 * K + 2] = r[7 * K + 3] = 0;
        store_record<kWords>(dst, r);
    }
};

// Record words of the quantised 8-wide nodes: origin[3], scale[3], then the
// six plane rows (qlo_x, qlo_y, qlo_z, qhi_x, qhi_y, qhi_z) of RW words each,
// child[8], nchild, zero padding.
template <int QMAX, int RW, int Words>
__device__ inline void quantized_words(uint32_t *r, const Box &pb, const Box *cb, const uint32_t *ref,
                                       int nc, uint32_t *err) {
    constexpr int K = 8;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        float clo[K], chi[K];
        uint32_t qlo[K], qhi[K];
#pragma unroll
        for (int k = 0; k < K; k++) {
            clo[k] = k < nc ? box_comp(cb[k], a) : 0.0f;
            chi[k] = k < nc ? box_comp(cb[k], a + 3) : 0.0f;
        }
        const float plo = box_comp(pb, a), phi = box_comp(pb, a + 3);
        const float sc = quantize_axis<K, QMAX>(plo, phi, clo, chi, nc, qlo, qhi, err);
        r[a] = __float_as_uint(plo);
        r[3 + a] = __float_as_uint(sc);
#pragma unroll
        for (int j = 0; j < RW; j++) {
            const int per = K / RW;  // q values per word: 4 (u8) or 2 (u16)
            uint32_t lo = 0, hi = 0;
#pragma unroll
            for (int t = 0; t < per; t++) {
                lo |= qlo[j * per + t] << (t * (32 / per));
                hi |= qhi[j * per + t] << (t * (32 / per));
            }
            r[6 + a * RW + j] = lo;
            r[6 + (3 + a) * RW + j] = hi;
        }
    }
    constexpr int c0 = 6 + 6 * RW;
#pragma unroll
    for (int k = 0; k < K; k++) r[c0 + k] = k < nc ? ref[k] : kRefEmpty;
    r[c0 + K] = (uint32_t)nc;
#pragma unroll
    for (int k = c0 + K + 1; k < Words; k++) r[k] = 0;
}

static_assert(offsetof(bvh_node_bvh4, child) == 24 * 4 && offsetof(bvh_node_bvh4, nchild) == 28 * 4,
              "bvh4 record words");
static_assert(offsetof(bvh_node_bvh8_q8, qlo_x) == 6 * 4 && offsetof(bvh_node_bvh8_q8, qhi_x) == 12 * 4 &&
                  offsetof(bvh_node_bvh8_q8, child) == 18 * 4 && offsetof(bvh_node_bvh8_q8, nchild) == 26 * 4,
              "bvh8-q8 record words");
static_assert(offsetof(bvh_node_bvh8_q16, qlo_x) == 6 * 4 && offsetof(bvh_node_bvh8_q16, qhi_x) == 18 * 4 &&
                  offsetof(bvh_node_bvh8_q16, child) == 30 * 4 && offsetof(bvh_node_bvh8_q16, nchild) == 38 * 4,
              "bvh8-q16 record words");

template <>
struct WideOut<BVH_LAYOUT_BVH8_Q8> {
    static constexpr int K = 8;
    static constexpr int kWords = sizeof(bvh_node_bvh8_q8) / 4;
    __device__ static void write(void *dst, const Box &pb, const Box *cb,
                                 const uint32_t *ref, int nc, uint32_t *err) {
        uint32_t r[kWords];
        quantized_words<255, 2, kWords>(r, pb, cb, ref, nc, err);
        store_record<kWords>(dst, r);
    }
};

template <>
struct WideOut<BVH_LAYOUT_BVH8_Q16> {
    static constexpr int K = 8;
    static constexpr int kWords = sizeof(bvh_node_bvh8_q16) / 4;
    __device__ static void write(void *dst, const Box &pb, const Box *cb,
                                 const uint32_t *ref, int nc, uint32_t *err) {
        uint32_t r[kWords];
        quantized_words<65535, 4, kWords>(r, pb, cb, ref, nc, err);
        store_record<kWords>(dst, r);
    }
};

// Where wide node w goes: nodes below spec_cap straight into the handle's
// node block (allocated ahead from an earlier build's count), the rest into
// the work area (moved into an exact block after the last level).
struct NodeSink {
    uint8_t *spec;
    uint32_t spec_cap;
    uint8_t *over;
    uint32_t bytes;
    __device__ void *at(uint32_t w) const {
        return w < spec_cap ? spec + (size_t)w * bytes : over + (size_t)w * bytes;
    }
};

// ---------------------------------------------------------------------------
// Wide packing by subtrees.  The wide tree's top levels, while a level holds
// at most kTopMaxFrontier nodes, are planned breadth-first by one workgroup;
// every node of the next level roots a subtree, which one workgroup plans
// breadth-first in a queue of its own.  A subtree's wide nodes number at most
// its primitive count less one (each has two children or more), so its queue
// sits at the subtree root's first primitive position in arrays of n entries,
// and the queues of different subtrees never overlap.  A scan of the subtree
// sizes then places each subtree contiguously after the top levels, and one
// launch over all node positions writes every record (a thread finds its
// subtree by a binary search over the subtree offsets, so uneven subtrees
// do not leave one workgroup with most of the work).  Node order: the top
// levels breadth-first, then subtree by subtree in the order of their roots,
// each breadth-first; a subtree's nodes are thus close together in memory.
// Only the final node count goes to the host.
//
// Plan entries: the binary node x, its aux word (the stack entries its
// ancestors leave behind in the low 16 bits, its depth in the high 16) and
// the queue index of its first interior child (the others follow it).
// ---------------------------------------------------------------------------
constexpr uint32_t kTopMaxFrontier = 1024;
constexpr uint32_t kTopMaxLevels = 64;
constexpr uint32_t kTopMaxNodes = kTopMaxFrontier * kTopMaxLevels;
constexpr int kPlanItems = 4;         // consecutive queue entries per thread and pass
constexpr int kTopThreads = 512;      // the top levels: one workgroup
static_assert(kTopMaxFrontier <= kTopThreads * kPlanItems, "a top level is planned in one pass");
constexpr int kSubThreads = 64;       // a subtree: one wave (its scans need no barrier)
constexpr uint32_t kPlanBlocks = 8192;  // subtree planning: waves, striding over the roots
constexpr int kPlaceThreads = 1024;

struct WidePlan {
    int32_t *t_node;  // top levels, node i at position i (kTopMaxNodes)
    uint32_t *t_aux, *t_noff;
    int32_t *f_node;  // subtree roots (K * kTopMaxFrontier)
    uint32_t *f_aux, *f_size, *f_off, *f_q0;
    int32_t *s_node;  // subtree queues (n entries, by primitive position)
    uint32_t *s_aux, *s_noff;
    uint32_t *meta;   // [0] top nodes, [1] subtrees, [2] all nodes
};

// One pass over queue entries [c, min(c + THREADS * kPlanItems, hi)), kPlanItems
// consecutive ones per thread: their child lists and interior-slot words are
// loaded together, the interior-child counts scanned over the block (child
// indices from `start`), each entry's first-child index stored in qo.  The
// entries stay in registers for plan_children.  Every thread calls it.
template <int K>
struct PlanRegs {
    int32_t cand[kPlanItems][K];
    uint32_t aux[kPlanItems], word[kPlanItems], off[kPlanItems];
};

template <int K, int THREADS>
__device__ inline uint32_t plan_pass(const int32_t *qn, const uint32_t *qa, uint32_t *qo, uint32_t c,
                                     uint32_t hi, uint32_t start, const int32_t *cand_all,
                                     const uint32_t *ni_all, uint32_t *wsum, PlanRegs<K> &R) {
    const uint32_t i0 = c + threadIdx.x * kPlanItems;
    int32_t x[kPlanItems];
#pragma unroll
    for (int k = 0; k < kPlanItems; k++) {
        const bool in = i0 + k < hi;
        x[k] = in ? qn[i0 + k] : -1;
        R.aux[k] = in ? qa[i0 + k] : 0u;
    }
    uint32_t sum = 0;
#pragma unroll
    for (int k = 0; k < kPlanItems; k++) {
        R.word[k] = x[k] >= 0 ? ni_all[x[k]] : 0u;
#pragma unroll
        for (int j = 0; j < K; j++) R.cand[k][j] = x[k] >= 0 ? cand_all[(size_t)x[k] * K + j] : -1;
        sum += R.word[k] & 0xFFu;
    }
    uint32_t tot;
    uint32_t run = start + block_excl_scan<THREADS>(sum, &tot, wsum);
#pragma unroll
    for (int k = 0; k < kPlanItems; k++) {
        R.off[k] = run;
        if (i0 + k < hi) qo[i0 + k] = run;
        run += R.word[k] & 0xFFu;
    }
    return tot;
}

// Appends the pass's interior children (candidate order) at dst[off - dbase].
template <int K>
__device__ inline void plan_children(const PlanRegs<K> &R, uint32_t c, uint32_t hi, int32_t *dst_node,
                                     uint32_t *dst_aux, uint32_t dbase) {
    const uint32_t i0 = c + threadIdx.x * kPlanItems;
#pragma unroll
    for (int k = 0; k < kPlanItems; k++) {
        if (i0 + k >= hi) continue;
        int nc = 0;
#pragma unroll
        for (int j = 0; j < K; j++) nc += R.cand[k][j] >= 0;
        const uint32_t a = R.aux[k];
        const uint32_t caux = (((a & 0xFFFFu) + (uint32_t)(nc - 1)) & 0xFFFFu) | (((a >> 16) + 1) << 16);
        const uint32_t mask = R.word[k] >> 8;
        uint32_t at = R.off[k] - dbase;
#pragma unroll
        for (int j = 0; j < K; j++) {
            if (!((mask >> j) & 1u)) continue;
            dst_node[at] = R.cand[k][j];
            dst_aux[at] = caux;
            at++;
        }
    }
}

template <int K>
__global__ __launch_bounds__(kTopThreads) void k_wide_plan_top(const int32_t *cand_all,
                                                               const uint32_t *ni_all, WidePlan p) {
    __shared__ uint32_t wsum[kTopThreads / kWave];
    if (threadIdx.x == 0) {  // level 0 = {root}, nothing stacked, depth 0
        p.t_node[0] = 0;
        p.t_aux[0] = 0;
    }
    __syncthreads();
    uint32_t lo = 0, hi = 1, total = 0;
    bool frontier = false;
    for (uint32_t level = 0;; level++) {
        PlanRegs<K> R;
        total = plan_pass<K, kTopThreads>(p.t_node, p.t_aux, p.t_noff, lo, hi, hi, cand_all, ni_all,
                                          wsum, R);
        // the same in every thread: the next level becomes the subtree roots
        // when it is too wide for one pass or the top is too deep
        frontier = total > kTopMaxFrontier || level + 1 >= kTopMaxLevels || hi + total > kTopMaxNodes;
        if (frontier)
            plan_children<K>(R, lo, hi, p.f_node, p.f_aux, hi);
        else
            plan_children<K>(R, lo, hi, p.t_node, p.t_aux, 0);
        __syncthreads();
        if (frontier || total == 0) break;
        lo = hi;
        hi += total;
    }
    if (threadIdx.x == 0) {
        p.meta[0] = hi;
        p.meta[1] = frontier ? total : 0u;
    }
}

template <int K>
__global__ __launch_bounds__(kSubThreads) void k_wide_plan_sub(TreeView tv, const int32_t *cand_all,
                                                               const uint32_t *ni_all, WidePlan p,
                                                               BuildInfo *info) {
    __shared__ uint32_t wsum[kSubThreads / kWave];
    const uint32_t roots = p.meta[1];
    for (uint32_t b = blockIdx.x; b < roots; b += gridDim.x) {
        const int32_t x = p.f_node[b];
        const uint32_t q0 = tv.first(x), qcap = tv.count(x);
        int32_t *qn = p.s_node + q0;
        uint32_t *qa = p.s_aux + q0, *qo = p.s_noff + q0;
        if (threadIdx.x == 0) {
            qn[0] = x;
            qa[0] = p.f_aux[b];
            p.f_q0[b] = q0;
        }
        __syncthreads();
        uint32_t lo = 0, hi = 1;
        bool bad = false;
        while (lo < hi && !bad) {
            uint32_t next = hi;
            for (uint32_t c = lo; c < hi; c += kSubThreads * kPlanItems) {
                PlanRegs<K> R;
                const uint32_t tot =
                    plan_pass<K, kSubThreads>(qn, qa, qo, c, hi, next, cand_all, ni_all, wsum, R);
                if (next + tot > qcap) {  // cannot happen (see above): the tree is malformed
                    bad = true;
                    break;
                }
                plan_children<K>(R, c, hi, qn, qa, 0);
                next += tot;
            }
            __syncthreads();
            lo = hi;
            hi = bad ? lo : next;
        }
        if (threadIdx.x == 0) {
            if (bad) atomicOr(&info->err, 4u);
            p.f_size[b] = hi;
        }
    }
}

// Places the subtrees (f_off = absolute position of a subtree's first node)
// and publishes the node count (meta[2] and a host-mapped word).
__global__ __launch_bounds__(kPlaceThreads) void k_wide_place(WidePlan p, uint32_t cap,
                                                              BuildInfo *info, uint32_t *host_word) {
    __shared__ uint32_t wsum[kPlaceThreads / kWave];
    const uint32_t base = p.meta[0], count = p.meta[1];
    uint32_t carry = 0;
    for (uint32_t c = 0; c < count; c += kPlaceThreads * kPlanItems) {
        const uint32_t b0 = c + threadIdx.x * kPlanItems;
        uint32_t v[kPlanItems], sum = 0;
#pragma unroll
        for (int k = 0; k < kPlanItems; k++) {
            v[k] = b0 + k < count ? p.f_size[b0 + k] : 0u;
            sum += v[k];
        }
        uint32_t tot;
        uint32_t run = base + carry + block_excl_scan<kPlaceThreads>(sum, &tot, wsum);
#pragma unroll
        for (int k = 0; k < kPlanItems; k++) {
            if (b0 + k < count) p.f_off[b0 + k] = run;
            run += v[k];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) {
        const uint32_t all = base + carry;
        if (all > cap) atomicOr(&info->err, 4u);
        p.meta[2] = all;
        *host_word = all;
        __threadfence_system();  // the host polls the word
    }
}

// Writes wide node x at position at; pos(r) is the position of its r-th
// interior child.
template <int Layout, typename Pos>
__device__ inline void wide_write(const TreeView &tv, int32_t x, uint32_t aux, uint32_t at,
                                  uint32_t cap, const int32_t *cand, Pos pos, NodeSink sink,
                                  BuildInfo *info, uint32_t *stack_out, uint32_t *depth_out) {
    constexpr int K = WideOut<Layout>::K;
    if (at >= cap) {
        atomicOr(&info->err, 4u);
        return;
    }
    // every load first, so the candidates' loads are issued together
    int c[K];
    Box cb[K];
    uint32_t cnt[K], fst[K];
#pragma unroll
    for (int k = 0; k < K; k++) c[k] = cand[k];  // valid candidates are the first nc slots
#pragma unroll
    for (int k = 0; k < K; k++) {
        cb[k] = box_empty();
        cnt[k] = fst[k] = 0;
        if (c[k] < 0) continue;
        cb[k] = tv.nbox[c[k]];  // box and range in one load
        cnt[k] = range_count(cb[k]);
        fst[k] = range_first(cb[k]);
    }
    uint32_t ref[K];
    int nc = 0;
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < K; k++) {
        ref[k] = kRefEmpty;
        if (c[k] < 0) continue;
        nc++;
        if (cnt[k] <= (uint32_t)tv.leaf_size) {
            ref[k] = ref_leaf(fst[k], cnt[k]);
        } else {
            const uint32_t q = pos(r++);
            if (q >= cap) {
                atomicOr(&info->err, 4u);
                return;
            }
            ref[k] = ref_interior(q);
        }
    }
    WideOut<Layout>::write(sink.at(at), tv.nbox[x], cb, ref, nc, &info->err);
    *stack_out = max(*stack_out, (aux & 0xFFFFu) + (uint32_t)(nc - 1));
    *depth_out = max(*depth_out, (aux >> 16) + 2);  // its children's level and the leaf level below
}

// One thread per node position (launched for the largest possible count).
// The subtree offsets (at most K * kTopMaxFrontier) are staged in LDS for the
// search.
template <int Layout>
__global__ __launch_bounds__(kBlock) void k_wide_write(TreeView tv, const int32_t *cand_all,
                                                       WidePlan p, uint32_t cap, NodeSink sink,
                                                       BuildInfo *info) {
    constexpr int K = WideOut<Layout>::K;
    __shared__ uint32_t s_off[K * kTopMaxFrontier];
    const uint32_t base = p.meta[0], roots = min(p.meta[1], (uint32_t)(K * kTopMaxFrontier)),
                   all = p.meta[2];
    const uint32_t at = blockIdx.x * kBlock + threadIdx.x;
    if (blockIdx.x * kBlock < all && (blockIdx.x + 1) * kBlock > base) {  // the same in the block
        for (uint32_t b = threadIdx.x; b < roots; b += kBlock) s_off[b] = p.f_off[b];
        __syncthreads();
    }
    uint32_t stack = 0, depth = 0;
    if (at < base) {
        const uint32_t no = p.t_noff[at];
        const int32_t x = p.t_node[at];
        // the last top level's children are subtree roots
        wide_write<Layout>(tv, x, p.t_aux[at], at, cap, cand_all + (size_t)x * K,
                           [&](uint32_t r) {
                               const uint32_t j = no + r;
                               return j < base ? j : p.f_off[j - base];
                           },
                           sink, info, &stack, &depth);
    } else if (at < all) {
        // the subtree b with f_off[b] <= at < f_off[b + 1]
        uint32_t lo = 0, hi = roots;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (s_off[mid] <= at) lo = mid; else hi = mid;
        }
        const uint32_t off = s_off[lo];
        const uint32_t q = p.f_q0[lo] + (at - off);
        const uint32_t no = p.s_noff[q];
        const int32_t x = p.s_node[q];
        wide_write<Layout>(tv, x, p.s_aux[q], at, cap, cand_all + (size_t)x * K,
                           [&](uint32_t r) { return off + no + r; }, sink, info, &stack, &depth);
    }
    wave_max_to_slots(tv.stack_slots, stack);
    wave_max_to_slots(tv.depth_slots, depth);
}

// Folds the per-wave maxima slots into info->max_stack / max_depth.
__global__ __launch_bounds__(kBlock) void k_fold_max_slots(const uint32_t *stack_slots,
                                                           const uint32_t *depth_slots,
                                                           BuildInfo *info) {
    __shared__ uint32_t red[2][kBlock / kWave];
    uint32_t a = 0, b = 0;
    for (int i = threadIdx.x; i < kMaxSlots; i += kBlock) {
        a = max(a, stack_slots[i * kSlotStride]);
        b = max(b, depth_slots[i * kSlotStride]);
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        a = max(a, (uint32_t)__shfl_xor((int)a, o, kWave));
        b = max(b, (uint32_t)__shfl_xor((int)b, o, kWave));
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        red[0][threadIdx.x / kWave] = a;
        red[1][threadIdx.x / kWave] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // a, b already hold wave 0's maxima
        for (int w = 1; w < kBlock / kWave; w++) {
            a = max(a, red[0][w]);
            b = max(b, red[1][w]);
        }
        info->max_stack = max(info->max_stack, a);
        info->max_depth = max(info->max_depth, b);
    }
}

// ---------------------------------------------------------------------------
// Leaf data
// ---------------------------------------------------------------------------
// The build reports out-of-range vertex indices only after this kernel has
// run (the wide layouts do not wait for the bounds pass's verdict), so a
// triangle with such an index is written as zeros instead of being read.
__global__ __launch_bounds__(kBlock) void k_leaf_compact(const float *verts, int64_t n_verts,
                                                         const int32_t *tris, const uint32_t *perm,
                                                         uint32_t n, bvh_tri *out) {
    const uint32_t j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= n) return;
    const uint32_t t = perm[j];
    const int32_t i0 = tris[3 * (size_t)t], i1 = tris[3 * (size_t)t + 1], i2 = tris[3 * (size_t)t + 2];
    float p0[3] = {0.f, 0.f, 0.f}, e1[3] = {0.f, 0.f, 0.f}, e2[3] = {0.f, 0.f, 0.f};
    if (i0 >= 0 && i0 < n_verts && i1 >= 0 && i1 < n_verts && i2 >= 0 && i2 < n_verts) {
        const float *q0 = verts + 3 * (size_t)i0;
        const float *q1 = verts + 3 * (size_t)i1;
        const float *q2 = verts + 3 * (size_t)i2;
        for (int a = 0; a < 3; a++) {
            p0[a] = q0[a];
            e1[a] = q1[a] - q0[a];  // the f32 edges of the intersection test
            e2[a] = q2[a] - q0[a];
        }
    }
    // the 48-B record as three 16-B stores
    float4 *o = reinterpret_cast<float4 *>(out + j);
    o[0] = make_float4(p0[0], p0[1], p0[2], e1[0]);
    o[1] = make_float4(e1[1], e1[2], e2[0], e2[1]);
    o[2] = make_float4(e2[2], __int_as_float((int)t), 0.0f, 0.0f);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
// Small host words that kernels write directly (pinned, coherent, mapped into
// the device's address space), one set per host thread.  Polling them lets
// the host learn a count as soon as the kernel that produces it has run,
// while later kernels of the same level are still queued or running, instead
// of waiting for the whole stream and a copy.
constexpr uint32_t kPending = 0xFFFFFFFFu;

uint32_t *host_words() {
    static thread_local void *buf = nullptr;
    if (!buf && hipHostMalloc(&buf, 256, hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
        (void)hipGetLastError();
        buf = nullptr;
    }
    return static_cast<uint32_t *>(buf);
}

// Waits until the kernel-written word p no longer holds kPending.  The wait
// is bounded by the stream: if the stream has finished (or failed) and the
// word is still pending, it reports an error instead of spinning on.
int32_t wait_host_word(volatile uint32_t *p, hipStream_t s, uint32_t *out) {
    for (uint64_t spin = 1;; spin++) {
        const uint32_t v = *p;
        if (v != kPending) {
            *out = v;
            return BVH_OK;
        }
        if ((spin & 255u) == 0) {
            const hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) {
                const uint32_t w = *p;
                if (w != kPending) {
                    *out = w;
                    return BVH_OK;
                }
                return set_error(BVH_EHIP, "bvh_build: internal error (count not written)");
            }
            if (e != hipErrorNotReady) {
                return set_error(BVH_EHIP, "bvh_build: %s", hipGetErrorString(e));
            }
        }
    }
}

// Small pinned host staging area for device-to-host readbacks (one per thread).
template <typename T>
T *pinned_scratch() {
    static thread_local void *buf = nullptr;
    if (!buf && hipHostMalloc(&buf, 256, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        buf = nullptr;
    }
    static_assert(sizeof(T) <= 256, "pinned scratch too small");
    return static_cast<T *>(buf);
}

// Scene frame of the scene-frame quantised layouts: origin and top = scene box
// corners, scale = the smallest step with fmaf(steps, s, o) >= top and
// fmaf(-steps, s, top) <= o (std::fmaf rounds like the device's fmaf).
// Non-finite extents give scale 0 (reported elsewhere).
WorldFrame world_frame(const float *lo, const float *hi, float steps) {
    WorldFrame fr;
    for (int a = 0; a < 3; a++) {
        fr.o[a] = lo[a];
        fr.top[a] = hi[a];
        const float ext = hi[a] - lo[a];
        float sc = 0.0f;
        if (ext > 0.0f && std::isfinite(ext)) {
            sc = ext / steps;
            // full range both ways: up from lo reaches hi, down from hi reaches lo
            for (int g = 0; g < 64 && (std::fmaf(steps, sc, lo[a]) < hi[a] ||
                                       std::fmaf(-steps, sc, hi[a]) > lo[a]); g++)
                sc = std::nextafter(sc, INFINITY);
        }
        fr.s[a] = sc;
    }
    return fr;
}

int32_t check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(BVH_EHIP, "%s: launch failed: %s", what, hipGetErrorString(e));
    return BVH_OK;
}

// The handle's two allocations.  Their hipMalloc calls block the host, so
// the build issues each one while queued kernels keep the GPU busy: the leaf
// block (size known from the input) before the host waits for the leaf
// count, the node block once the leaf data kernels are queued.
int32_t alloc_leaf_block(bvh_handle_s *h) {
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t n = (size_t)h->n_tris;
    const bool compact = h->leaf_mode == BVH_LEAF_COMPACT;
    const size_t b_leaf = up(n * (compact ? sizeof(bvh_tri) : sizeof(int32_t)));
    const size_t b_verts = compact ? 0 : up((size_t)h->n_verts * 3 * sizeof(float));
    const size_t b_tris = compact ? 0 : up(n * 3 * sizeof(int32_t));
    BVH_HIP_TRY(hipMalloc(&h->block, b_leaf + b_verts + b_tris));
    char *p = static_cast<char *>(h->block);
    h->leaf = p;
    if (!compact) {
        h->verts = reinterpret_cast<float *>(p + b_leaf);
        h->tris = reinterpret_cast<int32_t *>(p + b_leaf + b_verts);
    }
    return BVH_OK;
}

int32_t alloc_node_block(bvh_handle_s *h, int64_t n_nodes) {
    BVH_HIP_TRY(hipMalloc(&h->node_block, (size_t)n_nodes * (size_t)h->node_bytes));
    h->node_block_cap = (uint32_t)n_nodes;
    h->nodes = h->node_block;
    return BVH_OK;
}

// Leaf data of the handle (a8): compacted triangles in leaf order, or the
// permutation plus the handle's own copies of the vertices and indices.
struct LeafSource {
    const float *verts;
    int64_t n_verts;
    const int32_t *tris;
    const uint32_t *perm;
    uint32_t n;
};

int32_t emit_leaf_data(bvh_handle_s *h, const LeafSource &ls, hipStream_t s) {
    if (h->leaf_mode == BVH_LEAF_COMPACT) {
        k_leaf_compact<<<grid_for(ls.n), kBlock, 0, s>>>(ls.verts, ls.n_verts, ls.tris, ls.perm,
                                                          ls.n, static_cast<bvh_tri *>(h->leaf));
    } else {
        BVH_HIP_TRY(hipMemcpyAsync(h->leaf, ls.perm, (size_t)ls.n * sizeof(int32_t),
                                   hipMemcpyDeviceToDevice, s));
        BVH_HIP_TRY(hipMemcpyAsync(h->verts, ls.verts, (size_t)ls.n_verts * 3 * sizeof(float),
                                   hipMemcpyDeviceToDevice, s));
        BVH_HIP_TRY(hipMemcpyAsync(h->tris, ls.tris, (size_t)ls.n * 3 * sizeof(int32_t),
                                   hipMemcpyDeviceToDevice, s));
    }
    return check_launch("leaf packing");
}

// Wide node counts of earlier builds, keyed by device, layout, leaf size,
// builder and triangle count.  A build whose key was seen allocates its node
// block up front (count + 1/64 + 64 nodes) while queued kernels run, and
// packs straight into it; without a hint, or when the tree turns out larger,
// the nodes go to the work area and into an exact block after the last level
// (a host-blocking hipMalloc with the GPU idle, then a copy).  Repeated
// builds of one mesh, as in per-frame rebuilds, hit the hint.
class NodeCountHints {
  public:
    using Key = std::array<int64_t, 5>;
    int64_t get(const Key &k) {
        std::lock_guard<std::mutex> g(mu_);
        auto it = map_.find(k);
        return it == map_.end() ? 0 : it->second;
    }
    void put(const Key &k, int64_t v) {
        std::lock_guard<std::mutex> g(mu_);
        if (map_.size() >= kMaxEntries) map_.clear();
        map_[k] = v;
    }

  private:
    static constexpr size_t kMaxEntries = 4096;
    std::mutex mu_;
    std::map<Key, int64_t> map_;
};

NodeCountHints &node_count_hints() {
    static NodeCountHints hints;
    return hints;
}

NodeCountHints::Key node_hint_key(const bvh_handle_s *h) {
    return NodeCountHints::Key{h->device, h->layout, h->leaf_size, h->builder, h->n_tris};
}

// The node block of a wide layout, sized from the hint (none without one);
// called while queued kernels keep the GPU busy.
int32_t alloc_node_block_ahead(bvh_handle_s *h) {
    const int64_t hint = node_count_hints().get(node_hint_key(h));
    if (hint <= 0) return BVH_OK;
    const int64_t want = std::min<int64_t>(std::max<int64_t>(1, h->n_tris - 1), hint + hint / 64 + 64);
    if (hipMalloc(&h->node_block, (size_t)want * h->node_bytes) != hipSuccess) {
        (void)hipGetLastError();  // no block ahead: the exact one comes after packing
        h->node_block = nullptr;
        return BVH_OK;
    }
    h->node_block_cap = (uint32_t)want;
    return BVH_OK;
}

// A second stream per host thread and device (default priority), with two
// events, for build work off the critical path: the leaf data needs only the
// sorted order, so it runs beside the hierarchy and packing kernels, which
// leave much of the GPU idle.  Null stream when creation fails.
struct SideStream {
    hipStream_t stream = nullptr;
    hipEvent_t ready = nullptr, done = nullptr;
};

SideStream *side_stream(int device) {
    static thread_local std::map<int, SideStream> streams;
    SideStream &ss = streams[device];
    if (!ss.stream) {
        if (hipStreamCreateWithFlags(&ss.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ss.ready, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ss.done, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            ss = SideStream{};
            return nullptr;
        }
    }
    return &ss;
}

// The wide packing does not wait for the whole build so far: the leaf data
// and the child lists (which need no count) are queued first, then the host
// reads the leaf count from the word the collapse scan writes (*nleaf_word,
// host-mapped) while those kernels run.  cand_all / ni_all hold max(n-1, 1)
// lists of K.  The plan, placement and writing kernels are queued at once;
// the host waits only for the final node count.
template <int Layout>
int32_t pack_wide(TreeView tv, volatile uint32_t *nleaf_word, int32_t *cand_all, uint32_t *ni_all,
                  BuildInfo *info, bvh_handle_s *h, const LeafSource &ls, hipStream_t s) {
    constexpr int K = WideOut<Layout>::K;
    const uint32_t m = std::max<uint32_t>(1, (uint32_t)tv.n - 1);  // binary nodes with a list
    (void)ls;  // the leaf data is already queued (build_impl, on the side stream)
    k_wide_open_all<K><<<grid_for(m), kBlock, 0, s>>>(tv, m, cand_all, ni_all);
    BVH_TRY(check_launch("wide packing (child lists)"));
    uint32_t n_leaves = 0;
    BVH_TRY(wait_host_word(nleaf_word, s, &n_leaves));
    if (n_leaves < 1 || n_leaves > (uint32_t)tv.n)
        return set_error(BVH_EHIP, "bvh_build: internal error (leaf count %u)", n_leaves);
    h->n_leaves = n_leaves;
    const uint32_t cap = std::max<uint32_t>(1, n_leaves - 1);  // alive interior nodes (or 1)
    constexpr uint32_t kRoots = K * kTopMaxFrontier;
    const size_t nq = std::max<size_t>(1, (size_t)tv.n);
    uint8_t *wnodes;
    WidePlan p;
    Arena arena;
    arena.request(&wnodes, (size_t)cap * h->node_bytes);
    arena.request(&p.t_node, kTopMaxNodes);
    arena.request(&p.t_aux, kTopMaxNodes);
    arena.request(&p.t_noff, kTopMaxNodes);
    arena.request(&p.f_node, kRoots);
    arena.request(&p.f_aux, kRoots);
    arena.request(&p.f_size, kRoots);
    arena.request(&p.f_off, kRoots);
    arena.request(&p.f_q0, kRoots);
    arena.request(&p.s_node, nq);
    arena.request(&p.s_aux, nq);
    arena.request(&p.s_noff, nq);
    arena.request(&p.meta, 4);
    BVH_TRY(arena.bind(s, kAreaBuildWide));
    uint32_t *hw = host_words();
    if (!hw) return set_error(BVH_ENOMEM, "hipHostMalloc failed");
    volatile uint32_t *vw = hw;
    vw[0] = kPending;
    NodeSink sink{static_cast<uint8_t *>(h->node_block), h->node_block ? h->node_block_cap : 0u,
                  wnodes, (uint32_t)h->node_bytes};
    const NodeCountHints::Key key = node_hint_key(h);
    k_wide_plan_top<K><<<1, kTopThreads, 0, s>>>(cand_all, ni_all, p);
    k_wide_plan_sub<K><<<std::min(kRoots, kPlanBlocks), kSubThreads, 0, s>>>(tv, cand_all, ni_all,
                                                                           p, info);
    k_wide_place<<<1, kPlaceThreads, 0, s>>>(p, cap, info, hw);
    k_wide_write<Layout><<<grid_for(cap), kBlock, 0, s>>>(tv, cand_all, p, cap, sink, info);
    // the stack and depth bounds, queued before the host waits for the count
    k_fold_max_slots<<<1, kBlock, 0, s>>>(tv.stack_slots, tv.depth_slots, info);
    BVH_TRY(check_launch("wide packing"));
    uint32_t base = 0;
    BVH_TRY(wait_host_word(vw, s, &base));
    if (base > cap) return set_error(BVH_EHIP, "wide packing overflow");
    h->n_nodes = base;
    // the wide traversal kernels address node fields with 32-bit byte offsets
    if ((uint64_t)base * (uint64_t)h->node_bytes >= (1ull << 32))
        return set_error(BVH_EUNSUPPORTED,
                         "bvh_build: wide node buffer of %llu bytes exceeds 4 GiB (raise leaf_size)",
                         (unsigned long long)base * (unsigned long long)h->node_bytes);
    node_count_hints().put(key, base);
    if (sink.spec && base <= sink.spec_cap) {  // every node is in place
        h->nodes = h->node_block;
        return BVH_OK;
    }
    void *spec = h->node_block;  // too small (or absent): move into an exact block
    h->node_block = nullptr;
    const int32_t rc = alloc_node_block(h, base);
    if (rc == BVH_OK) {
        const size_t nb0 = (size_t)std::min(base, sink.spec_cap) * h->node_bytes;
        const size_t all = (size_t)base * h->node_bytes;
        hipError_t e = hipSuccess;
        if (nb0 > 0) e = hipMemcpyAsync(h->nodes, spec, nb0, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(static_cast<uint8_t *>(h->nodes) + nb0, wnodes + nb0, all - nb0,
                               hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && spec) e = hipStreamSynchronize(s);
        if (spec) (void)hipFree(spec);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_error(BVH_EHIP, "wide packing: node copy failed: %s", hipGetErrorString(e));
        }
        return BVH_OK;
    }
    if (spec) (void)hipFree(spec);
    return rc;
}

// ---------------------------------------------------------------------------
// a4 alternative: binned-SAH topology (32 bins per axis; Sec. 9.2.1).  Top
// down: a node bins its primitives' centroids along each axis over their
// exact bounds, takes the cheapest split A(L) N(L) + A(R) N(R) (A = half
// the surface area of a side's union box; ties to the lower axis, then the
// lower split), and partitions stably; coincident centroids split at the
// index median.  Splitting goes down to single primitives, and the result
// is the same tree view the Karras hierarchy produces (internal nodes
// 0 .. n-2, primitive at leaf position k is node n-1+k, ranges of the
// permutation), so boxes, collapse and packing follow unchanged.
//
// Internal node ids: a node whose split falls between leaf positions m-1
// and m gets id m-1 (unique), except that the root takes id 0 and the node
// with natural id 0 takes the root's natural id.
//
// Large nodes (more than kSahSmall primitives) are processed level by level
// with many blocks each: centroid bounds, binning into per-node global bins,
// one wave per node for the sweep, then a stable partition by one global
// scan.  Nodes of at most kSahSmall primitives are finished by one wave
// each with the primitives held in the lanes.
// ---------------------------------------------------------------------------
constexpr int kSahBins = 32;
constexpr uint32_t kSahSmall = 64;
constexpr uint32_t kSahChunk = 2048;
constexpr int kSahMaxLevels = kStackMax + 1;
constexpr uint32_t kSahBinWords = 3 * kSahBins * 7;  // per node: count + ordered box per bin

struct SahTask {
    uint32_t first, count;
    int32_t parent;  // id of the parent (-1: root)
    uint32_t side;   // 0: left child of the parent, 1: right
};

struct SahSplit {
    int32_t axis;  // split axis (0 for an index-median split)
    int32_t k;     // last bin of the left side (-1: index median)
    uint32_t nl;   // primitives on the left
    uint32_t id;   // the node's id
};

// Floats as order-preserving ints, so min/max can use integer atomics.
__device__ inline int f2o(float f) {
    const int i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__device__ inline float o2f(int i) { return __int_as_float(i >= 0 ? i : i ^ 0x7FFFFFFF); }

__device__ inline float sah_centroid(const Box &b, int a) {
    const float lo = a == 0 ? b.lo.x : (a == 1 ? b.lo.y : b.lo.z);
    const float hi = a == 0 ? b.hi.x : (a == 1 ? b.hi.y : b.hi.z);
    return 0.5f * lo + 0.5f * hi;
}

// Binning frame of one axis: valid when the centroid extent is positive and
// finite; then bin(c) = min(31, trunc((c - lo) * scale)), scale = 32 / ext.
struct SahFrame {
    float4 lo, scale;  // per axis in x, y, z
    uint32_t valid;    // bit a: axis a can be binned
    // the axis is picked among register values, never by indexing memory, so
    // a run-time axis does not send the frame to scratch memory
    __device__ bool ok(int a) const { return (valid >> a) & 1u; }
};

__device__ inline float axis_of(const float4 v, int a) { return a == 0 ? v.x : (a == 1 ? v.y : v.z); }

__device__ inline SahFrame sah_frame(const float *cl, const float *ch) {
    SahFrame f;
    float lo[3], sc[3];
    f.valid = 0;
#pragma unroll
    for (int a = 0; a < 3; a++) {
        const float ext = ch[a] - cl[a];
        const bool v = ext > 0.0f && !isinf(ext);
        f.valid |= (v ? 1u : 0u) << a;
        lo[a] = cl[a];
        sc[a] = v ? __fdiv_rn((float)kSahBins, ext) : 0.0f;
    }
    f.lo = make_float4(lo[0], lo[1], lo[2], 0.0f);
    f.scale = make_float4(sc[0], sc[1], sc[2], 0.0f);
    return f;
}

__device__ inline int sah_bin(const SahFrame f, int a, float c) {
    const float4 lo4 = f.lo, sc4 = f.scale;
    const int b = (int)((c - axis_of(lo4, a)) * axis_of(sc4, a));  // c >= lo: b >= 0 for finite input
    return b < 0 ? 0 : (b < kSahBins - 1 ? b : kSahBins - 1);
}

__device__ inline float half_area3(float lx, float ly, float lz, float hx, float hy, float hz) {
    const float dx = hx - lx, dy = hy - ly, dz = hz - lz;
    return (dx * dy + dy * dz) + dz * dx;
}

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Cheapest split of one axis from its 32 bins (lane k of the wave holds bin
// k: count and box as floats; empty bins hold an empty box).  Returns, in
// every lane, the minimal cost and its split k (the lowest k on ties), or
// +inf when no split leaves both sides non-empty.
__device__ inline void sah_sweep(uint32_t cnt, float lx, float ly, float lz, float hx, float hy,
                                 float hz, float &best_cost, int &best_k, uint32_t &best_nl) {
    const int lane = threadIdx.x & (kWave - 1);
    // inclusive prefix over lanes 0..k and suffix over lanes k..31 (lanes 32-63
    // hold empty bins and scan among themselves)
    const auto add = [](uint32_t x, uint32_t y) { return x + y; };
    const auto mn = [](float x, float y) { return fminf(x, y); };
    const auto mx = [](float x, float y) { return fmaxf(x, y); };
    const uint32_t pc = half_scan<uint32_t>(cnt, 0u, add);
    const uint32_t sc = half_suffix_scan<uint32_t>(cnt, 0u, add, lane);
    const float in[6] = {lx, ly, lz, hx, hy, hz};
    float p[6], q[6];
#pragma unroll
    for (int j = 0; j < 3; j++) {
        p[j] = half_scan<float>(in[j], INFINITY, mn);
        q[j] = half_suffix_scan<float>(in[j], INFINITY, mn, lane);
        p[3 + j] = half_scan<float>(in[3 + j], -INFINITY, mx);
        q[3 + j] = half_suffix_scan<float>(in[3 + j], -INFINITY, mx, lane);
    }
    // right side of split k is the suffix starting at bin k + 1 (wave_shl:1)
    const uint32_t rc = dpp<0x130, 0xf>(0u, sc);
    float r[6];
#pragma unroll
    for (int j = 0; j < 6; j++) r[j] = dpp<0x130, 0xf>(j < 3 ? INFINITY : -INFINITY, q[j]);
    float cost = INFINITY;
    if (lane < kSahBins - 1 && pc > 0 && rc > 0)
        cost = half_area3(p[0], p[1], p[2], p[3], p[4], p[5]) * (float)pc +
               half_area3(r[0], r[1], r[2], r[3], r[4], r[5]) * (float)rc;
    // minimum over the lanes, lowest k on ties
    const float c = wave_min(cost);
    const uint64_t at = __builtin_amdgcn_ballot_w64(lane < kSahBins - 1 && cost == c);
    best_cost = c;
    best_k = (c < INFINITY && at != 0) ? (int)__builtin_ctzll(at) : -1;
    best_nl = readlane_t(pc, best_k < 0 ? 0 : best_k);
}

// Two sweeps at once: the bins of one axis in lanes 0-31 and of another in
// lanes 32-63 (the scans above stay within each half).  Per half: the lowest
// cost, the lowest bin among equal costs (-1 when no split has a finite
// cost) and its left count, exactly as sah_sweep gives them for one axis.
__device__ inline void sah_sweep2(uint32_t cnt, float lx, float ly, float lz, float hx, float hy,
                                  float hz, float &cost0, int &k0, uint32_t &nl0, float &cost1,
                                  int &k1, uint32_t &nl1) {
    const int lane = threadIdx.x & (kWave - 1);
    const int hl = lane & (kSahBins - 1);  // the bin in the lane's half
    const auto add = [](uint32_t x, uint32_t y) { return x + y; };
    const auto mn = [](float x, float y) { return fminf(x, y); };
    const auto mx = [](float x, float y) { return fmaxf(x, y); };
    const uint32_t pc = half_scan<uint32_t>(cnt, 0u, add);
    const uint32_t sc = half_suffix_scan<uint32_t>(cnt, 0u, add, lane);
    const float in[6] = {lx, ly, lz, hx, hy, hz};
    float p[6], q[6];
#pragma unroll
    for (int j = 0; j < 3; j++) {
        p[j] = half_scan<float>(in[j], INFINITY, mn);
        q[j] = half_suffix_scan<float>(in[j], INFINITY, mn, lane);
        p[3 + j] = half_scan<float>(in[3 + j], -INFINITY, mx);
        q[3 + j] = half_suffix_scan<float>(in[3 + j], -INFINITY, mx, lane);
    }
    // the right side of split k is the suffix from bin k + 1 (wave_shl:1;
    // the last bin of each half has no split)
    const uint32_t rc = dpp<0x130, 0xf>(0u, sc);
    float r[6];
#pragma unroll
    for (int j = 0; j < 6; j++) r[j] = dpp<0x130, 0xf>(j < 3 ? INFINITY : -INFINITY, q[j]);
    float cost = INFINITY;
    if (hl < kSahBins - 1 && pc > 0 && rc > 0)
        cost = half_area3(p[0], p[1], p[2], p[3], p[4], p[5]) * (float)pc +
               half_area3(r[0], r[1], r[2], r[3], r[4], r[5]) * (float)rc;
    const float m = half_scan<float>(cost, INFINITY, mn);  // each half's minimum at its last lane
    cost0 = readlane_t(m, kSahBins - 1);
    cost1 = readlane_t(m, kWave - 1);
    const uint64_t at = __builtin_amdgcn_ballot_w64(hl < kSahBins - 1 && cost == (lane < kSahBins ? cost0 : cost1));
    const uint32_t at0 = (uint32_t)at, at1 = (uint32_t)(at >> 32);
    k0 = (cost0 < INFINITY && at0 != 0) ? (int)__builtin_ctz(at0) : -1;
    k1 = (cost1 < INFINITY && at1 != 0) ? (int)__builtin_ctz(at1) : -1;
    nl0 = readlane_t(pc, k0 < 0 ? 0 : k0);
    nl1 = readlane_t(pc, kSahBins + (k1 < 0 ? 0 : k1));
}

// Id of the node that splits at leaf position m (m-1 naturally; see above).
__device__ inline uint32_t sah_node_id(uint32_t m, bool is_root, uint32_t root_nat) {
    if (is_root) return 0u;
    const uint32_t nat = m - 1u;
    return nat == 0u ? root_nat : nat;
}

struct SahTree {
    int32_t *ileft, *iright, *parent;
    uint32_t *ifirst, *icount;
    uint8_t *iaxis;
    int n;
};

// Records node id (range, axis, parent link) and links its leaf children.
__device__ inline void sah_write_node(const SahTree &tr, uint32_t id, uint32_t first,
                                      uint32_t count, int axis, uint32_t nl, int32_t parent,
                                      uint32_t side) {
    tr.ifirst[id] = first;
    tr.icount[id] = count;
    tr.iaxis[id] = (uint8_t)axis;
    tr.parent[id] = parent;
    if (parent >= 0) (side ? tr.iright : tr.ileft)[parent] = (int32_t)id;
    if (nl == 1) {
        const int32_t leaf = tr.n - 1 + (int32_t)first;
        tr.ileft[id] = leaf;
        tr.parent[leaf] = (int32_t)id;
    }
    if (count - nl == 1) {
        const int32_t leaf = tr.n - 1 + (int32_t)(first + nl);
        tr.iright[id] = leaf;
        tr.parent[leaf] = (int32_t)id;
    }
}

// Per-level state of the large-node phase (device).
struct SahLevel {
    const SahTask *task;      // this level's nodes
    const uint32_t *chunk;    // per chunk: task index
    const uint32_t *cstart;   // per chunk: first position
    int *cb;                  // per task: centroid bounds (ordered ints, lo xyz, hi xyz)
    int *bins;                // per task: kSahBinWords
    SahSplit *split;          // per task
    uint32_t ntask;
    const uint32_t *tc0;      // per task: its first chunk (a task's chunks are consecutive)
    int *cbins;               // per chunk: kSahBinWords (the chunk's partial bins)
    int *gbins;               // merge groups > 1: per task and group, kSahBinWords
    uint32_t groups;          // chunk groups per task in the merge (1 or kMergeGroups)
};

// Chunk groups of a task of nch chunks in a level merged with `groups` groups.
__device__ inline uint32_t merge_groups(uint32_t nch, uint32_t groups) { return min(nch, groups); }

__global__ __launch_bounds__(kBlock) void k_sah_clear(int *cb, uint32_t ntask) {
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    const int inf = f2o(INFINITY), ninf = f2o(-INFINITY);
    if (i < (uint64_t)ntask * 6) cb[i] = (i % 6) < 3 ? inf : ninf;
}

__global__ __launch_bounds__(kBlock) void k_sah_bounds(SahLevel lv, const uint32_t *ord,
                                                       const Box *pbox) {
    __shared__ float red[6][kBlock / kWave];
    const uint32_t t = lv.chunk[blockIdx.x];
    const SahTask tk = lv.task[t];
    const uint32_t p0 = lv.cstart[blockIdx.x], p1 = min(p0 + kSahChunk, tk.first + tk.count);
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (uint32_t p = p0 + threadIdx.x; p < p1; p += kBlock) {
        const Box b = pbox[ord[p]];
        for (int a = 0; a < 3; a++) {
            const float c = sah_centroid(b, a);
            v[a] = fminf(v[a], c);
            v[3 + a] = fmaxf(v[3 + a], c);
        }
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    for (int j = 0; j < 6; j++) {
        const float r = j < 3 ? wave_min(v[j]) : wave_max(v[j]);
        if (lane == 0) red[j][w] = r;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int j = threadIdx.x;
        float r = red[j][0];
        for (int k = 1; k < kBlock / kWave; k++) r = j < 3 ? fminf(r, red[j][k]) : fmaxf(r, red[j][k]);
        if (j < 3) atomicMin(&lv.cb[6 * t + j], f2o(r));
        else atomicMax(&lv.cb[6 * t + j], f2o(r));
    }
}

__device__ inline SahFrame sah_task_frame(const int *cb) {
    float cl[3], ch[3];
    for (int a = 0; a < 3; a++) {
        cl[a] = o2f(cb[a]);
        ch[a] = o2f(cb[3 + a]);
    }
    return sah_frame(cl, ch);
}

// Binning of one chunk.  Neighbouring primitives (in the current order)
// mostly fall in one bin, so the lanes of a wave instruction would update the
// same LDS words: the block keeps kBinCopies copies of the bins, lane i using
// copy i % kBinCopies (copies a bank apart), which divides those conflicts by
// kBinCopies; the copies are combined when the chunk is done.
constexpr int kBinCopies = 8;
constexpr int kBinCopyStride = kSahBinWords + 1;  // odd: copies in different banks

__global__ __launch_bounds__(kBlock) void k_sah_bin(SahLevel lv, const uint32_t *ord,
                                                    const Box *pbox) {
    __shared__ int sb[kBinCopies * kBinCopyStride];
    const uint32_t t = lv.chunk[blockIdx.x];
    const SahTask tk = lv.task[t];
    const uint32_t p0 = lv.cstart[blockIdx.x], p1 = min(p0 + kSahChunk, tk.first + tk.count);
    const int inf = f2o(INFINITY), ninf = f2o(-INFINITY);
    for (uint32_t i = threadIdx.x; i < kBinCopies * kBinCopyStride; i += kBlock) {
        const uint32_t w = (i % kBinCopyStride) % 7;
        sb[i] = w == 0 ? 0 : (w <= 3 ? inf : ninf);
    }
    __syncthreads();
    const SahFrame f = sah_task_frame(lv.cb + 6 * t);
    int *mine = sb + (threadIdx.x % kBinCopies) * kBinCopyStride;
    for (uint32_t p = p0 + threadIdx.x; p < p1; p += kBlock) {
        const Box b = pbox[ord[p]];
        for (int a = 0; a < 3; a++) {
            if (!f.ok(a)) continue;
            int *bin = mine + (a * kSahBins + sah_bin(f, a, sah_centroid(b, a))) * 7;
            atomicAdd(bin, 1);
            atomicMin(bin + 1, f2o(b.lo.x));
            atomicMin(bin + 2, f2o(b.lo.y));
            atomicMin(bin + 3, f2o(b.lo.z));
            atomicMax(bin + 4, f2o(b.hi.x));
            atomicMax(bin + 5, f2o(b.hi.y));
            atomicMax(bin + 6, f2o(b.hi.z));
        }
    }
    __syncthreads();
    // the chunk's partial bins, every word (k_sah_merge combines a task's
    // chunks; device atomics from every chunk of a large task into one set of
    // words serialised across the XCDs)
    int *cbin = lv.cbins + (size_t)blockIdx.x * kSahBinWords;
    for (uint32_t i = threadIdx.x; i < kSahBinWords; i += kBlock) {
        const uint32_t kind = i % 7;
        int v = sb[i];
        for (int c = 1; c < kBinCopies; c++) {
            const int x = sb[c * kBinCopyStride + i];
            v = kind == 0 ? v + x : (kind <= 3 ? min(v, x) : max(v, x));
        }
        cbin[i] = v;
    }
}

// bins of task t = the combination of its chunks' partial bins: counts
// added, ordered-int lower corners by minimum, upper corners by maximum (the
// same integers in any order).  Block (t, g) combines chunk group g of task
// t: with one group it writes the task's bins, with several its group's
// partial bins (sah_split_node combines the groups; levels of few, large
// tasks use several, so that one block does not read all the chunks of the
// root).  A task of one chunk is read from its chunk directly.
constexpr uint32_t kMergeGroups = 16;
constexpr uint32_t kMergeGroupTasks = 256;  // most tasks of a level merged with several groups

__device__ inline int bin_combine(uint32_t kind, int v, int x) {
    return kind == 0 ? v + x : (kind <= 3 ? min(v, x) : max(v, x));
}

__global__ __launch_bounds__(kBlock) void k_sah_merge(SahLevel lv) {
    const uint32_t t = blockIdx.x, g = blockIdx.y;
    const uint32_t nch = (lv.task[t].count + kSahChunk - 1) / kSahChunk, c0 = lv.tc0[t];
    const uint32_t ng = merge_groups(nch, lv.groups);
    if (nch < 2 || g >= ng) return;
    const uint32_t j0 = (uint32_t)((uint64_t)g * nch / ng), j1 = (uint32_t)((uint64_t)(g + 1) * nch / ng);
    int *dst = ng > 1 ? lv.gbins + ((size_t)t * kMergeGroups + g) * kSahBinWords
                      : lv.bins + (size_t)t * kSahBinWords;
    for (uint32_t w = threadIdx.x; w < (uint32_t)kSahBinWords; w += kBlock) {
        const int *src = lv.cbins + (size_t)c0 * kSahBinWords + w;
        const uint32_t kind = w % 7;  // 0: count, 1-3: lower corner, 4-6: upper corner
        int v = src[(size_t)j0 * kSahBinWords];
        uint32_t j = j0 + 1;
        for (; j + 4 <= j1; j += 4) {  // four independent loads in flight
            const int x0 = src[(size_t)j * kSahBinWords], x1 = src[(size_t)(j + 1) * kSahBinWords];
            const int x2 = src[(size_t)(j + 2) * kSahBinWords], x3 = src[(size_t)(j + 3) * kSahBinWords];
            v = bin_combine(kind, v, bin_combine(kind, bin_combine(kind, x0, x1), bin_combine(kind, x2, x3)));
        }
        for (; j < j1; j++) v = bin_combine(kind, v, src[(size_t)j * kSahBinWords]);
        dst[w] = v;
    }
}

// The sweep and record of node t (one wave); leaves its task, id and left
// count in tk, id, nl (the same in every lane).
__device__ inline void sah_split_node(SahLevel lv, SahTree tr, uint32_t *root_nat, bool root_level,
                                      uint32_t t, int lane, SahTask &tk, uint32_t &id,
                                      uint32_t &nl_out) {
    tk = lv.task[t];
    const uint32_t nch = (tk.count + kSahChunk - 1) / kSahChunk;
    const uint32_t ng = nch < 2 ? 1u : merge_groups(nch, lv.groups);
    // one chunk: its chunk's bins; several in one group: the merged bins;
    // several groups: the groups' partial bins, combined here
    const int *gb = nch < 2 ? lv.cbins + (size_t)lv.tc0[t] * kSahBinWords
                            : (ng > 1 ? lv.gbins + (size_t)t * kMergeGroups * kSahBinWords
                                      : lv.bins + (size_t)t * kSahBinWords);
    const SahFrame f = sah_task_frame(lv.cb + 6 * t);
    float best = INFINITY;
    int axis = -1, bk = -1;
    uint32_t nl = 0;
    for (int a = 0; a < 3; a++) {
        if (!f.ok(a)) continue;
        const int *bin = gb + (a * kSahBins + (lane < kSahBins ? lane : 0)) * 7;
        const bool in = lane < kSahBins;
        int wv[7];
        for (int j = 0; j < 7; j++) wv[j] = bin[j];
        for (uint32_t g = 1; g < ng; g++)
            for (int j = 0; j < 7; j++) wv[j] = bin_combine((uint32_t)j, wv[j], bin[(size_t)g * kSahBinWords + j]);
        const uint32_t c = in ? (uint32_t)wv[0] : 0u;
        float cost;
        int k;
        uint32_t l;
        sah_sweep(c, in ? o2f(wv[1]) : INFINITY, in ? o2f(wv[2]) : INFINITY,
                  in ? o2f(wv[3]) : INFINITY, in ? o2f(wv[4]) : -INFINITY,
                  in ? o2f(wv[5]) : -INFINITY, in ? o2f(wv[6]) : -INFINITY, cost, k, l);
        if (cost < best) {
            best = cost;
            axis = a;
            bk = k;
            nl = l;
        }
    }
    if (axis < 0) {
        axis = 0;
        bk = -1;
        nl = tk.count / 2;
    }
    const uint32_t m = tk.first + nl;
    if (root_level && lane == 0) *root_nat = m - 1;
    const uint32_t rn = root_level ? m - 1 : *root_nat;
    id = sah_node_id(m, tk.parent < 0, rn);
    nl_out = nl;
    if (lane == 0) {
        lv.split[t] = SahSplit{axis, bk, nl, id};
        sah_write_node(tr, id, tk.first, tk.count, axis, nl, tk.parent, tk.side);
    }
}

// One wave per node: the sweep over the three axes, then the node's id and
// record, and its children: single primitives are linked here, small ones
// queued for the per-wave finisher, large ones queued (with their chunks)
// for the next level.  The queue slots of a block's nodes are taken with one
// device atomic per queue and block (per-node atomics on the three counters
// serialised across the XCDs: 0.2-0.45 ms per level with thousands of nodes).
constexpr int kSplitThreads = 1024;
constexpr int kSplitWaves = kSplitThreads / kWave;

__global__ __launch_bounds__(kSplitThreads) void k_sah_split(SahLevel lv, SahTree tr,
                                                             uint32_t *root_nat, bool root_level,
                                                             SahTask *next, uint32_t *next_chunk,
                                                             uint32_t *next_cstart,
                                                             uint32_t *next_tc0,
                                                             uint32_t *counters, SahTask *small,
                                                             uint32_t *small_count) {
    __shared__ uint32_t need[3][kSplitWaves];  // per wave: small tasks, next tasks, next chunks
    __shared__ uint32_t base[3];
    const int wv = threadIdx.x / kWave;
    const uint32_t t = blockIdx.x * kSplitWaves + wv;
    const bool live = t < lv.ntask;
    const int lane = threadIdx.x & (kWave - 1);
    SahTask tk{0, 0, -1, 0};
    uint32_t id = 0, nl = 0;
    if (live) sah_split_node(lv, tr, root_nat, root_level, t, lane, tk, id, nl);
    // the node's children that need queue slots
    const uint32_t cf[2] = {tk.first, tk.first + nl}, cc[2] = {nl, tk.count - nl};
    uint32_t ns = 0, nn = 0, nc = 0;
    if (live) {
        for (int sd = 0; sd < 2; sd++) {
            if (cc[sd] < 2) continue;
            if (cc[sd] <= kSahSmall) {
                ns++;
            } else {
                nn++;
                nc += (cc[sd] + kSahChunk - 1) / kSahChunk;
            }
        }
    }
    if (lane == 0) {
        need[0][wv] = ns;
        need[1][wv] = nn;
        need[2][wv] = nc;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        uint32_t tot = 0;
        for (int w = 0; w < kSplitWaves; w++) tot += need[threadIdx.x][w];
        uint32_t *ctr = threadIdx.x == 0 ? small_count : &counters[threadIdx.x - 1];
        base[threadIdx.x] = tot ? atomicAdd(ctr, tot) : 0u;
    }
    __syncthreads();
    if (!live || lane != 0) return;
    uint32_t so = base[0], no = base[1], co = base[2];
    for (int w = 0; w < wv; w++) {
        so += need[0][w];
        no += need[1][w];
        co += need[2][w];
    }
    for (int sd = 0; sd < 2; sd++) {
        if (cc[sd] < 2) continue;
        const SahTask ch{cf[sd], cc[sd], (int32_t)id, (uint32_t)sd};
        if (cc[sd] <= kSahSmall) {
            small[so++] = ch;
        } else {
            const uint32_t slot = no++;
            next[slot] = ch;
            next_tc0[slot] = co;
            const uint32_t nch = (cc[sd] + kSahChunk - 1) / kSahChunk;
            for (uint32_t j = 0; j < nch; j++) {
                next_chunk[co + j] = slot;
                next_cstart[co + j] = cf[sd] + j * kSahChunk;
            }
            co += nch;
        }
    }
}


__global__ __launch_bounds__(kBlock) void k_sah_flags(SahLevel lv, const uint32_t *ord,
                                                      const Box *pbox, uint32_t *flags) {
    const uint32_t t = lv.chunk[blockIdx.x];
    const SahTask tk = lv.task[t];
    const SahSplit sp = lv.split[t];
    const uint32_t p0 = lv.cstart[blockIdx.x], p1 = min(p0 + kSahChunk, tk.first + tk.count);
    const SahFrame f = sah_task_frame(lv.cb + 6 * t);
    for (uint32_t p = p0 + threadIdx.x; p < p1; p += kBlock) {
        bool left;
        if (sp.k < 0) left = p - tk.first < sp.nl;
        else left = sah_bin(f, sp.axis, sah_centroid(pbox[ord[p]], sp.axis)) <= sp.k;
        flags[p] = left ? 1u : 0u;
    }
}

__global__ __launch_bounds__(kBlock) void k_sah_scatter(SahLevel lv, const uint32_t *ord,
                                                        const uint32_t *flags, const uint32_t *offs,
                                                        uint32_t *ord_next, uint32_t *perm,
                                                        uint32_t *err) {
    const uint32_t t = lv.chunk[blockIdx.x];
    const SahTask tk = lv.task[t];
    const SahSplit sp = lv.split[t];
    const uint32_t p0 = lv.cstart[blockIdx.x], p1 = min(p0 + kSahChunk, tk.first + tk.count);
    const uint32_t base = offs[tk.first];
    for (uint32_t p = p0 + threadIdx.x; p < p1; p += kBlock) {
        const uint32_t lrank = offs[p] - base;
        const bool left = flags[p] != 0u;
        const uint32_t dst = left ? tk.first + lrank : tk.first + sp.nl + (p - tk.first - lrank);
        if (dst >= tk.first + tk.count || (left ? lrank >= sp.nl : false)) {
            atomicOr(err, 1u);  // the flags disagree with the split's count
            continue;
        }
        const uint32_t prim = ord[p];
        ord_next[dst] = prim;
        const uint32_t child = left ? sp.nl : tk.count - sp.nl;
        if (child <= kSahSmall) perm[dst] = prim;
    }
}

// Finishes nodes of at most kSahSmall primitives, one wave each, with the
// primitives in the lanes (lane i holds position first + i of the node's
// current order).  Subtrees are split in turn from a per-wave stack.
__global__ __launch_bounds__(kBlock) void k_sah_small(const SahTask *small, uint32_t nsmall,
                                                      const Box *pbox, uint32_t *perm, SahTree tr,
                                                      const uint32_t *root_nat_p, uint32_t leaf_size,
                                                      uint32_t *err) {
    constexpr int W = kBlock / kWave;
    __shared__ int sbins[W][kSahBinWords];
    __shared__ uint32_t sstack[W][kSahSmall][4];
    __shared__ float sx[W][kSahSmall][7];  // exchange: prim id bits, box
    const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const uint32_t t = blockIdx.x * W + w;
    if (t >= nsmall) return;
    const SahTask tk = small[t];
    const bool root_task = tk.parent < 0;
    uint32_t root_nat = root_task ? 0u : *root_nat_p;
    uint32_t prim = 0;
    Box b;
    b.lo = make_float4(INFINITY, INFINITY, INFINITY, 0.0f);
    b.hi = make_float4(-INFINITY, -INFINITY, -INFINITY, 0.0f);
    if ((uint32_t)lane < tk.count) {
        prim = perm[tk.first + lane];
        b = pbox[prim];
    }
    int *bins = sbins[w];
    uint32_t sp = 0;
    sstack[w][0][0] = 0;
    sstack[w][0][1] = tk.count;
    sstack[w][0][2] = (uint32_t)tk.parent;
    sstack[w][0][3] = tk.side;
    sp = 1;
    wave_sync();
    while (sp > 0) {
        sp--;
        const uint32_t sf = sstack[w][sp][0], sc = sstack[w][sp][1];
        const int32_t par = (int32_t)sstack[w][sp][2];
        const uint32_t sd = sstack[w][sp][3];
        wave_sync();
        const bool act = (uint32_t)lane >= sf && (uint32_t)lane < sf + sc;
        // a node of at most leaf_size primitives becomes one leaf whatever
        // its subtree: it is split at the index median without binning (no
        // reordering), so only the order inside the leaf differs from a full
        // SAH split
        const bool in_leaf = sc <= leaf_size;
        float cl[3], ch[3], c[3];
        for (int a = 0; a < 3; a++) {
            c[a] = sah_centroid(b, a);
            cl[a] = in_leaf ? 0.0f : wave_min(act ? c[a] : INFINITY);
            ch[a] = in_leaf ? 0.0f : wave_max(act ? c[a] : -INFINITY);
        }
        const SahFrame f = sah_frame(cl, ch);  // no valid axis for a leaf-sized node
        float best = INFINITY;
        int axis = -1, bk = -1;
        uint32_t nl = 0;
        // x and y in one sweep (x's bins in lanes 0-31, y's in lanes 32-63),
        // then z; the costs are compared in axis order with a strict <, so a
        // lower axis wins a tie as when the axes are swept one after another
#pragma unroll
        for (int pass = 0; pass < 2; pass++) {
            const int a0 = pass == 0 ? 0 : 2, a1 = pass == 0 ? 1 : -1;
            const bool v0 = f.ok(a0), v1 = a1 >= 0 && f.ok(a1);
            if (!v0 && !v1) continue;  // the same in the whole wave
            const int inf = f2o(INFINITY), ninf = f2o(-INFINITY);
            {  // lane l clears bin l: the low half's axis, then the high half's
                int *bin = bins + lane * 7;
                bin[0] = 0;
                bin[1] = bin[2] = bin[3] = inf;
                bin[4] = bin[5] = bin[6] = ninf;
            }
            wave_sync();
            if (act) {
                const int qlx = f2o(b.lo.x), qly = f2o(b.lo.y), qlz = f2o(b.lo.z);
                const int qhx = f2o(b.hi.x), qhy = f2o(b.hi.y), qhz = f2o(b.hi.z);
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    if (!(h == 0 ? v0 : v1)) continue;
                    const int a = h == 0 ? a0 : a1;
                    const float ca = a == 0 ? c[0] : (a == 1 ? c[1] : c[2]);
                    int *bin = bins + (h * kSahBins + sah_bin(f, a, ca)) * 7;
                    atomicAdd(bin, 1);
                    atomicMin(bin + 1, qlx);
                    atomicMin(bin + 2, qly);
                    atomicMin(bin + 3, qlz);
                    atomicMax(bin + 4, qhx);
                    atomicMax(bin + 5, qhy);
                    atomicMax(bin + 6, qhz);
                }
            }
            wave_sync();
            const int *bin = bins + lane * 7;
            float cost0, cost1;
            int k0, k1;
            uint32_t l0, l1;
            sah_sweep2((uint32_t)bin[0], o2f(bin[1]), o2f(bin[2]), o2f(bin[3]), o2f(bin[4]),
                       o2f(bin[5]), o2f(bin[6]), cost0, k0, l0, cost1, k1, l1);
            wave_sync();
            if (v0 && cost0 < best) {
                best = cost0;
                axis = a0;
                bk = k0;
                nl = l0;
            }
            if (v1 && cost1 < best) {
                best = cost1;
                axis = a1;
                bk = k1;
                nl = l1;
            }
        }
        bool left;
        if (axis < 0) {
            axis = 0;
            nl = sc / 2;
            left = (uint32_t)lane - sf < nl;
        } else {
            left = sah_bin(f, axis, axis == 0 ? c[0] : (axis == 1 ? c[1] : c[2])) <= bk;
        }
        const uint32_t m = tk.first + sf + nl;
        const bool is_root = root_task && par < 0;
        if (is_root) root_nat = m - 1;
        const uint32_t id = sah_node_id(m, is_root, root_nat);
        if (lane == 0) sah_write_node(tr, id, tk.first + sf, sc, axis, nl, par, sd);
        // stable partition of the active lanes
        const uint64_t lmask = __builtin_amdgcn_ballot_w64(act && left);
        const uint64_t rmask = __builtin_amdgcn_ballot_w64(act && !left);
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        if ((uint32_t)__builtin_popcountll(lmask) != nl) {
            if (lane == 0) atomicOr(err, 1u);  // the lanes disagree with the split's count
            break;
        }
        if (act) {
            const uint32_t dst = left ? sf + (uint32_t)__builtin_popcountll(lmask & below)
                                      : sf + nl + (uint32_t)__builtin_popcountll(rmask & below);
            float *x = sx[w][dst];
            x[0] = __uint_as_float(prim);
            x[1] = b.lo.x; x[2] = b.lo.y; x[3] = b.lo.z;
            x[4] = b.hi.x; x[5] = b.hi.y; x[6] = b.hi.z;
        }
        wave_sync();
        if (act) {
            const float *x = sx[w][lane];
            prim = __float_as_uint(x[0]);
            b.lo = make_float4(x[1], x[2], x[3], 0.0f);
            b.hi = make_float4(x[4], x[5], x[6], 0.0f);
        }
        wave_sync();
        // children of two or more primitives go on the stack
        if (lane == 0) {
            if (sc - nl >= 2) {
                sstack[w][sp][0] = sf + nl;
                sstack[w][sp][1] = sc - nl;
                sstack[w][sp][2] = id;
                sstack[w][sp][3] = 1;
                sp++;
            }
            if (nl >= 2) {
                sstack[w][sp][0] = sf;
                sstack[w][sp][1] = nl;
                sstack[w][sp][2] = id;
                sstack[w][sp][3] = 0;
                sp++;
            }
        }
        sp = (uint32_t)__shfl(sp, 0, kWave);
        wave_sync();
    }
    if ((uint32_t)lane < tk.count) perm[tk.first + lane] = prim;
}

__global__ void k_sah_init(uint32_t *ord, uint32_t *perm, uint32_t n, SahTask *task,
                           uint32_t *chunk, uint32_t *cstart, uint32_t *tc0, SahTask *small,
                           uint32_t *nsmall) {
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        ord[i] = i;
        perm[i] = i;
    }
    if (i == 0) {
        const SahTask root{0u, n, -1, 0u};
        if (n > kSahSmall) {
            task[0] = root;
            tc0[0] = 0;
        } else {
            small[0] = root;
            *nsmall = 1;
        }
    }
    const uint32_t nch = (n + kSahChunk - 1) / kSahChunk;
    if (n > kSahSmall && i < nch) {
        chunk[i] = 0;
        cstart[i] = i * kSahChunk;
    }
}

__global__ void k_sah_publish(const uint32_t *src, uint32_t *dst, int k) {
    if (threadIdx.x == 0) {
        for (int i = 0; i < k; i++) dst[i] = src[i];
        __threadfence_system();
    }
}

// Host side of the binned-SAH topology: fills perm and the tree arrays.
int32_t sah_topology(const Box *pbox, uint32_t n, uint32_t *perm, SahTree tr, uint32_t *tile,
                     int leaf_size, hipStream_t s) {
    if (n < 2) {
        if (n == 1) BVH_HIP_TRY(hipMemsetAsync(perm, 0, sizeof(uint32_t), s));
        return BVH_OK;
    }
    const uint32_t cap_task = n / (kSahSmall + 1) + 1;
    const uint32_t cap_chunk = (n + kSahChunk - 1) / kSahChunk + cap_task;
    uint32_t *ord[2], *flags, *offs, *chunk[2], *cstart[2], *tc0[2], *counters, *small_count,
        *root_nat;
    SahTask *task[2], *small;
    SahSplit *split;
    int *cb, *bins, *cbins, *gbins;
    Arena ar;
    ar.request(&ord[0], n);
    ar.request(&ord[1], n);
    ar.request(&flags, n);
    ar.request(&offs, n);
    ar.request(&task[0], cap_task);
    ar.request(&task[1], cap_task);
    ar.request(&chunk[0], cap_chunk);
    ar.request(&chunk[1], cap_chunk);
    ar.request(&cstart[0], cap_chunk);
    ar.request(&cstart[1], cap_chunk);
    ar.request(&split, cap_task);
    ar.request(&cb, (size_t)cap_task * 6);
    ar.request(&bins, (size_t)cap_task * kSahBinWords);
    ar.request(&cbins, (size_t)cap_chunk * kSahBinWords);
    ar.request(&gbins, (size_t)kMergeGroupTasks * kMergeGroups * kSahBinWords);
    ar.request(&tc0[0], cap_task);
    ar.request(&tc0[1], cap_task);
    ar.request(&small, n / 2 + 1);
    ar.request(&counters, 2 * kSahMaxLevels + 4);
    BVH_TRY(ar.bind(s, kAreaSah));
    small_count = counters + 2 * kSahMaxLevels;
    root_nat = small_count + 1;
    uint32_t *err = small_count + 2;
    BVH_HIP_TRY(hipMemsetAsync(counters, 0, (2 * kSahMaxLevels + 4) * sizeof(uint32_t), s));
    BVH_HIP_TRY(hipMemsetAsync(flags, 0, (size_t)n * sizeof(uint32_t), s));
    k_sah_init<<<grid_for(n), kBlock, 0, s>>>(ord[0], perm, n, task[0], chunk[0], cstart[0], tc0[0],
                                              small, small_count);
    BVH_TRY(check_launch("sah init"));
    uint32_t *hw = host_words();
    if (!hw) return set_error(BVH_ENOMEM, "hipHostMalloc failed");
    volatile uint32_t *vw = hw + 8;
    uint32_t ntask = n > kSahSmall ? 1u : 0u;
    uint32_t nchunk = (n + kSahChunk - 1) / kSahChunk;
    int cur = 0;
    for (int level = 0; ntask > 0; level++) {
        if (level >= kSahMaxLevels)
            return set_error(BVH_EUNSUPPORTED,
                             "bvh_build: SAH tree deeper than the traversal stack bound %d", kStackMax);
        // few tasks with several chunks each: merge them with several groups
        const uint32_t groups = (ntask <= kMergeGroupTasks && nchunk >= 2 * ntask) ? kMergeGroups : 1u;
        SahLevel lv{task[cur], chunk[cur], cstart[cur], cb, bins, split, ntask, tc0[cur], cbins,
                    gbins, groups};
        k_sah_clear<<<grid_for((uint64_t)ntask * 6), kBlock, 0, s>>>(cb, ntask);
        k_sah_bounds<<<nchunk, kBlock, 0, s>>>(lv, ord[cur], pbox);
        k_sah_bin<<<nchunk, kBlock, 0, s>>>(lv, ord[cur], pbox);
        k_sah_merge<<<dim3(ntask, groups), kBlock, 0, s>>>(lv);
        k_sah_split<<<(ntask + kSplitWaves - 1) / kSplitWaves, kSplitThreads, 0, s>>>(
            lv, tr, root_nat, level == 0, task[cur ^ 1], chunk[cur ^ 1], cstart[cur ^ 1],
            tc0[cur ^ 1], counters + 2 * level, small, small_count);
        k_sah_flags<<<nchunk, kBlock, 0, s>>>(lv, ord[cur], pbox, flags);
        scan_u32(flags, offs, n, tile, nullptr, s);
        k_sah_scatter<<<nchunk, kBlock, 0, s>>>(lv, ord[cur], flags, offs, ord[cur ^ 1], perm, err);
        vw[0] = vw[1] = kPending;
        k_sah_publish<<<1, 64, 0, s>>>(counters + 2 * level, hw + 8, 2);
        BVH_TRY(check_launch("sah level"));
        BVH_TRY(wait_host_word(vw, s, &ntask));
        BVH_TRY(wait_host_word(vw + 1, s, &nchunk));
        if (ntask > cap_task || nchunk > cap_chunk)
            return set_error(BVH_EHIP, "bvh_build: internal error (SAH task overflow)");
        cur ^= 1;
    }
    vw[2] = kPending;
    k_sah_publish<<<1, 64, 0, s>>>(small_count, hw + 10, 1);
    uint32_t nsmall = 0;
    BVH_TRY(wait_host_word(vw + 2, s, &nsmall));
    if (nsmall > n / 2 + 1) return set_error(BVH_EHIP, "bvh_build: internal error (SAH small overflow)");
    if (nsmall > 0)
        k_sah_small<<<(nsmall + kBlock / kWave - 1) / (kBlock / kWave), kBlock, 0, s>>>(
            small, nsmall, pbox, perm, tr, root_nat, (uint32_t)leaf_size, err);
    vw[3] = kPending;
    k_sah_publish<<<1, 64, 0, s>>>(err, hw + 11, 1);
    BVH_TRY(check_launch("sah small nodes"));
    uint32_t bad = 0;
    BVH_TRY(wait_host_word(vw + 3, s, &bad));
    if (bad) return set_error(BVH_EHIP, "bvh_build: internal error (SAH partition)");
    return BVH_OK;
}

// a2, a3: Morton keys of the box centres, then a stable LSD radix sort of
// (key, primitive index), 8 bits per pass over the 3 * mbits key bits;
// returns which of the two buffers holds the sorted pairs.
template <typename KeyT>
int sort_morton(const Box *pbox, uint32_t n, const BuildInfo *info, int mbits, KeyT **keys,
                uint32_t **vals, uint32_t *hist, uint32_t nsort, hipStream_t s) {
    const uint32_t nhist = nsort * kRadix;
    k_morton<<<grid_for(n), kBlock, 0, s>>>(pbox, n, info, mbits, keys[0], vals[0]);
    int cur = 0;
    for (int shift = 0; shift < 3 * mbits; shift += 8) {
        k_radix_hist<<<nsort, kBlock, 0, s>>>(keys[cur], n, shift, hist, nsort);
        k_radix_offsets<<<kRadix, kBlock, 0, s>>>(hist, nsort, hist + nhist);
        k_radix_scatter<<<nsort, kBlock, 0, s>>>(keys[cur], vals[cur], keys[cur ^ 1],
                                                 vals[cur ^ 1], n, shift, hist, hist + nhist,
                                                 nsort);
        cur ^= 1;
    }
    return cur;
}

int32_t build_impl(const float *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                   bvh_handle_s *h, hipStream_t s) {
    const int n = (int)n_tris;
    const int L = h->leaf_size;

    Box *pbox, *nbox;
    float *partial;
    BuildInfo *info;
    uint64_t *keys[2];
    uint32_t *vals[2], *hist, *tile, *ifirst, *icount, *mark;
    int32_t *ileft, *iright, *parent;
    uint8_t *iaxis;
    const uint32_t nb = grid_for(n);
    const uint32_t nsort = (uint32_t)((n + kSortTile - 1) / kSortTile);
    const uint32_t nhist = nsort * kRadix;
    const uint32_t max_scan = std::max<uint32_t>(nhist, (uint32_t)n);
    const int nblocks = (n + kRangeBlock - 1) / kRangeBlock;
    int levels = 1;
    while ((1 << levels) <= nblocks) levels++;
    Box *table, *pre, *suf;
    float *area;
    Arena arena;
    arena.request(&pbox, n);
    arena.request(&partial, (size_t)nb * 12);
    arena.request(&info, 1);
    arena.request(&keys[0], n);
    arena.request(&keys[1], n);
    arena.request(&vals[0], n);
    arena.request(&vals[1], n);
    arena.request(&hist, nhist + kRadix);  // counts, then the digit totals
    arena.request(&tile, (max_scan + kScanTile - 1) / kScanTile + 1);
    arena.request(&ileft, n - 1);
    arena.request(&iright, n - 1);
    arena.request(&ifirst, n - 1);
    arena.request(&icount, n - 1);
    arena.request(&iaxis, n - 1);
    arena.request(&parent, 2 * (size_t)n - 1);
    arena.request(&nbox, 2 * (size_t)n - 1);
    arena.request(&mark, n);
    arena.request(&table, (size_t)levels * nblocks);
    arena.request(&pre, n);
    arena.request(&suf, n);
    arena.request(&area, n - 1);
    uint32_t *bound_slots;
    arena.request(&bound_slots, 3 * kMaxSlots * kSlotStride);  // stack, depth, leaf-count slots
    int32_t *cand_all = nullptr;  // wide layouts: the child list of every binary node
    uint32_t *ni_all = nullptr;
    if (layout_arity(h->layout) > 2) {
        const size_t m = (size_t)std::max(1, n - 1);
        arena.request(&cand_all, m * (size_t)layout_arity(h->layout));
        arena.request(&ni_all, m);
    }
    BVH_TRY(arena.bind(s, kAreaBuild));

    const bool wide = h->layout == BVH_LAYOUT_BVH4 || h->layout == BVH_LAYOUT_BVH8_Q8 ||
                      h->layout == BVH_LAYOUT_BVH8_Q16;
    {
        // k_karras writes the parent of every node (the root's too) when n > 1
        const uint32_t nslots = 3 * kMaxSlots * kSlotStride;
        const uint32_t nmark = wide ? 0u : (uint32_t)n;
        const uint64_t nparent =
            (h->builder == BVH_BUILDER_SAH || n == 1) ? 2 * (uint64_t)n - 1 : 0u;
        const uint64_t m = std::max<uint64_t>(std::max<uint64_t>(nslots, nmark), nparent);
        k_build_init<<<grid_for(m), kBlock, 0, s>>>(info, bound_slots, nslots, mark, nmark, parent,
                                                    nparent);
    }

    // a1, a2
    const uint32_t nbp = (uint32_t)(((uint64_t)n + kPrimItems * kBlock - 1) / (kPrimItems * kBlock));
    k_prim_bounds<<<nbp, kBlock, 0, s>>>(verts, n_verts, tris, n, pbox, partial, info);
    k_bounds_final<<<1, kBlock, 0, s>>>(partial, nbp, info);
    const uint32_t *perm = nullptr;
    SideStream *side = nullptr;
    // a8 leaf data for the wide layouts, queued as soon as the order is final,
    // on the side stream: the leaf block's hipMalloc (and the node block's,
    // from the hint) block the host while the queued kernels run, then the
    // leaf kernel overlaps the hierarchy kernels
    // the point of the stream after which the sorted order is final: the
    // side stream's leaf data waits for it (and not for the kernels queued
    // on the build stream after it)
    bool sorted_marked = false;
    auto mark_sorted = [&]() -> int32_t {
        if (!wide || sorted_marked) return BVH_OK;
        sorted_marked = true;
        side = side_stream(h->device);
        if (side) BVH_HIP_TRY(hipEventRecord(side->ready, s));
        return BVH_OK;
    };
    auto leaf_data_early = [&]() -> int32_t {
        if (!wide) return BVH_OK;
        BVH_TRY(mark_sorted());
        BVH_TRY(alloc_leaf_block(h));
        BVH_TRY(alloc_node_block_ahead(h));
        const LeafSource early{verts, n_verts, tris, perm, (uint32_t)n};
        if (!side) return emit_leaf_data(h, early, s);
        BVH_HIP_TRY(hipStreamWaitEvent(side->stream, side->ready, 0));
        BVH_TRY(emit_leaf_data(h, early, side->stream));
        BVH_HIP_TRY(hipEventRecord(side->done, side->stream));
        return BVH_OK;
    };
    uint32_t *karras_leaves = nullptr;  // leaf-count slots filled by k_karras (else by k_count_leaves)
    if (h->builder == BVH_BUILDER_SAH) {
        // a4 alternative: binned-SAH topology over the primitive boxes
        BVH_TRY(check_launch("bounds"));
        SahTree tr{ileft, iright, parent, ifirst, icount, iaxis, n};
        BVH_TRY(sah_topology(pbox, (uint32_t)n, vals[0], tr, tile, L, s));
        perm = vals[0];
        BVH_TRY(leaf_data_early());
    } else {
        // a2, a3: keys of 3 * mbits bits, in 32-bit words when they fit
        // (the key buffers hold 64-bit words either way)
        const int mbits = morton_bits(n);
        const bool narrow = 3 * mbits <= 32;
        uint32_t *k32[2] = {reinterpret_cast<uint32_t *>(keys[0]),
                            reinterpret_cast<uint32_t *>(keys[1])};
        int cur = 0;
        if (narrow)
            cur = sort_morton(pbox, (uint32_t)n, info, mbits, k32, vals, hist, nsort, s);
        else
            cur = sort_morton(pbox, (uint32_t)n, info, mbits, keys, vals, hist, nsort, s);
        BVH_TRY(check_launch("morton/radix sort"));
        perm = vals[cur];
        BVH_TRY(mark_sorted());

        // a4 (for the wide layouts, also the leaf count of the collapse),
        // queued before the leaf data's allocations so that the GPU does not
        // wait for them
        if (n > 1) {
            karras_leaves = wide ? bound_slots + 2 * kMaxSlots * kSlotStride : nullptr;
            if (narrow)
                k_karras<<<grid_for(n - 1), kBlock, 0, s>>>(k32[cur], n, ileft, iright, ifirst,
                                                            icount, iaxis, parent, L, karras_leaves);
            else
                k_karras<<<grid_for(n - 1), kBlock, 0, s>>>(keys[cur], n, ileft, iright, ifirst,
                                                            icount, iaxis, parent, L, karras_leaves);
        }
        BVH_TRY(leaf_data_early());
    }
    {  // a5
        k_leaf_boxes<<<nb, kBlock, 0, s>>>(pbox, perm, n, nbox, table, pre, suf);
        for (int k = 1; k < levels; k += 3)
            k_table_levels<<<grid_for(nblocks), kBlock, 0, s>>>(table, nblocks, k,
                                                                std::min(3, levels - k));
        if (n > 1)
            k_internal_boxes<<<grid_for(n - 1), kBlock, 0, s>>>(ifirst, icount, n, table, nblocks,
                                                                pre, suf, nbox, area);
    }
    BVH_TRY(check_launch("hierarchy/boxes"));
    // a6
    TreeView tv{n, L, ileft, iright, parent, ifirst, icount, iaxis, nbox, area, bound_slots,
                bound_slots + kMaxSlots * kSlotStride};
    uint32_t *hw = host_words();
    if (!hw) return set_error(BVH_ENOMEM, "hipHostMalloc failed");
    volatile uint32_t *nleaf_word = hw + 8;
    *nleaf_word = kPending;
    // the wide layouts read the leaf count from a host-mapped word instead of
    // draining the stream (and need no leaf marks); the others need the scene
    // box and the marks' exclusive scan before packing
    if (wide) {
        uint32_t *leaf_slots = bound_slots + 2 * kMaxSlots * kSlotStride;
        if (!karras_leaves)
            k_count_leaves<<<grid_for(2 * (uint64_t)n - 1), kBlock, 0, s>>>(tv, leaf_slots);
        k_fold_leaf_count<<<1, kBlock, 0, s>>>(leaf_slots, hw + 8);
    } else {
        k_mark_leaves<<<grid_for(2 * (uint64_t)n - 1), kBlock, 0, s>>>(tv, mark);
        scan_u32(mark, mark, n, tile, &info->n_leaves, s);
    }
    BVH_TRY(check_launch("collapse"));
    BuildInfo hi;
    BuildInfo *pin = pinned_scratch<BuildInfo>();
    if (!pin) return set_error(BVH_ENOMEM, "hipHostMalloc failed");
    const LeafSource ls{verts, n_verts, tris, perm, (uint32_t)n};
    if (!wide) {
        BVH_HIP_TRY(hipMemcpyAsync(pin, info, sizeof(hi), hipMemcpyDeviceToHost, s));
        BVH_TRY(alloc_leaf_block(h));  // while the queued kernels run
        BVH_HIP_TRY(hipStreamSynchronize(s));
        hi = *pin;
        if (hi.err & 1u) return set_error(BVH_EINVAL, "bvh_build: a vertex index is outside [0, n_verts)");
        for (int a = 0; a < 3; a++) {
            h->scene_lo[a] = hi.slo[a];
            h->scene_hi[a] = hi.shi[a];
        }
        h->n_leaves = hi.n_leaves;
    }

    // a7
    if (h->layout == BVH_LAYOUT_AABB2) {
        h->n_nodes = 2 * (int64_t)hi.n_leaves - 1;
        BVH_TRY(emit_leaf_data(h, ls, s));
        BVH_TRY(alloc_node_block(h, h->n_nodes));
        k_emit_aabb2<<<grid_for(2 * (uint64_t)n - 1), kBlock, 0, s>>>(
            tv, mark, static_cast<bvh_node_aabb2 *>(h->nodes), (uint32_t)h->n_nodes, info);
        BVH_TRY(check_launch("aabb2 packing"));
    } else if (h->layout == BVH_LAYOUT_PBRT_SOAOS) {
        // the AABB2 records, split into a box array and a topology array
        h->n_nodes = 2 * (int64_t)hi.n_leaves - 1;
        Arena ar;
        bvh_node_aabb2 *tmp = nullptr;
        ar.request(&tmp, (size_t)h->n_nodes);
        BVH_TRY(ar.bind(s, kAreaBuildWide));
        BVH_TRY(emit_leaf_data(h, ls, s));
        BVH_TRY(alloc_node_block(h, h->n_nodes));
        k_emit_aabb2<<<grid_for(2 * (uint64_t)n - 1), kBlock, 0, s>>>(tv, mark, tmp,
                                                                      (uint32_t)h->n_nodes, info);
        k_split_aabb2<<<grid_for((uint64_t)h->n_nodes), kBlock, 0, s>>>(
            tmp, (uint32_t)h->n_nodes, static_cast<bvh_node_box_f32 *>(h->nodes),
            const_cast<bvh_node_topo *>(static_cast<const bvh_node_topo *>(
                topo_of(h->nodes, h->n_nodes, h->layout))));
        BVH_TRY(check_launch("pbrt-soaos packing"));
    } else if (h->layout == BVH_LAYOUT_SHARED_SLAB) {
        // the AABB2 tree with one slab per node in place of its box
        h->n_nodes = 2 * (int64_t)hi.n_leaves - 1;
        Arena ar;
        bvh_node_aabb2 *tmp = nullptr;
        ar.request(&tmp, (size_t)h->n_nodes);
        BVH_TRY(ar.bind(s, kAreaBuildWide));
        BVH_TRY(emit_leaf_data(h, ls, s));
        BVH_TRY(alloc_node_block(h, h->n_nodes));
        k_emit_aabb2<<<grid_for(2 * (uint64_t)n - 1), kBlock, 0, s>>>(tv, mark, tmp,
                                                                      (uint32_t)h->n_nodes, info);
        k_pack_slab<<<grid_for((uint64_t)h->n_nodes), kBlock, 0, s>>>(
            tmp, (uint32_t)h->n_nodes, info, static_cast<bvh_node_slab *>(h->nodes));
        BVH_TRY(check_launch("shared-slab packing"));
    } else if (layout_scene_frame(h->layout)) {
        // the AABB2 tree, re-encoded node by node in the scene frame
        const bool pq = !layout_sg_eq(h->layout);
        h->n_nodes = 2 * (int64_t)hi.n_leaves - 1;
        const WorldFrame fr = world_frame(hi.slo, hi.shi, pq ? 65535.0f : 1023.0f);
        for (int a = 0; a < 3; a++) {
            h->frame_origin[a] = fr.o[a];
            h->frame_scale[a] = fr.s[a];
            h->frame_top[a] = pq ? 0.0f : fr.top[a];
        }
        Arena ar;
        bvh_node_aabb2 *tmp = nullptr;
        ar.request(&tmp, (size_t)h->n_nodes);
        BVH_TRY(ar.bind(s, kAreaBuildWide));
        BVH_TRY(emit_leaf_data(h, ls, s));
        BVH_TRY(alloc_node_block(h, h->n_nodes));
        k_emit_aabb2<<<grid_for(2 * (uint64_t)n - 1), kBlock, 0, s>>>(tv, mark, tmp,
                                                                      (uint32_t)h->n_nodes, info);
        const unsigned g = grid_for((uint64_t)h->n_nodes);
        const uint32_t nn = (uint32_t)h->n_nodes;
        if (h->layout == BVH_LAYOUT_PBRT_Q16)
            k_pack_pbrt_q16<false><<<g, kBlock, 0, s>>>(
                tmp, nn, fr, static_cast<bvh_node_pbrt_q16 *>(h->nodes), nullptr, nullptr, info);
        else if (h->layout == BVH_LAYOUT_PBRT_Q16_SOAOS)
            k_pack_pbrt_q16<true><<<g, kBlock, 0, s>>>(
                tmp, nn, fr, nullptr, static_cast<bvh_node_box_q16 *>(h->nodes),
                static_cast<uint32_t *>(const_cast<void *>(topo_of(h->nodes, h->n_nodes, h->layout))),
                info);
        else if (h->layout == BVH_LAYOUT_SG_EQ)
            k_pack_sg_eq<false><<<g, kBlock, 0, s>>>(tmp, nn, fr, h->nodes, info);
        else
            k_pack_sg_eq<true><<<g, kBlock, 0, s>>>(tmp, nn, fr, h->nodes, info);
        BVH_TRY(check_launch("scene-frame packing"));
    } else if (h->layout == BVH_LAYOUT_BVH4) {
        BVH_TRY(pack_wide<BVH_LAYOUT_BVH4>(tv, nleaf_word, cand_all, ni_all, info, h, ls, s));
    } else if (h->layout == BVH_LAYOUT_BVH8_Q8) {
        BVH_TRY(pack_wide<BVH_LAYOUT_BVH8_Q8>(tv, nleaf_word, cand_all, ni_all, info, h, ls, s));
    } else {
        BVH_TRY(pack_wide<BVH_LAYOUT_BVH8_Q16>(tv, nleaf_word, cand_all, ni_all, info, h, ls, s));
    }
    if (!wide) {  // pack_wide folds them itself
        k_fold_max_slots<<<1, kBlock, 0, s>>>(tv.stack_slots, tv.depth_slots, info);
        BVH_TRY(check_launch("stack bound"));
    }
    if (side) BVH_HIP_TRY(hipStreamWaitEvent(s, side->done, 0));  // the leaf data is part of the build
    BVH_HIP_TRY(hipMemcpyAsync(pin, info, sizeof(hi), hipMemcpyDeviceToHost, s));
    BVH_HIP_TRY(hipStreamSynchronize(s));
    hi = *pin;
    if (wide) {
        if (hi.err & 1u) return set_error(BVH_EINVAL, "bvh_build: a vertex index is outside [0, n_verts)");
        for (int a = 0; a < 3; a++) {
            h->scene_lo[a] = hi.slo[a];
            h->scene_hi[a] = hi.shi[a];
        }
    }
    if (hi.err & 4u) return set_error(BVH_EHIP, "bvh_build: internal error (malformed hierarchy)");
    if (hi.err & 2u)
        return set_error(BVH_EUNSUPPORTED, "bvh_build: non-finite box extent (coordinates too large?)");
    h->depth = (int32_t)hi.max_depth;
    h->max_stack = (int32_t)hi.max_stack;
    if (h->max_stack > kStackMax)
        return set_error(BVH_EUNSUPPORTED, "bvh_build: traversal stack bound %d exceeds %d",
                         h->max_stack, kStackMax);
    return BVH_OK;
}

}  // namespace
}  // namespace bvhlib

using namespace bvhlib;

namespace bvhlib {

int32_t build_handle(const float *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                     int32_t layout, int32_t leaf_size, int32_t leaf_mode, int32_t stack_lds,
                     int32_t builder, hipStream_t s, bvh_handle_s **out) {
    *out = nullptr;
    BVH_TRY(require_device());
    int dev = 0;
    BVH_HIP_TRY(hipGetDevice(&dev));
    bvh_handle_s *h = new bvh_handle_s;
    h->device = dev;
    h->layout = layout;
    h->leaf_mode = leaf_mode;
    h->leaf_size = leaf_size;
    h->stack_lds = stack_lds;
    h->builder = builder;
    h->arity = layout_arity(layout);
    h->n_tris = n_tris;
    h->n_verts = n_verts;
    h->node_bytes = node_record_bytes(layout);
    if (n_tris == 0) {
        *out = h;
        return BVH_OK;
    }
    int32_t rc = build_impl(verts, n_verts, tris, n_tris, h, s);
    if (rc != BVH_OK) {
        std::string msg = bvh_last_error();
        bvh_destroy(h);
        return set_error(rc, "%s", msg.c_str());
    }
    *out = h;
    return BVH_OK;
}

}  // namespace bvhlib

extern "C" int32_t bvh_build(const float *verts, int64_t n_verts, const int32_t *tris,
                             int64_t n_tris, int32_t layout, const bvh_build_opts *opts,
                             void *stream, bvh_handle_t *out) {
    if (!out) return set_error(BVH_EINVAL, "bvh_build: out is null");
    *out = nullptr;
    if (n_tris < 0 || n_verts < 0) return set_error(BVH_EINVAL, "bvh_build: negative size");
    if (n_tris > 0 && (!verts || !tris)) return set_error(BVH_EINVAL, "bvh_build: null mesh pointer");
    if (n_tris > 0 && n_verts == 0) return set_error(BVH_EINVAL, "bvh_build: triangles without vertices");
    if (layout < 0 || layout >= BVH_NUM_LAYOUTS)
        return set_error(BVH_EINVAL, "bvh_build: unknown layout %d", layout);
    // LDS stack default: binary trees push one entry per level (32 entries of
    // 4 B); wide trees push up to arity-1 entries of 8 B (16 entries)
    int32_t leaf_size = 4, leaf_mode = BVH_LEAF_COMPACT;
    int32_t stack_lds = layout_arity(layout) == 2 ? 32 : 16;
    int32_t builder = BVH_BUILDER_LBVH;
    if (opts) {
        for (int k = 0; k < 4; k++)
            if (opts->reserved[k] != 0) return set_error(BVH_EINVAL, "bvh_build: reserved option set");
        if (opts->leaf_size != 0) leaf_size = opts->leaf_size;
        if (opts->leaf_mode != 0) leaf_mode = opts->leaf_mode;
        if (opts->stack_lds != 0) stack_lds = opts->stack_lds;
        builder = opts->builder;
    }
    if (builder != BVH_BUILDER_LBVH && builder != BVH_BUILDER_SAH)
        return set_error(BVH_EINVAL, "bvh_build: unknown builder %d", builder);
    const int32_t max_leaf =  // the scene-frame binary layouts store a u4 count
        layout_scene_frame(layout) ? 15 : kMaxLeafSize;
    if (leaf_size < 1 || leaf_size > max_leaf)
        return set_error(BVH_EINVAL, "bvh_build: leaf_size %d outside 1..%d", leaf_size, max_leaf);
    if (leaf_mode != BVH_LEAF_COMPACT && leaf_mode != BVH_LEAF_INDEXED)
        return set_error(BVH_EINVAL, "bvh_build: unknown leaf mode %d", leaf_mode);
    if (stack_lds != 8 && stack_lds != 16 && stack_lds != 32)
        return set_error(BVH_EINVAL, "bvh_build: stack_lds %d is not 8, 16 or 32", stack_lds);
    if (n_tris > kMaxTris)
        return set_error(BVH_EUNSUPPORTED, "bvh_build: %lld triangles exceed %lld",
                         (long long)n_tris, (long long)kMaxTris);
    const int32_t rc = build_handle(verts, n_verts, tris, n_tris, layout, leaf_size, leaf_mode,
                                    stack_lds, builder, static_cast<hipStream_t>(stream), out);
    if (rc == BVH_OK && *out) (*out)->stack_lds_default = !(opts && opts->stack_lds != 0);
    return rc;
}
