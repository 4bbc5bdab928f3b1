// Backward pass of closest-hit tracing with the hit primitive held fixed.
//
// The hit of ray i on its fixed triangle p is recomputed from the ray and
// the triangle's vertices with the forward's own ray/triangle arithmetic
// (tri_numerators, the same FP32 operations), so (t, u, v) are exactly the
// forward's hit when verts, tris and rays are the ones traced; the hits
// buffer supplies only the primitive id.  The hit point obeys
// F = o + t d - p0 - u e1 - v e2 = 0 with e1 = p1 - p0, e2 = p2 - p0 (the
// barycentric form of App. G: b0 = 1-u-v, b1 = u, b2 = v).  With
// J = dF/d(t,u,v) = [d | -e1 | -e2] and g = dL/d(t,u,v), the solution of
// J^T lam = g gives dL/dx = -lam^T dF/dx for every input x:
//   dL/do = -lam, dL/dd = -t lam, dL/dp0 = (1-u-v) lam, dL/dp1 = u lam,
//   dL/dp2 = v lam.
// Cramer's rule on the rows d, -e1, -e2 of J^T, whose determinant is
// d . (e1 x e2) = -det (det = e1 . (d x e2) of the forward test):
//   lam = -(g_t (e1 x e2) + g_u (d x e2) + g_v (e1 x d)) / det.
#include "traverse.h"

namespace bvhlib {
namespace {

constexpr int kBlock = 256;

// Vertex-gradient contributions of a block are first summed in an LDS hash
// table keyed by vertex index (open addressing, linear probing), then added
// to grad_verts with one atomic per distinct vertex and component.  Rays of
// a block (neighbouring pixels) share most of their vertices, so this cuts
// the global atomics several-fold and removes same-address conflicts within
// an instruction.  A block touches at most 3 * kBlock vertices, below the
// table size, so an insertion always finds a slot.
constexpr int kTableSlots = 1024;
static_assert(kTableSlots >= 3 * kBlock, "hash table must hold every vertex of a block");

__device__ inline uint32_t slot_of(int32_t v) {
    return ((uint32_t)v * 2654435761u) >> (32 - 10);  // Fibonacci hashing, 10 bits
}

__device__ inline void cross_fma(float ax, float ay, float az, float bx, float by, float bz,
                                 float &cx, float &cy, float &cz) {
    cx = fmaf(ay, bz, -(az * by));
    cy = fmaf(az, bx, -(ax * bz));
    cz = fmaf(ax, by, -(ay * bx));
}

// lam, the hit weights and the ray gradient of ray i; false for a miss, an
// out-of-range primitive or vertex index, or a singular system (det = 0 or
// not finite).
__device__ inline bool ray_grad(const float *verts, int64_t n_verts, const int32_t *tris,
                                int64_t n_tris, const bvh_ray *rays, const bvh_hit *hits,
                                const float *grad_hits, uint64_t i, float *out, int32_t *idx,
                                float *w, float *lam) {
    const int32_t prim = reinterpret_cast<const int32_t *>(hits)[4 * i];
    if (prim < 0 || (int64_t)prim >= n_tris) return false;
    for (int k = 0; k < 3; k++) {
        idx[k] = tris[3 * (size_t)prim + k];
        if (idx[k] < 0 || (int64_t)idx[k] >= n_verts) return false;
    }
    const float4 *rp = reinterpret_cast<const float4 *>(rays + i);
    const float4 ra = rp[0], rb = rp[1];
    Ray r{};
    r.ox = ra.x; r.oy = ra.y; r.oz = ra.z;
    r.dx = rb.x; r.dy = rb.y; r.dz = rb.z;
    const float *q0 = verts + 3 * (size_t)idx[0];
    const float *q1 = verts + 3 * (size_t)idx[1];
    const float *q2 = verts + 3 * (size_t)idx[2];
    const float e1x = q1[0] - q0[0], e1y = q1[1] - q0[1], e1z = q1[2] - q0[2];
    const float e2x = q2[0] - q0[0], e2y = q2[1] - q0[1], e2z = q2[2] - q0[2];
    const TriNum nm = tri_numerators(r, q0[0], q0[1], q0[2], e1x, e1y, e1z, e2x, e2y, e2z);
    if (!(nm.adet > 0.0f && nm.adet < INFINITY)) return false;
    const float inv = 1.0f / nm.adet;
    const float t = nm.T * inv, u = nm.U * inv, v = nm.V * inv;
    float nx, ny, nz, px, py, pz, mx, my, mz;
    cross_fma(e1x, e1y, e1z, e2x, e2y, e2z, nx, ny, nz);     // e1 x e2
    cross_fma(r.dx, r.dy, r.dz, e2x, e2y, e2z, px, py, pz);  // d x e2
    cross_fma(e1x, e1y, e1z, r.dx, r.dy, r.dz, mx, my, mz);  // e1 x d
    const float gt = grad_hits[3 * i], gu = grad_hits[3 * i + 1], gv = grad_hits[3 * i + 2];
    // 1 / det = sign(det) / |det|: the sign of det is that of e1 . (d x e2)
    const float det = fmaf(e1z, pz, fmaf(e1y, py, e1x * px));
    const float ninv = det < 0.0f ? inv : -inv;  // -1 / det
    lam[0] = fmaf(gv, mx, fmaf(gu, px, gt * nx)) * ninv;
    lam[1] = fmaf(gv, my, fmaf(gu, py, gt * ny)) * ninv;
    lam[2] = fmaf(gv, mz, fmaf(gu, pz, gt * nz)) * ninv;
    for (int k = 0; k < 3; k++) {
        out[k] = -lam[k];
        out[3 + k] = -t * lam[k];
    }
    w[0] = (1.0f - u) - v;
    w[1] = u;
    w[2] = v;
    return true;
}

__global__ __launch_bounds__(kBlock) void k_backward(const float *verts, int64_t n_verts,
                                                     const int32_t *tris, int64_t n_tris,
                                                     const bvh_ray *rays, uint64_t n,
                                                     const bvh_hit *hits, const float *grad_hits,
                                                     float *grad_verts, float *grad_rays) {
    __shared__ int32_t skey[kTableSlots];
    __shared__ float sval[3][kTableSlots];
    for (int s = threadIdx.x; s < kTableSlots; s += kBlock) {
        skey[s] = -1;
        sval[0][s] = sval[1][s] = sval[2][s] = 0.0f;
    }
    __syncthreads();
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) {
        float out[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, w[3], lam[3];
        int32_t idx[3];
        if (ray_grad(verts, n_verts, tris, n_tris, rays, hits, grad_hits, i, out, idx, w, lam)) {
            for (int k = 0; k < 3; k++) {
                uint32_t h = slot_of(idx[k]);
                for (int probe = 0; probe < kTableSlots; probe++) {
                    const int32_t prev = atomicCAS(&skey[h], -1, idx[k]);
                    if (prev == -1 || prev == idx[k]) break;
                    h = (h + 1u) & (kTableSlots - 1);
                }
                atomicAdd(&sval[0][h], w[k] * lam[0]);
                atomicAdd(&sval[1][h], w[k] * lam[1]);
                atomicAdd(&sval[2][h], w[k] * lam[2]);
            }
        }
        float *gr = grad_rays + 6 * i;
        for (int k = 0; k < 6; k++) gr[k] = out[k];
    }
    __syncthreads();
    for (int s = threadIdx.x; s < kTableSlots; s += kBlock) {
        const int32_t key = skey[s];
        if (key < 0) continue;
        float *g = grad_verts + 3 * (size_t)key;
        unsafeAtomicAdd(g + 0, sval[0][s]);
        unsafeAtomicAdd(g + 1, sval[1][s]);
        unsafeAtomicAdd(g + 2, sval[2][s]);
    }
}

// ---------------------------------------------------------------------------
// Vertex gradients without atomics.  Every ray contributes to three vertices,
// and a vertex collects contributions from rays all over the ray array (for
// the sphere-of-cameras workload, a 256-ray block reaches 1.26 distinct
// vertices per ray, a whole camera still 0.82, against 0.16 overall), so
// per-block pre-summing still leaves millions of scattered read-modify-write
// updates, and device-scope float atomics on scattered addresses run at
// about 20 G/s here.  Instead the contributions are partitioned by vertex
// range and each range is summed in LDS by one workgroup:
//   k_backward_part: a block of kPartRays rays computes each ray's gradient
//     (grad_rays written as in k_backward) and its three (vertex, w lam)
//     records, sorts the block's records by vertex range in LDS (counting
//     sort over the ranges) and writes them, with the per-range offsets, to
//     its own segment of a work area;
//   k_backward_sum: one block per range of 2^shift vertices reads that
//     range's records from every segment, sums them in a dense LDS
//     accumulator and adds the sums to grad_verts (the range is its own, so
//     plain loads and stores).
// Ranges: shift in [8, 12] with at most kPartMaxRanges ranges, so up to
// 2^22 vertices; larger meshes use k_backward.
// ---------------------------------------------------------------------------
constexpr int kPartThreads = 256;
constexpr int kPartRaysPerThread = 4;
constexpr int kPartRays = kPartThreads * kPartRaysPerThread;
constexpr int kPartRecs = 3 * kPartRays;
constexpr int kPartMaxRanges = 1024;
constexpr int kPartMinShift = 8, kPartMaxShift = 12;
constexpr int kSumThreads = 512;

struct VertRec {
    int32_t v;
    float g[3];
};
static_assert(sizeof(VertRec) == 16, "record");

// Exclusive prefix sum over the block (THREADS threads) of one value per
// thread; wsum holds THREADS / 64 words.
template <int THREADS>
__device__ inline uint32_t block_excl_scan_u32(uint32_t x, uint32_t *wsum, uint32_t *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < THREADS / 64; k++) {
        const uint32_t s = wsum[k];
        off += k < w ? s : 0u;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + inc - x;
}

__global__ __launch_bounds__(kPartThreads) void k_backward_part(
    const float *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris, const bvh_ray *rays,
    uint64_t n, const bvh_hit *hits, const float *grad_hits, float *grad_rays, int shift,
    uint32_t n_ranges, VertRec *seg, uint32_t *offs) {
    __shared__ uint32_t cnt[kPartMaxRanges];
    __shared__ uint32_t wsum[kPartThreads / 64];
    __shared__ VertRec sorted[kPartRecs];
    for (uint32_t p = threadIdx.x; p < n_ranges; p += kPartThreads) cnt[p] = 0;
    __syncthreads();
    int32_t rv[kPartRecs / kPartThreads];
    float rg[kPartRecs / kPartThreads][3];
#pragma unroll
    for (int k = 0; k < kPartRaysPerThread; k++) {
        const uint64_t i = (uint64_t)blockIdx.x * kPartRays + k * kPartThreads + threadIdx.x;
        float out[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, w[3] = {0.f, 0.f, 0.f};
        float lam[3] = {0.f, 0.f, 0.f};
        int32_t idx[3] = {0, 0, 0};
        bool ok = false;
        if (i < n) {
            ok = ray_grad(verts, n_verts, tris, n_tris, rays, hits, grad_hits, i, out, idx, w, lam);
            float *gr = grad_rays + 6 * i;
            for (int c = 0; c < 6; c++) gr[c] = out[c];
        }
#pragma unroll
        for (int c = 0; c < 3; c++) {
            rv[3 * k + c] = ok ? idx[c] : -1;
            rg[3 * k + c][0] = w[c] * lam[0];
            rg[3 * k + c][1] = w[c] * lam[1];
            rg[3 * k + c][2] = w[c] * lam[2];
            if (ok) atomicAdd(&cnt[(uint32_t)idx[c] >> shift], 1u);
        }
    }
    __syncthreads();
    // exclusive offsets of the ranges; each thread scans a run of them
    constexpr int kRun = kPartMaxRanges / kPartThreads;
    uint32_t c[kRun], sum = 0;
#pragma unroll
    for (int k = 0; k < kRun; k++) {
        const uint32_t p = threadIdx.x * kRun + k;
        c[k] = p < n_ranges ? cnt[p] : 0u;
        sum += c[k];
    }
    uint32_t total;
    uint32_t run = block_excl_scan_u32<kPartThreads>(sum, wsum, &total);
    // offsets range-major: offs[q * n_blocks + block], q = n_ranges holding
    // the block's total, so the summing block of range q reads two
    // contiguous rows
    const size_t nbl = gridDim.x;
#pragma unroll
    for (int k = 0; k < kRun; k++) {
        const uint32_t p = threadIdx.x * kRun + k;
        if (p < n_ranges) {
            offs[(size_t)p * nbl + blockIdx.x] = run;
            cnt[p] = run;  // becomes the range's insertion cursor
        }
        run += c[k];
    }
    if (threadIdx.x == 0) offs[(size_t)n_ranges * nbl + blockIdx.x] = total;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPartRecs / kPartThreads; r++) {
        if (rv[r] >= 0) {
            const uint32_t pos = atomicAdd(&cnt[(uint32_t)rv[r] >> shift], 1u);
            sorted[pos] = VertRec{rv[r], {rg[r][0], rg[r][1], rg[r][2]}};
        }
    }
    __syncthreads();
    float4 *dst = reinterpret_cast<float4 *>(seg + (size_t)blockIdx.x * kPartRecs);
    const float4 *src = reinterpret_cast<const float4 *>(sorted);
    for (uint32_t q = threadIdx.x; q < total; q += kPartThreads) dst[q] = src[q];
}

// One block per vertex range.  The range's records are spread over every
// segment: the block first gathers each segment's record count for the range
// (start offset and count, kSumMaxBlocks segments per pass) into LDS and
// scans them, then walks the pass's records as one flat list (a binary
// search over the scanned counts finds a record's segment), so every thread
// has several independent record loads in flight instead of a chain per
// segment.
//
// Summation.  kPrivate (ranges of 2^kSumPrivShift vertices): every wave owns
// an LDS accumulator of the range, so no two waves touch one word; within a
// wave instruction, the lanes holding one vertex find each other with one
// ballot per bit of the vertex's index in the range, the lowest of them adds
// the others' values (ds_bpermute) and alone updates the accumulator with a
// plain read and write.  The copies are added at the end.  LDS float atomics
// (ds_add_f32) cost about 32 LDS cycles per wave instruction, three per
// record; the plain update costs a read and a write per record.  Larger
// ranges (whose copies would not fit in LDS) share one accumulator updated
// with LDS atomics.
constexpr int kSumMaxBlocks = 2048;  // segments per pass
constexpr int kSumUnroll = 4;
constexpr int kSumPrivShift = 8;
constexpr int kSumWaves = kSumThreads / 64;

__device__ inline float bperm_f(float x, uint32_t src) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute((int)(src << 2), __float_as_int(x)));
}

template <bool kPrivate>
__global__ __launch_bounds__(kSumThreads) void k_backward_sum(const VertRec *seg,
                                                              const uint32_t *offs,
                                                              uint32_t n_blocks, int shift,
                                                              uint32_t n_ranges, int64_t n_verts,
                                                              float *grad_verts) {
    // kPrivate: kSumWaves copies of 3 * 2^kSumPrivShift floats; otherwise one
    // copy of 3 * 2^shift floats (dynamic)
    extern __shared__ float acc[];
    __shared__ uint32_t lo[kSumMaxBlocks];
    __shared__ uint32_t start[kSumMaxBlocks + 1];
    __shared__ uint32_t wsum[kSumThreads / 64];
    const uint32_t p = blockIdx.x;
    const uint32_t nv = 1u << shift;
    const int64_t v0 = (int64_t)p << shift;
    const uint32_t n_acc = kPrivate ? kSumWaves : 1;
    for (uint32_t q = threadIdx.x; q < 3 * nv * n_acc; q += kSumThreads) acc[q] = 0.0f;
    float *const my = acc + (kPrivate ? (threadIdx.x >> 6) * 3 * nv : 0);
    const uint32_t lane = threadIdx.x & 63;
    constexpr int kPer = kSumMaxBlocks / kSumThreads;
    for (uint32_t b0 = 0; b0 < n_blocks; b0 += kSumMaxBlocks) {
        const uint32_t nb = min((uint32_t)kSumMaxBlocks, n_blocks - b0);
        // this thread's run of kPer segments: their starts and counts
        uint32_t c[kPer], sum = 0;
#pragma unroll
        for (int k = 0; k < kPer; k++) {
            const uint32_t j = k * kSumThreads + threadIdx.x;  // coalesced over the rows
            uint32_t l = 0, h = 0;
            if (j < nb) {
                l = offs[(size_t)p * n_blocks + b0 + j];
                h = min(offs[(size_t)(p + 1) * n_blocks + b0 + j], (uint32_t)kPartRecs);
                h = h > l ? h : l;
                lo[j] = l;
            }
            c[k] = h - l;
        }
        // segment j's start: scan over j (thread t's run is segments t*kPer..)
        __syncthreads();
        for (int k = 0; k < kPer; k++) {
            const uint32_t j = k * kSumThreads + threadIdx.x;
            start[j] = c[k];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kPer; k++) {
            c[k] = start[threadIdx.x * kPer + k];
            sum += c[k];
        }
        uint32_t total;
        uint32_t run = block_excl_scan_u32<kSumThreads>(sum, wsum, &total);
        __syncthreads();  // every count read before the starts overwrite them
#pragma unroll
        for (int k = 0; k < kPer; k++) {
            const uint32_t j = threadIdx.x * kPer + k;
            if (j < nb) start[j] = run;
            run += c[k];
        }
        if (threadIdx.x == 0) start[nb] = total;
        __syncthreads();
        for (uint32_t q0 = 0; q0 < total; q0 += kSumThreads * kSumUnroll) {
            float4 x[kSumUnroll];
            bool ok[kSumUnroll];
#pragma unroll
            for (int u = 0; u < kSumUnroll; u++) {
                const uint32_t q = q0 + u * kSumThreads + threadIdx.x;
                ok[u] = q < total;
                if (ok[u]) {
                    // the segment j with start[j] <= q < start[j + 1]
                    uint32_t a = 0, b = nb;
                    while (b - a > 1) {
                        const uint32_t m = (a + b) >> 1;
                        if (start[m] <= q) a = m; else b = m;
                    }
                    const VertRec *rec = seg + (size_t)(b0 + a) * kPartRecs + lo[a] + (q - start[a]);
                    x[u] = *reinterpret_cast<const float4 *>(rec);
                }
            }
#pragma unroll
            for (int u = 0; u < kSumUnroll; u++) {
                const uint32_t local = (uint32_t)(__float_as_int(x[u].x) - (int32_t)v0);
                const bool mine = ok[u] && local < nv;  // always in range for a consistent segment
                if constexpr (kPrivate) {
                    uint64_t peers = __builtin_amdgcn_ballot_w64(mine);
#pragma unroll
                    for (int b = 0; b < kSumPrivShift; b++) {
                        const bool bit = (local >> b) & 1u;
                        const uint64_t m = __builtin_amdgcn_ballot_w64(bit);
                        peers &= bit ? m : ~m;
                    }
                    const uint64_t self = uint64_t(1) << lane;
                    const bool leader = mine && (peers & (self - 1)) == 0;
                    uint64_t rest = leader ? peers & ~self : 0;
                    float gx = x[u].y, gy = x[u].z, gz = x[u].w;
                    while (__builtin_amdgcn_ballot_w64(rest != 0)) {
                        const uint32_t src = rest ? (uint32_t)__builtin_ctzll(rest) : lane;
                        const float ax = bperm_f(x[u].y, src), ay = bperm_f(x[u].z, src),
                                    az = bperm_f(x[u].w, src);
                        if (rest) {
                            gx += ax;
                            gy += ay;
                            gz += az;
                            rest &= rest - 1;
                        }
                    }
                    if (leader) {
                        float *a = my + 3 * local;
                        a[0] += gx;
                        a[1] += gy;
                        a[2] += gz;
                    }
                } else if (mine) {
                    atomicAdd(&acc[3 * local + 0], x[u].y);
                    atomicAdd(&acc[3 * local + 1], x[u].z);
                    atomicAdd(&acc[3 * local + 2], x[u].w);
                }
            }
        }
        __syncthreads();
    }
    const int64_t cnt = min((int64_t)nv, n_verts - v0);
    float *g = grad_verts + 3 * v0;
    for (int64_t q = threadIdx.x; q < 3 * cnt; q += kSumThreads) {
        float a = acc[q];
        for (uint32_t w = 1; w < n_acc; w++) a += acc[w * 3 * nv + q];
        g[q] += a;
    }
}

// Smallest range shift (within [kPartMinShift, kPartMaxShift]) that covers
// n_verts with at most kPartMaxRanges ranges; -1 when none does.
inline int part_shift(int64_t n_verts) {
    for (int s = kPartMinShift; s <= kPartMaxShift; s++)
        if (((n_verts + (int64_t(1) << s) - 1) >> s) <= kPartMaxRanges) return s;
    return -1;
}

}  // namespace
}  // namespace bvhlib

using namespace bvhlib;

extern "C" int32_t bvh_trace_backward(const float *verts, int64_t n_verts, const int32_t *tris,
                                      int64_t n_tris, const bvh_ray *rays, int64_t n,
                                      const bvh_hit *hits, const float *grad_hits,
                                      float *grad_verts, float *grad_rays, void *stream) {
    if (n_verts < 0 || n_tris < 0 || n < 0)
        return set_error(BVH_EINVAL, "bvh_trace_backward: negative size");
    if (n > 0 && (!rays || !hits || !grad_hits || !grad_rays))
        return set_error(BVH_EINVAL, "bvh_trace_backward: null ray, hit or gradient buffer");
    if (n_tris > 0 && !tris) return set_error(BVH_EINVAL, "bvh_trace_backward: null tris");
    if (n_verts > 0 && (!verts || !grad_verts))
        return set_error(BVH_EINVAL, "bvh_trace_backward: null verts or grad_verts");
    if (n == 0) return BVH_OK;
    if ((uint64_t)n > (uint64_t)0xFFFFFFFFu * kBlock)
        return set_error(BVH_EUNSUPPORTED, "bvh_trace_backward: too many rays");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const int shift = part_shift(n_verts);
    if (n_verts > 0 && shift >= 0) {
        const uint32_t ranges = (uint32_t)((n_verts + (int64_t(1) << shift) - 1) >> shift);
        const uint64_t blocks = ((uint64_t)n + kPartRays - 1) / kPartRays;
        const size_t seg_bytes = (size_t)blocks * kPartRecs * sizeof(VertRec);
        const size_t off_bytes = (size_t)blocks * (ranges + 1) * sizeof(uint32_t);
        void *ws = nullptr;
        BVH_TRY(stream_workspace(s, kAreaBackward, seg_bytes + off_bytes, &ws));
        VertRec *seg = static_cast<VertRec *>(ws);
        uint32_t *offs = reinterpret_cast<uint32_t *>(static_cast<char *>(ws) + seg_bytes);
        k_backward_part<<<(unsigned)blocks, kPartThreads, 0, s>>>(
            verts, n_verts, tris, n_tris, rays, (uint64_t)n, hits, grad_hits, grad_rays, shift,
            ranges, seg, offs);
        if (shift == kSumPrivShift)
            k_backward_sum<true><<<ranges, kSumThreads, kSumWaves * (3u << shift) * sizeof(float),
                                   s>>>(seg, offs, (uint32_t)blocks, shift, ranges, n_verts,
                                        grad_verts);
        else
            k_backward_sum<false><<<ranges, kSumThreads, (3u << shift) * sizeof(float), s>>>(
                seg, offs, (uint32_t)blocks, shift, ranges, n_verts, grad_verts);
    } else {
        const unsigned grid = (unsigned)(((uint64_t)n + kBlock - 1) / kBlock);
        k_backward<<<grid, kBlock, 0, s>>>(verts, n_verts, tris, n_tris, rays, (uint64_t)n, hits,
                                           grad_hits, grad_verts, grad_rays);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(BVH_EHIP, "bvh_trace_backward: launch failed: %s", hipGetErrorString(e));
    return BVH_OK;
}
