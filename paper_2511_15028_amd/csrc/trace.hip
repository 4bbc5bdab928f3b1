// Per-scene closest-hit / any-hit traversal kernels (one ray per lane) and
// the bvh_trace / bvh_trace_counts entry points.
#include "traverse.h"

namespace bvhlib {
namespace {

// Fast pass: one ray per lane, LDS stack of SL entries.  A ray whose stack
// would overflow is appended to the fallback list instead of writing a hit.
template <int LeafMode, int Mode, bool Count, int SL>
__global__ __launch_bounds__(kTraceBlock) void k_trace_aabb2(const bvh_node_aabb2 *nodes,
                                                             int64_t n_nodes, LeafData ld,
                                                             const bvh_ray *rays, uint64_t n,
                                                             bvh_hit *hits, uint32_t *counts,
                                                             Fallback fb) {
    __shared__ uint32_t s_ref[SL * kTraceBlock];
    const uint64_t i = (uint64_t)blockIdx.x * kTraceBlock + threadIdx.x;
    if (i >= n) return;
    const Ray r = load_ray(rays, i);
    uint32_t nfetch = 0, ntri = 0;
    bool incomplete = false;
    LdsStack<false, SL> st(s_ref, nullptr);
    const Best best = trace_aabb2<LeafMode, Mode>(nodes, n_nodes, ld, r, st, nfetch, ntri, incomplete);
    if (incomplete) {
        fallback_append(fb, (uint32_t)i);
        return;
    }
    store_hit(hits, i, best);
    if (Count) {
        counts[2 * i] = nfetch;
        counts[2 * i + 1] = ntri;
    }
}

template <class Dec, int LeafMode, int Mode, bool Count, int SL>
__global__ __launch_bounds__(kTraceBlock) void k_trace_wide(const void *nodes, int64_t n_nodes,
                                                            LeafData ld, const bvh_ray *rays,
                                                            uint64_t n, bvh_hit *hits,
                                                            uint32_t *counts, Fallback fb) {
    __shared__ uint32_t s_ref[SL * kTraceBlock];
    __shared__ float s_t[SL * kTraceBlock];
    const uint64_t i = (uint64_t)blockIdx.x * kTraceBlock + threadIdx.x;
    if (i >= n) return;
    const Ray r = load_ray(rays, i);
    uint32_t nfetch = 0, ntri = 0;
    bool incomplete = false;
    LdsStack<true, SL> st(s_ref, s_t);
    const Best best =
        trace_wide<Dec, LeafMode, Mode>(nodes, n_nodes, ld, r, st, nfetch, ntri, incomplete);
    if (incomplete) {
        fallback_append(fb, (uint32_t)i);
        return;
    }
    store_hit(hits, i, best);
    if (Count) {
        counts[2 * i] = nfetch;
        counts[2 * i + 1] = ntri;
    }
}

// Fallback pass: a small fixed grid re-traces the listed rays from the root
// with a deep stack in global memory.  Launched after every fast pass; it
// exits at once when the list is empty.
template <int Layout, int LeafMode, int Mode, bool Count>
__global__ __launch_bounds__(kTraceBlock) void k_trace_fallback(const void *nodes, int64_t n_nodes,
                                                                LeafData ld, const bvh_ray *rays,
                                                                bvh_hit *hits, uint32_t *counts,
                                                                Fallback fb) {
    const uint32_t lane = blockIdx.x * kTraceBlock + threadIdx.x;
    const uint32_t total = *fb.count;
    for (uint32_t k = lane; k < total; k += kFallbackLanes) {
        const uint32_t i = fb.list[k];
        const Ray r = load_ray(rays, i);
        uint32_t nfetch = 0, ntri = 0;
        bool incomplete = false;
        Best best;
        if (Layout == BVH_LAYOUT_AABB2) {
            GlobalStack<false> st(fb.stack_ref + (size_t)lane * kStackMax, nullptr);
            best = trace_aabb2<LeafMode, Mode>(static_cast<const bvh_node_aabb2 *>(nodes), n_nodes,
                                               ld, r, st, nfetch, ntri, incomplete);
        } else {
            GlobalStack<true> st(fb.stack_ref + (size_t)lane * kStackMax,
                                 fb.stack_t + (size_t)lane * kStackMax);
            if (Layout == BVH_LAYOUT_BVH4)
                best = trace_wide<DecodeBVH4, LeafMode, Mode>(nodes, n_nodes, ld, r, st, nfetch,
                                                             ntri, incomplete);
            else if (Layout == BVH_LAYOUT_BVH8_Q8)
                best = trace_wide<DecodeBVH8Q8, LeafMode, Mode>(nodes, n_nodes, ld, r, st, nfetch,
                                                               ntri, incomplete);
            else
                best = trace_wide<DecodeBVH8Q16, LeafMode, Mode>(nodes, n_nodes, ld, r, st, nfetch,
                                                                ntri, incomplete);
        }
        store_hit(hits, i, best);
        if (Count) {
            counts[2 * (size_t)i] = nfetch;
            counts[2 * (size_t)i + 1] = ntri;
        }
    }
}

template <int LeafMode, int Mode, bool Count, int SL>
void launch_sl(const bvh_handle_s *h, const LeafData &ld, const bvh_ray *rays, uint64_t n,
               bvh_hit *hits, uint32_t *counts, const Fallback &fb, hipStream_t s) {
    const unsigned grid = (unsigned)((n + kTraceBlock - 1) / kTraceBlock);
    switch (h->layout) {
        case BVH_LAYOUT_AABB2:
            k_trace_aabb2<LeafMode, Mode, Count, SL><<<grid, kTraceBlock, 0, s>>>(
                static_cast<const bvh_node_aabb2 *>(h->nodes), h->n_nodes, ld, rays, n, hits, counts, fb);
            k_trace_fallback<BVH_LAYOUT_AABB2, LeafMode, Mode, Count>
                <<<kFallbackBlocks, kTraceBlock, 0, s>>>(h->nodes, h->n_nodes, ld, rays, hits, counts, fb);
            break;
        case BVH_LAYOUT_BVH4:
            k_trace_wide<DecodeBVH4, LeafMode, Mode, Count, SL><<<grid, kTraceBlock, 0, s>>>(
                h->nodes, h->n_nodes, ld, rays, n, hits, counts, fb);
            k_trace_fallback<BVH_LAYOUT_BVH4, LeafMode, Mode, Count>
                <<<kFallbackBlocks, kTraceBlock, 0, s>>>(h->nodes, h->n_nodes, ld, rays, hits, counts, fb);
            break;
        case BVH_LAYOUT_BVH8_Q8:
            k_trace_wide<DecodeBVH8Q8, LeafMode, Mode, Count, SL><<<grid, kTraceBlock, 0, s>>>(
                h->nodes, h->n_nodes, ld, rays, n, hits, counts, fb);
            k_trace_fallback<BVH_LAYOUT_BVH8_Q8, LeafMode, Mode, Count>
                <<<kFallbackBlocks, kTraceBlock, 0, s>>>(h->nodes, h->n_nodes, ld, rays, hits, counts, fb);
            break;
        default:
            k_trace_wide<DecodeBVH8Q16, LeafMode, Mode, Count, SL><<<grid, kTraceBlock, 0, s>>>(
                h->nodes, h->n_nodes, ld, rays, n, hits, counts, fb);
            k_trace_fallback<BVH_LAYOUT_BVH8_Q16, LeafMode, Mode, Count>
                <<<kFallbackBlocks, kTraceBlock, 0, s>>>(h->nodes, h->n_nodes, ld, rays, hits, counts, fb);
            break;
    }
}

template <int LeafMode, int Mode, bool Count>
int32_t launch_mode(const bvh_handle_s *h, const bvh_ray *rays, uint64_t n, bvh_hit *hits,
                    uint32_t *counts, hipStream_t s) {
    const LeafData ld{h->leaf, h->verts, h->tris, (uint32_t)h->n_tris};
    // fallback work area of this stream (grow-only, reused across calls)
    void *ws = nullptr;
    BVH_TRY(stream_workspace(s, kAreaTrace, fallback_bytes(n), &ws));
    const Fallback fb = fallback_view(ws, n);
    hipError_t e = hipMemsetAsync(fb.count, 0, sizeof(uint32_t), s);
    if (e == hipSuccess) {
        if (h->stack_lds == 8)
            launch_sl<LeafMode, Mode, Count, 8>(h, ld, rays, n, hits, counts, fb, s);
        else if (h->stack_lds == 32)
            launch_sl<LeafMode, Mode, Count, 32>(h, ld, rays, n, hits, counts, fb, s);
        else
            launch_sl<LeafMode, Mode, Count, 16>(h, ld, rays, n, hits, counts, fb, s);
        e = hipGetLastError();
    }
    if (e != hipSuccess) return set_error(BVH_EHIP, "bvh_trace: launch failed: %s", hipGetErrorString(e));
    return BVH_OK;
}

template <bool Count>
int32_t launch(const bvh_handle_s *h, const bvh_ray *rays, uint64_t n, bvh_hit *hits, int32_t mode,
               uint32_t *counts, hipStream_t s) {
    if (h->leaf_mode == BVH_LEAF_COMPACT)
        return mode == BVH_TRACE_ANY
                   ? launch_mode<BVH_LEAF_COMPACT, BVH_TRACE_ANY, Count>(h, rays, n, hits, counts, s)
                   : launch_mode<BVH_LEAF_COMPACT, BVH_TRACE_CLOSEST, Count>(h, rays, n, hits, counts, s);
    return mode == BVH_TRACE_ANY
               ? launch_mode<BVH_LEAF_INDEXED, BVH_TRACE_ANY, Count>(h, rays, n, hits, counts, s)
               : launch_mode<BVH_LEAF_INDEXED, BVH_TRACE_CLOSEST, Count>(h, rays, n, hits, counts, s);
}

int32_t validate(bvh_handle_t h, const bvh_ray *rays, int64_t n, bvh_hit *hits, int32_t mode,
                 const char *who) {
    if (!h) return set_error(BVH_EINVAL, "%s: null handle", who);
    if (n < 0) return set_error(BVH_EINVAL, "%s: negative ray count", who);
    if (n > 0 && (!rays || !hits)) return set_error(BVH_EINVAL, "%s: null ray or hit buffer", who);
    if (mode != BVH_TRACE_CLOSEST && mode != BVH_TRACE_ANY)
        return set_error(BVH_EINVAL, "%s: unknown mode %d", who, mode);
    if ((uint64_t)n > (uint64_t)0xFFFFFFFFu)
        return set_error(BVH_EUNSUPPORTED, "%s: more than 2^32 - 1 rays", who);
    return BVH_OK;
}

}  // namespace

int32_t trace_launch(const bvh_handle_s *h, const bvh_ray *rays, uint64_t n, bvh_hit *hits,
                     int32_t mode, hipStream_t s) {
    return launch<false>(h, rays, n, hits, mode, nullptr, s);
}

int32_t check_handle_device(const bvh_handle_s *h, const char *who) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return set_error(BVH_ENODEV, "%s: no HIP device", who);
    if (dev != h->device)
        return set_error(BVH_EINVAL, "%s: handle belongs to device %d, current device is %d", who,
                         h->device, dev);
    return BVH_OK;
}

}  // namespace bvhlib

using namespace bvhlib;

extern "C" int32_t bvh_trace(bvh_handle_t h, const bvh_ray *rays, int64_t n, bvh_hit *hits,
                             int32_t mode, void *stream) {
    BVH_TRY(validate(h, rays, n, hits, mode, "bvh_trace"));
    if (n == 0) return BVH_OK;
    BVH_TRY(check_handle_device(h, "bvh_trace"));
    return launch<false>(h, rays, (uint64_t)n, hits, mode, nullptr, static_cast<hipStream_t>(stream));
}

extern "C" int32_t bvh_trace_counts(bvh_handle_t h, const bvh_ray *rays, int64_t n, bvh_hit *hits,
                                    int32_t mode, uint32_t *counts, void *stream) {
    BVH_TRY(validate(h, rays, n, hits, mode, "bvh_trace_counts"));
    if (n > 0 && !counts) return set_error(BVH_EINVAL, "bvh_trace_counts: null counts buffer");
    if (n == 0) return BVH_OK;
    BVH_TRY(check_handle_device(h, "bvh_trace_counts"));
    return launch<true>(h, rays, (uint64_t)n, hits, mode, counts, static_cast<hipStream_t>(stream));
}
