// Per-scene closest-hit / any-hit traversal kernels (one ray per lane) and
// the bvh_trace / bvh_trace_counts entry points.
#include <algorithm>
#include <mutex>

#include "traverse.h"

namespace bvhlib {
namespace {

// One ray per lane, LDS stack of SL entries.  A ray whose stack would
// overflow is appended to the fallback list instead of writing a hit.
template <int Layout, int LeafMode, int Mode, bool Count, int SL>
__global__ __launch_bounds__(kTraceBlock) void k_trace(const void *nodes, int64_t n_nodes,
                                                       SceneData ld, const bvh_ray *rays,
                                                       uint64_t n, bvh_hit *hits,
                                                       uint32_t *counts, Fallback fb) {
    using Tr = typename TracerFor<Layout>::type;
    __shared__ uint32_t s_ref[SL * kTraceBlock];
    __shared__ float s_t[(Tr::kWithT ? SL : 1) * kTraceBlock];
    const uint64_t i = (uint64_t)blockIdx.x * kTraceBlock + threadIdx.x;
    if (i >= n) return;
    const Ray r = load_ray(rays, i, ld.coord_max);
    uint32_t nfetch = 0, ntri = 0;
    bool incomplete = false;
    LdsStack<Tr::kWithT, SL> st(s_ref, s_t);
    const Best best =
        trace_ray<Layout, LeafMode, Mode>(nodes, n_nodes, ld, r, st, nfetch, ntri, incomplete);
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

// Persistent kernel: the grid holds as many blocks as fit on the GPU at
// once, and every lane traces ray after ray.  A lane whose ray ends is
// refilled from its wave's pool of claimed rays once enough lanes of the
// wave are idle (a wave claims 64 consecutive rays per atomic), so the
// wave's lanes stay busy on long rays instead of idling until the slowest
// ray of a fixed group ends.  A wave whose rays were coherent waits until
// all its lanes are idle and then takes 64 consecutive rays, which keeps
// neighbouring camera rays together (they end at nearly the same time).
// The first three quarters of the rays are dealt to the waves round-robin in
// 64-ray chunks (no atomics); the rest is claimed from a queue, which
// balances the tail.  Each lane's stack is a ring in LDS over a spill
// area in global memory that the lane owns for the launch; rays that outgrow
// both go to the fallback pass.  Every wave leaves the loop once the queue is
// drained and its lanes are idle, so the grid always drains.
constexpr uint32_t kNoRay = 0xFFFFFFFFu;
constexpr uint32_t kRefillLanes = 16;  // idle lanes of a wave that trigger a refill
constexpr uint32_t kClaim = 64;        // rays claimed from the queue per atomic

template <int Layout, int LeafMode, int Mode, bool Count, int SL>
__global__ __launch_bounds__(kTraceBlock) void k_trace_persist(const void *nodes, int64_t n_nodes,
                                                               SceneData ld, const bvh_ray *rays,
                                                               uint64_t n, bvh_hit *hits,
                                                               uint32_t *counts, Fallback fb,
                                                               SpillArea sa) {
    using Tr = typename TracerFor<Layout>::type;
    __shared__ uint32_t s_ref[SL * kTraceBlock];
    __shared__ float s_t[(Tr::kWithT ? SL : 1) * kTraceBlock];
    __shared__ WaveLeafLds s_wl[Tr::kBatchLeaves ? kWavesPerBlock : 1];
    WaveLeafLds *wl = &s_wl[Tr::kBatchLeaves ? (threadIdx.x >> 6) : 0];
    SpillStack<Tr::kWithT, SL> st(s_ref, s_t, sa);
    uint32_t ray = kNoRay;
    Ray r{};
    typename Tr::Prep prep{};
    typename Tr::State ts = Tr::start(0);
    uint32_t nfetch = 0, ntri = 0;
    bool incomplete = false;
    // wave-uniform: the wave's pool of claimed rays [pool, pool_end), and
    // whether the queue is exhausted
    uint64_t pool = 0, pool_end = 0;
    bool drained = false;
    const uint32_t waves = gridDim.x * (kTraceBlock / 64u);
    const uint32_t wave =  // the same in every lane: keep it scalar
        blockIdx.x * (kTraceBlock / 64u) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t static_rounds = (n * 3u / 4u) / ((uint64_t)waves * kClaim);
    const uint64_t static_end = static_rounds * waves * kClaim;
    uint64_t round = 0;  // static chunks taken by this wave
    uint32_t queue = wave % kQueues;  // the wave's current dynamic queue (wave-uniform)
    bool coherent = true;  // the wave's last rays all pointed into one octant
    for (;;) {
        const uint64_t idle = __builtin_amdgcn_ballot_w64(ray == kNoRay);
        const uint32_t nidle = (uint32_t)__builtin_popcountll(idle);
        const uint32_t need = coherent ? 64u : kRefillLanes;
        if (nidle >= need && !(drained && pool == pool_end)) {
            const uint32_t avail = (uint32_t)(pool_end - pool);
            uint64_t fresh = 0, fresh_end = 0;  // a newly claimed range
            if (avail < nidle && !drained) {
                if (round < static_rounds) {
                    fresh = (round * waves + wave) * kClaim;
                    fresh_end = fresh + kClaim;
                    round++;
                } else if (!claim_dynamic(fb, static_end, n, kClaim,
                                          (uint32_t)__builtin_ctzll(idle), queue, fresh,
                                          fresh_end)) {
                    drained = true;
                }
            }
            const uint32_t fresh_n = (uint32_t)(fresh_end - fresh);
            if (ray == kNoRay) {
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
                uint64_t my = kNoRay;
                if (rank < avail) my = pool + rank;
                else if (rank - avail < fresh_n) my = fresh + (rank - avail);
                if (my != kNoRay) {
                    ray = (uint32_t)my;
                    r = load_ray(rays, my, ld.coord_max);
                    prep = Tr::prep(r);
                    ts = Tr::start(n_nodes);
                    st.reset();
                    nfetch = ntri = 0;
                    incomplete = false;
                }
            }
            // advance the pool past what was handed out
            if (avail >= nidle) {
                pool += nidle;
            } else if (fresh_n > 0) {
                pool = fresh + min(nidle - avail, fresh_n);
                pool_end = fresh + fresh_n;
            } else {
                pool = pool_end;
            }
        }
        const uint64_t busy = __builtin_amdgcn_ballot_w64(ray != kNoRay);
        if (busy == 0) {
            if (drained && pool == pool_end) break;
            continue;
        }
        // computed by every lane (converged), so the values stay wave-uniform
        coherent = rays_share_octant(r, ray != kNoRay, busy);
        const bool fast = __builtin_amdgcn_ballot_w64(ray != kNoRay && !r.fast) == 0;
        if (coherent) {
            if (ray != kNoRay)
                Tr::template round<LeafMode, Mode>(nodes, n_nodes, ld, r, prep, fast, st, ts,
                                                   nfetch, ntri, incomplete);
        } else if constexpr (Tr::kBatchLeaves) {
            Tr::template round_wave<LeafMode, Mode>(nodes, n_nodes, ld, r, prep, fast, st, ts,
                                                    ray != kNoRay, wl, nfetch, ntri, incomplete);
        } else if (ray != kNoRay) {
            Tr::template step<LeafMode, Mode>(nodes, n_nodes, ld, r, prep, fast, st, ts, nfetch,
                                              ntri, incomplete);
        }
        if (ray != kNoRay) {
            if (Tr::done(ts)) {
                if (incomplete) {
                    fallback_append(fb, ray);
                } else {
                    store_hit(hits, ray, ts.best);
                    if (Count) {
                        counts[2 * (size_t)ray] = nfetch;
                        counts[2 * (size_t)ray + 1] = ntri;
                    }
                }
                ray = kNoRay;
            }
        }
    }
}

// Fallback pass: a small fixed grid re-traces the listed rays from the root
// with a deep stack in global memory (one stack per thread of the grid).
// Launched after every fast pass; it exits at once when the list is empty.
template <int Layout, int LeafMode, int Mode, bool Count>
__global__ __launch_bounds__(kTraceBlock) void k_trace_fallback(const void *nodes, int64_t n_nodes,
                                                                SceneData ld, const bvh_ray *rays,
                                                                bvh_hit *hits, uint32_t *counts,
                                                                Fallback fb) {
    using Tr = typename TracerFor<Layout>::type;
    const uint32_t lane = blockIdx.x * kTraceBlock + threadIdx.x;
    const uint32_t lanes = gridDim.x * kTraceBlock;
    const uint32_t total = *fb.count;
    for (uint32_t k = lane; k < total; k += lanes) {
        const uint32_t i = fb.list[k];
        const Ray r = load_ray(rays, i, ld.coord_max);
        uint32_t nfetch = 0, ntri = 0;
        bool incomplete = false;
        GlobalStack<Tr::kWithT> st(fb.stack_ref + (size_t)lane * kStackMax,
                                   fb.stack_t + (size_t)lane * kStackMax);
        const Best best =
            trace_ray<Layout, LeafMode, Mode>(nodes, n_nodes, ld, r, st, nfetch, ntri, incomplete);
        store_hit(hits, i, best);
        if (Count) {
            counts[2 * (size_t)i] = nfetch;
            counts[2 * (size_t)i + 1] = ntri;
        }
    }
}

// Shared-slab layout: a node's box is the box inherited from its parent with
// the node's one slab axis replaced, so every stack entry carries the box its
// node inherits.  Grid-stride over the rays; single-loop order, near child
// (split axis and ray sign) first.
template <int LeafMode, int Mode, bool Count>
__global__ __launch_bounds__(kTraceBlock) void k_trace_slab(const bvh_node_slab *nodes,
                                                            int64_t n_nodes, SceneData ld,
                                                            const bvh_ray *rays, uint64_t n,
                                                            bvh_hit *hits, uint32_t *counts,
                                                            CarriedStack cs) {
    const uint32_t lane = blockIdx.x * kTraceBlock + threadIdx.x;
    for (uint64_t i = lane; i < n; i += cs.lanes) {
        const Ray r = load_ray(rays, i, ld.coord_max);
        Best best{INFINITY, 0.0f, 0.0f, 0xFFFFFFFFu};
        uint32_t nfetch = 0, ntri = 0, sp = 0;
        uint32_t cur = n_nodes > 0 ? 0u : kRefEmpty;
        float lo[3] = {ld.fo[0], ld.fo[1], ld.fo[2]}, hi[3] = {ld.ft[0], ld.ft[1], ld.ft[2]};
        for (;;) {
            if (cur == kRefEmpty) {
                if (sp == 0) break;
                sp--;
                cur = cs.ref[(size_t)sp * cs.lanes + lane];
                for (int k = 0; k < 3; k++) {
                    lo[k] = cs.box[((size_t)sp * 6 + k) * cs.lanes + lane];
                    hi[k] = cs.box[((size_t)sp * 6 + 3 + k) * cs.lanes + lane];
                }
            }
            if (cur >= (uint64_t)n_nodes) break;  // bounds guard; a valid tree never takes it
            const bvh_node_slab nd = nodes[cur];
            nfetch++;
            const uint32_t cnt = nd.meta & 0xFFFFu, sa = (nd.meta >> 16) & 3u;
            const uint32_t split = (nd.meta >> 18) & 3u;
            for (int k = 0; k < 3; k++) {
                lo[k] = (uint32_t)k == sa ? nd.slo : lo[k];
                hi[k] = (uint32_t)k == sa ? nd.shi : hi[k];
            }
            const float tcur = best_bound<Mode>(r, best);
            const float tn = r.fast ? slab<true>(r, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], tcur)
                                    : slab<false>(r, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], tcur);
            if (tn == INFINITY) {
                cur = kRefEmpty;
                continue;
            }
            if (cnt > 0) {
                if (test_leaf<LeafMode, Mode>(ld, r, nd.offset, cnt, best, ntri)) break;
                cur = kRefEmpty;
                continue;
            }
            const bool neg = split == 0 ? r.nx : (split == 1 ? r.ny : r.nz);
            const uint32_t left = cur + 1u, right = cur + nd.offset;
            if (sp < cs.cap) {  // the build bounds the pushes per path by cap - 1
                cs.ref[(size_t)sp * cs.lanes + lane] = neg ? left : right;
                for (int k = 0; k < 3; k++) {
                    cs.box[((size_t)sp * 6 + k) * cs.lanes + lane] = lo[k];
                    cs.box[((size_t)sp * 6 + 3 + k) * cs.lanes + lane] = hi[k];
                }
                sp++;
            }
            cur = neg ? right : left;
        }
        store_hit(hits, i, best);
        if (Count) {
            counts[2 * (size_t)i] = nfetch;
            counts[2 * (size_t)i + 1] = ntri;
        }
    }
}

template <int LeafMode, int Mode, bool Count>
int32_t launch_slab(const bvh_handle_s *h, const SceneData &ld, const bvh_ray *rays, uint64_t n,
                    bvh_hit *hits, uint32_t *counts, hipStream_t s) {
    CarriedStack cs;
    unsigned grid = 0;
    BVH_TRY(carried_stack(s, n, h->max_stack, 6, cs, grid));
    k_trace_slab<LeafMode, Mode, Count><<<grid, kTraceBlock, 0, s>>>(
        static_cast<const bvh_node_slab *>(h->nodes), h->n_nodes, ld, rays, n, hits, counts, cs);
    return BVH_OK;
}

constexpr bool kPersistent = true;

// Fallback grid of a launch that brings its own (fixed-size) work area.
constexpr int kFixedFallbackBlocks = 16;

// Work area of bvh_trace_noalloc: a file-scope device array (one copy per
// GPU, kept until the process ends) holding the fallback header, a list of
// up to kNoAllocMaxRays ray indices and the deep stacks of a fallback grid of
// kFixedFallbackBlocks blocks: 16 MiB + 2,304 B.
constexpr uint64_t kNoAllocMaxRays = uint64_t(1) << 21;
constexpr size_t kNoAllocScratchBytes =
    fallback_bytes(kNoAllocMaxRays, (size_t)kFixedFallbackBlocks * kTraceBlock);
static_assert(kNoAllocMaxRays == BVH_NOALLOC_MAX_RAYS, "bvh.h states the limit");

// fixed: when non-null, the launch uses this work area: one ray per lane with
// the LDS stack only, overflowing rays re-traced by a fallback grid of
// kFixedFallbackBlocks blocks.  Otherwise the area comes
// from the stream's grow-only work area and the persistent kernel runs.
template <int Layout, int LeafMode, int Mode, bool Count, int SL>
int32_t launch_layout(const bvh_handle_s *h, const SceneData &ld, const bvh_ray *rays, uint64_t n,
                      bvh_hit *hits, uint32_t *counts, const Fallback *fixed, hipStream_t s) {
    const uint64_t need = (n + kTraceBlock - 1) / kTraceBlock;
    if (fixed) {
        k_trace<Layout, LeafMode, Mode, Count, SL><<<(unsigned)need, kTraceBlock, 0, s>>>(
            h->nodes, h->n_nodes, ld, rays, n, hits, counts, *fixed);
        k_trace_fallback<Layout, LeafMode, Mode, Count>
            <<<kFixedFallbackBlocks, kTraceBlock, 0, s>>>(h->nodes, h->n_nodes, ld, rays, hits,
                                                           counts, *fixed);
        return BVH_OK;
    }
    TraceArea ta;
    if (kPersistent) {
        auto kernel = k_trace_persist<Layout, LeafMode, Mode, Count, SL>;
        unsigned resident = 0;
        BVH_TRY(resident_blocks(kernel, resident));
        const unsigned grid = (unsigned)std::min<uint64_t>(resident, need);
        BVH_TRY(trace_area(s, n, grid * kTraceBlock, ta));
        kernel<<<grid, kTraceBlock, 0, s>>>(h->nodes, h->n_nodes, ld, rays, n, hits, counts, ta.fb,
                                            ta.sa);
    } else {
        BVH_TRY(trace_area(s, n, 0, ta));
        k_trace<Layout, LeafMode, Mode, Count, SL><<<(unsigned)need, kTraceBlock, 0, s>>>(
            h->nodes, h->n_nodes, ld, rays, n, hits, counts, ta.fb);
    }
    k_trace_fallback<Layout, LeafMode, Mode, Count><<<kFallbackBlocks, kTraceBlock, 0, s>>>(
        h->nodes, h->n_nodes, ld, rays, hits, counts, ta.fb);
    return BVH_OK;
}

template <int LeafMode, int Mode, bool Count, int SL>
int32_t launch_sl(const bvh_handle_s *h, const SceneData &ld, const bvh_ray *rays, uint64_t n,
                  bvh_hit *hits, uint32_t *counts, const Fallback *fixed, hipStream_t s) {
    switch (h->layout) {
        case BVH_LAYOUT_AABB2:
            return launch_layout<BVH_LAYOUT_AABB2, LeafMode, Mode, Count, SL>(h, ld, rays, n, hits,
                                                                             counts, fixed, s);
        case BVH_LAYOUT_BVH4:
            return launch_layout<BVH_LAYOUT_BVH4, LeafMode, Mode, Count, SL>(h, ld, rays, n, hits,
                                                                            counts, fixed, s);
        case BVH_LAYOUT_BVH8_Q8:
            return launch_layout<BVH_LAYOUT_BVH8_Q8, LeafMode, Mode, Count, SL>(h, ld, rays, n,
                                                                               hits, counts, fixed, s);
        case BVH_LAYOUT_PBRT_Q16:
            return launch_layout<BVH_LAYOUT_PBRT_Q16, LeafMode, Mode, Count, SL>(h, ld, rays, n,
                                                                                hits, counts, fixed, s);
        case BVH_LAYOUT_SG_EQ:
            return launch_layout<BVH_LAYOUT_SG_EQ, LeafMode, Mode, Count, SL>(h, ld, rays, n, hits,
                                                                             counts, fixed, s);
        case BVH_LAYOUT_PBRT_SOAOS:
            return launch_layout<BVH_LAYOUT_PBRT_SOAOS, LeafMode, Mode, Count, SL>(h, ld, rays, n,
                                                                                  hits, counts, fixed, s);
        case BVH_LAYOUT_PBRT_Q16_SOAOS:
            return launch_layout<BVH_LAYOUT_PBRT_Q16_SOAOS, LeafMode, Mode, Count, SL>(
                h, ld, rays, n, hits, counts, fixed, s);
        case BVH_LAYOUT_SG_EQ_A16:
            return launch_layout<BVH_LAYOUT_SG_EQ_A16, LeafMode, Mode, Count, SL>(h, ld, rays, n,
                                                                                 hits, counts, fixed, s);
        default:
            return launch_layout<BVH_LAYOUT_BVH8_Q16, LeafMode, Mode, Count, SL>(h, ld, rays, n,
                                                                                hits, counts, fixed, s);
    }
}

template <int LeafMode, int Mode, bool Count>
int32_t launch_mode(const bvh_handle_s *h, const bvh_ray *rays, uint64_t n, bvh_hit *hits,
                    uint32_t *counts, const Fallback *fixed, hipStream_t s) {
    const SceneData ld = scene_data(h);
    int32_t rc;
    if (h->layout == BVH_LAYOUT_SHARED_SLAB)
        rc = fixed ? set_error(BVH_EUNSUPPORTED, "shared-slab layout needs a carried-box stack area")
                   : launch_slab<LeafMode, Mode, Count>(h, ld, rays, n, hits, counts, s);
    else if (h->stack_lds == 8)
        rc = launch_sl<LeafMode, Mode, Count, 8>(h, ld, rays, n, hits, counts, fixed, s);
    else if (h->stack_lds == 32)
        rc = launch_sl<LeafMode, Mode, Count, 32>(h, ld, rays, n, hits, counts, fixed, s);
    else
        rc = launch_sl<LeafMode, Mode, Count, 16>(h, ld, rays, n, hits, counts, fixed, s);
    if (rc != BVH_OK) return rc;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(BVH_EHIP, "bvh_trace: launch failed: %s", hipGetErrorString(e));
    return BVH_OK;
}

template <bool Count>
int32_t launch(const bvh_handle_s *h, const bvh_ray *rays, uint64_t n, bvh_hit *hits, int32_t mode,
               uint32_t *counts, hipStream_t s, const Fallback *fixed = nullptr) {
    if (h->leaf_mode == BVH_LEAF_COMPACT)
        return mode == BVH_TRACE_ANY
                   ? launch_mode<BVH_LEAF_COMPACT, BVH_TRACE_ANY, Count>(h, rays, n, hits, counts,
                                                                         fixed, s)
                   : launch_mode<BVH_LEAF_COMPACT, BVH_TRACE_CLOSEST, Count>(h, rays, n, hits,
                                                                             counts, fixed, s);
    return mode == BVH_TRACE_ANY
               ? launch_mode<BVH_LEAF_INDEXED, BVH_TRACE_ANY, Count>(h, rays, n, hits, counts,
                                                                     fixed, s)
               : launch_mode<BVH_LEAF_INDEXED, BVH_TRACE_CLOSEST, Count>(h, rays, n, hits, counts,
                                                                         fixed, s);
}

// ---------------------------------------------------------------------------
// bvh_trace_noalloc's work area.  In host code `scratch` names a host-side
// stand-in, not device memory: the kernels get the device address that
// hipGetSymbolAddress returns, looked up once per device (with that device
// current) and kept.
// ---------------------------------------------------------------------------
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int32_t scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices)
        return set_error(BVH_EUNSUPPORTED, "bvh_trace_noalloc: device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return set_error(BVH_EHIP, "bvh_trace_noalloc: hipGetSymbolAddress: %s",
                             hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return BVH_OK;
}

// Clears the first n words at p (the fallback header): a kernel rather than
// a memset node, so that the call can be captured into a graph.
__global__ __launch_bounds__(kTraceBlock) void k_zero_words(uint32_t *p, uint32_t n) {
    for (uint32_t k = threadIdx.x; k < n; k += kTraceBlock) p[k] = 0u;
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

extern "C" int32_t bvh_trace_noalloc(bvh_handle_t h, const bvh_ray *rays, int64_t n,
                                     bvh_hit *hits, int32_t mode, void *stream) {
    BVH_TRY(validate(h, rays, n, hits, mode, "bvh_trace_noalloc"));
    if ((uint64_t)n > kNoAllocMaxRays)
        return set_error(BVH_EINVAL, "bvh_trace_noalloc: %lld rays exceed the fixed work area's "
                         "%llu", (long long)n, (unsigned long long)kNoAllocMaxRays);
    if (h->layout == BVH_LAYOUT_SHARED_SLAB)
        return set_error(BVH_EUNSUPPORTED, "bvh_trace_noalloc: shared-slab layout not supported");
    if (n == 0) return BVH_OK;
    BVH_TRY(check_handle_device(h, "bvh_trace_noalloc"));
    void *ptr = nullptr;
    BVH_TRY(scratch_address(h->device, &ptr));
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const Fallback fb = fallback_view(ptr, (uint64_t)n, (size_t)kFixedFallbackBlocks * kTraceBlock);
    k_zero_words<<<1, kTraceBlock, 0, s>>>(static_cast<uint32_t *>(ptr),
                                            (uint32_t)(kFallbackHeaderBytes / 4));
    return launch<false>(h, rays, (uint64_t)n, hits, mode, nullptr, s, &fb);
}

extern "C" int32_t bvh_trace_counts(bvh_handle_t h, const bvh_ray *rays, int64_t n, bvh_hit *hits,
                                    int32_t mode, uint32_t *counts, void *stream) {
    BVH_TRY(validate(h, rays, n, hits, mode, "bvh_trace_counts"));
    if (n > 0 && !counts) return set_error(BVH_EINVAL, "bvh_trace_counts: null counts buffer");
    if (n == 0) return BVH_OK;
    BVH_TRY(check_handle_device(h, "bvh_trace_counts"));
    return launch<true>(h, rays, (uint64_t)n, hits, mode, counts, static_cast<hipStream_t>(stream));
}
