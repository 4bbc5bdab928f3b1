// Batched tracing of many scenes: per-scene autotuning of the node layout
// (and with it the tree arity) and of the LDS stack depth, then one hipGraph
// whose persistent kernels drain per-variant work queues of 64-ray tiles.
//
// The paper shows that the best layout depends on the scene and on the ray
// distribution (Sec. 9.2.2) and leaves execution scheduling to future work
// (Sec. 1); this file is that scheduling layer for one GPU.
#include <algorithm>
#include <cmath>
#include <map>
#include <string>
#include <vector>

#include "traverse.h"

namespace bvhlib {
namespace {

constexpr int kTile = 64;  // rays per work item: one wave64

// Device descriptor of one scene as seen by a batched kernel.
struct BatchScene {
    const void *nodes;
    int64_t n_nodes;
    const void *leaf;
    uint64_t ray_begin;
    uint32_t n_tris;
    uint32_t ray_count;
    float coord_max;
    float fo[3], fs[3], ft[3];  // PBRT_Q16 / SG_EQ scene frame
    const void *topo;           // split layouts: the topology array
};

// Largest s in [0, n) with tile_off[s] <= tile (tile_off has n + 1 entries,
// non-decreasing, tile_off[n] = total tiles > tile).
__device__ inline uint32_t find_scene(const uint32_t *tile_off, uint32_t n, uint32_t tile) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (tile_off[mid] <= tile) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Persistent kernel of one (layout, stack) group.  Waves take 64-ray tiles
// from the group's queue.  A wave works on one scene at a time: lanes whose
// ray ends are refilled from the wave's pool of claimed rays of that scene
// once 16 lanes are idle (a further tile of the same scene extends the pool);
// a claimed tile of another scene is held until every lane of the wave is
// idle, and then the wave switches scenes.  Each lane's stack is a ring in
// LDS over a spill area in global memory that the lane owns for the launch;
// rays that outgrow both go to the group's fallback list.  Every wave leaves
// the loop once the queue is drained and its lanes are idle (no wave ever
// waits on another), so the grid always drains.
constexpr uint32_t kNoRay = 0xFFFFFFFFu;
constexpr uint32_t kNoTile = 0xFFFFFFFFu;
constexpr uint32_t kBatchRefill = 16;
constexpr uint32_t kBatchSpillCap = 64;  // spill entries per lane beyond the LDS ring

template <int Layout, int SL>
__global__ __launch_bounds__(kTraceBlock) void k_batch_trace(const BatchScene *scenes,
                                                             const uint32_t *tile_off,
                                                             uint32_t n_scenes,
                                                             uint32_t total_tiles,
                                                             uint32_t *counter,
                                                             const bvh_ray *rays, bvh_hit *hits,
                                                             Fallback fb, SpillArea sa) {
    using Tr = typename TracerFor<Layout>::type;
    __shared__ uint32_t s_ref[SL * kTraceBlock];
    __shared__ float s_t[(Tr::kWithT ? SL : 1) * kTraceBlock];
    const uint32_t lane = threadIdx.x & 63u;
    SpillStack<Tr::kWithT, SL> st(s_ref, s_t, sa);
    // per lane
    uint32_t ray = kNoRay;  // ray index within the launch's ray array
    Ray r{};
    typename Tr::Prep prep{};
    typename Tr::State ts = Tr::start(0);
    uint32_t nf = 0, nt = 0;
    bool incomplete = false;
    // wave-uniform
    uint32_t scene = 0xFFFFFFFFu;  // scene of the wave's current rays
    uint64_t pool = 0, pool_end = 0;
    uint32_t pending = kNoTile;  // claimed tile of another scene
    bool drained = false;
    SceneData sd{};
    const void *nodes = nullptr;
    int64_t n_nodes = 0;
    for (;;) {
        const uint64_t idle = __builtin_amdgcn_ballot_w64(ray == kNoRay);
        const uint32_t nidle = (uint32_t)__builtin_popcountll(idle);
        if (nidle >= kBatchRefill) {
            // claim a further tile when the pool cannot fill the idle lanes
            if (pool_end - pool < nidle && pending == kNoTile && !drained) {
                const uint32_t leader = (uint32_t)__builtin_ctzll(idle);
                uint32_t t = 0;
                if (lane == leader) t = atomicAdd(counter, 1u);
                t = __builtin_amdgcn_readlane(t, leader);
                if (t >= total_tiles) drained = true;
                else pending = t;
            }
            // take the held tile once the pool is empty: at once for the same
            // scene, after every lane is idle for another scene
            if (pool == pool_end && pending != kNoTile) {
                const uint32_t s2 = find_scene(tile_off, n_scenes, pending);
                if (s2 == scene || nidle == 64u) {
                    const BatchScene c = scenes[s2];
                    if (s2 != scene) {
                        scene = s2;
                        nodes = c.nodes;
                        n_nodes = c.n_nodes;
                        sd = SceneData{c.leaf, nullptr, nullptr, c.n_tris, c.coord_max,
                                       {c.fo[0], c.fo[1], c.fo[2]}, {c.fs[0], c.fs[1], c.fs[2]},
                                       {c.ft[0], c.ft[1], c.ft[2]}, c.topo};
                    }
                    const uint64_t lo = (uint64_t)(pending - tile_off[s2]) * kTile;
                    pool = c.ray_begin + lo;
                    pool_end = c.ray_begin + min((uint64_t)c.ray_count, lo + kTile);
                    pending = kNoTile;
                }
            }
            const uint32_t avail = (uint32_t)(pool_end - pool);
            if (ray == kNoRay && avail > 0) {
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
                if (rank < avail) {
                    ray = (uint32_t)(pool + rank);
                    r = load_ray(rays, ray, sd.coord_max);
                    prep = Tr::prep(r);
                    ts = Tr::start(n_nodes);
                    st.reset();
                    nf = nt = 0;
                    incomplete = false;
                }
            }
            pool += min(avail, nidle);
        }
        const uint64_t busy = __builtin_amdgcn_ballot_w64(ray != kNoRay);
        if (busy == 0) {
            if (drained && pending == kNoTile && pool == pool_end) break;
            continue;
        }
        const bool coherent = rays_share_octant(r, ray != kNoRay, busy);
        if (ray != kNoRay) {
            const bool fast = wave_fast(r);
            if (coherent)
                Tr::template round<BVH_LEAF_COMPACT, BVH_TRACE_CLOSEST>(nodes, n_nodes, sd, r, prep,
                                                                        fast, st, ts, nf, nt,
                                                                        incomplete);
            else
                Tr::template step<BVH_LEAF_COMPACT, BVH_TRACE_CLOSEST>(nodes, n_nodes, sd, r, prep,
                                                                       fast, st, ts, nf, nt,
                                                                       incomplete);
            if (Tr::done(ts)) {
                if (incomplete) fallback_append(fb, ray);
                else store_hit(hits, ray, ts.best);
                ray = kNoRay;
            }
        }
    }
}

// The group's fallback: re-trace listed rays with a deep global stack; the
// scene of a ray is found from the scenes' ray ranges (disjoint, increasing).
template <int Layout>
__global__ __launch_bounds__(kTraceBlock) void k_batch_fallback(const BatchScene *scenes,
                                                                uint32_t n_scenes,
                                                                const bvh_ray *rays, bvh_hit *hits,
                                                                Fallback fb) {
    const uint32_t lane = blockIdx.x * kTraceBlock + threadIdx.x;
    const uint32_t total = *fb.count;
    for (uint32_t k = lane; k < total; k += kFallbackLanes) {
        const uint32_t i = fb.list[k];
        uint32_t lo = 0, hi = n_scenes;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (scenes[mid].ray_begin <= i) lo = mid;
            else hi = mid;
        }
        const BatchScene sc = scenes[lo];
        const Ray r = load_ray(rays, i, sc.coord_max);
        const SceneData ld{sc.leaf, nullptr, nullptr, sc.n_tris, sc.coord_max,
                               {sc.fo[0], sc.fo[1], sc.fo[2]}, {sc.fs[0], sc.fs[1], sc.fs[2]},
                               {sc.ft[0], sc.ft[1], sc.ft[2]}, sc.topo};
        uint32_t nf = 0, nt = 0;
        bool incomplete = false;
        GlobalStack<TracerFor<Layout>::type::kWithT> st(fb.stack_ref + (size_t)lane * kStackMax,
                                                        fb.stack_t + (size_t)lane * kStackMax);
        const Best b = trace_ray<Layout, BVH_LEAF_COMPACT, BVH_TRACE_CLOSEST>(
            sc.nodes, sc.n_nodes, ld, r, st, nf, nt, incomplete);
        store_hit(hits, i, b);
    }
}

__global__ void k_reset_counters(uint32_t *c, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0;
}

// 32-bit integer hash (C. Wellons' "lowbias32").
__device__ inline uint32_t hash32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
__device__ inline float unit_float(uint32_t h) { return (float)(h >> 8) * (1.0f / 16777216.0f); }

// Probe rays: origins uniform in the box, directions uniform on the sphere.
__global__ void k_probe_rays(bvh_ray *out, uint32_t n, float lx, float ly, float lz, float hx,
                             float hy, float hz, uint32_t seed) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t h = hash32(seed * 0x9E3779B9u ^ hash32(i));
    float u[5];
    for (int k = 0; k < 5; k++) {
        h = hash32(h + 0x632BE5ABu);
        u[k] = unit_float(h);
    }
    bvh_ray r;
    r.o[0] = lx + u[0] * (hx - lx);
    r.o[1] = ly + u[1] * (hy - ly);
    r.o[2] = lz + u[2] * (hz - lz);
    const float z = 2.0f * u[3] - 1.0f, phi = 6.2831853f * u[4];
    const float s = sqrtf(fmaxf(0.0f, 1.0f - z * z));
    r.d[0] = s * cosf(phi);
    r.d[1] = s * sinf(phi);
    r.d[2] = z;
    r.tmin = 0.0f;
    r.tmax = INFINITY;
    out[i] = r;
}

using KernelFn = void (*)(const BatchScene *, const uint32_t *, uint32_t, uint32_t, uint32_t *,
                          const bvh_ray *, bvh_hit *, Fallback, SpillArea);
using FallbackFn = void (*)(const BatchScene *, uint32_t, const bvh_ray *, bvh_hit *, Fallback);

FallbackFn fallback_for(int layout) {
    switch (layout) {
        case BVH_LAYOUT_AABB2: return &k_batch_fallback<BVH_LAYOUT_AABB2>;
        case BVH_LAYOUT_BVH4: return &k_batch_fallback<BVH_LAYOUT_BVH4>;
        case BVH_LAYOUT_BVH8_Q8: return &k_batch_fallback<BVH_LAYOUT_BVH8_Q8>;
        case BVH_LAYOUT_PBRT_Q16: return &k_batch_fallback<BVH_LAYOUT_PBRT_Q16>;
        case BVH_LAYOUT_SG_EQ: return &k_batch_fallback<BVH_LAYOUT_SG_EQ>;
        case BVH_LAYOUT_PBRT_SOAOS: return &k_batch_fallback<BVH_LAYOUT_PBRT_SOAOS>;
        case BVH_LAYOUT_PBRT_Q16_SOAOS: return &k_batch_fallback<BVH_LAYOUT_PBRT_Q16_SOAOS>;
        case BVH_LAYOUT_SG_EQ_A16: return &k_batch_fallback<BVH_LAYOUT_SG_EQ_A16>;
        default: return &k_batch_fallback<BVH_LAYOUT_BVH8_Q16>;
    }
}

template <int Layout>
KernelFn kernel_for_sl(int sl) {
    if (sl == 8) return &k_batch_trace<Layout, 8>;
    if (sl == 32) return &k_batch_trace<Layout, 32>;
    return &k_batch_trace<Layout, 16>;
}

KernelFn kernel_for(int layout, int sl) {
    switch (layout) {
        case BVH_LAYOUT_AABB2: return kernel_for_sl<BVH_LAYOUT_AABB2>(sl);
        case BVH_LAYOUT_BVH4: return kernel_for_sl<BVH_LAYOUT_BVH4>(sl);
        case BVH_LAYOUT_BVH8_Q8: return kernel_for_sl<BVH_LAYOUT_BVH8_Q8>(sl);
        case BVH_LAYOUT_PBRT_Q16: return kernel_for_sl<BVH_LAYOUT_PBRT_Q16>(sl);
        case BVH_LAYOUT_SG_EQ: return kernel_for_sl<BVH_LAYOUT_SG_EQ>(sl);
        case BVH_LAYOUT_PBRT_SOAOS: return kernel_for_sl<BVH_LAYOUT_PBRT_SOAOS>(sl);
        case BVH_LAYOUT_PBRT_Q16_SOAOS: return kernel_for_sl<BVH_LAYOUT_PBRT_Q16_SOAOS>(sl);
        case BVH_LAYOUT_SG_EQ_A16: return kernel_for_sl<BVH_LAYOUT_SG_EQ_A16>(sl);
        default: return kernel_for_sl<BVH_LAYOUT_BVH8_Q16>(sl);
    }
}

}  // namespace
}  // namespace bvhlib

using namespace bvhlib;

struct bvh_batch_s {
    int device = 0;
    std::vector<bvh_handle_s *> handles;
    std::vector<bvh_batch_scene_info> info;
    // graph cached for one (rays, hits, offsets) argument set
    const void *g_rays = nullptr;
    const void *g_hits = nullptr;
    std::vector<int64_t> g_offsets;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<void *> g_mem;  // device tables referenced by the graph

    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        for (void *p : g_mem) (void)hipFree(p);
        g_mem.clear();
        g_rays = g_hits = nullptr;
        g_offsets.clear();
    }
};

namespace bvhlib {
namespace {

// Times one handle on the probe rays: one warm-up launch, then the mean of
// three launches bracketed by events on the build stream.
int32_t time_trace(const bvh_handle_s *h, const bvh_ray *probe, uint64_t n, bvh_hit *hits,
                   hipStream_t s, hipEvent_t e0, hipEvent_t e1, float *ms) {
    BVH_TRY(trace_launch(h, probe, n, hits, BVH_TRACE_CLOSEST, s));
    BVH_HIP_TRY(hipEventRecord(e0, s));
    for (int k = 0; k < 3; k++) BVH_TRY(trace_launch(h, probe, n, hits, BVH_TRACE_CLOSEST, s));
    BVH_HIP_TRY(hipEventRecord(e1, s));
    BVH_HIP_TRY(hipEventSynchronize(e1));
    float t = 0.0f;
    BVH_HIP_TRY(hipEventElapsedTime(&t, e0, e1));
    *ms = t / 3.0f;
    return BVH_OK;
}

int32_t create_impl(const bvh_scene_desc *scenes, int32_t n_scenes, const bvh_tune_opts *opts,
                    hipStream_t s, bvh_batch_s *b) {
    const int32_t leaf_size = (opts && opts->leaf_size) ? opts->leaf_size : 4;
    // enough probe rays to fill the GPU, so that the timing sees the stack
    // depth's effect on occupancy as the batched launch will
    const int64_t probe_default = (opts && opts->probe_rays) ? opts->probe_rays : (1 << 19);
    int64_t max_probe = 0;
    for (int i = 0; i < n_scenes; i++) {
        int64_t np = probe_default;
        if (opts && opts->probe)
            np = std::min<int64_t>(np, opts->probe_offsets[i + 1] - opts->probe_offsets[i]);
        max_probe = std::max(max_probe, np);
    }
    bvh_ray *gen = nullptr;
    bvh_hit *hits = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int32_t rc = BVH_OK;
    auto cleanup = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (max_probe > 0) {
        Arena arena;
        arena.request(&hits, (size_t)max_probe);
        if (!(opts && opts->probe)) arena.request(&gen, (size_t)max_probe);
        rc = arena.bind(s, kAreaTune);
        if (rc != BVH_OK) return rc;
    }
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        cleanup();
        return set_error(BVH_EHIP, "bvh_batch_create: hipEventCreate failed");
    }
    b->handles.assign(n_scenes, nullptr);
    b->info.assign(n_scenes, bvh_batch_scene_info{});
    for (int i = 0; i < n_scenes && rc == BVH_OK; i++) {
        const bvh_scene_desc &sd = scenes[i];
        std::vector<int> layouts, sls;
        if (sd.layout >= 0) layouts.push_back(sd.layout);
        else {
            layouts = {BVH_LAYOUT_BVH8_Q8, BVH_LAYOUT_BVH4, BVH_LAYOUT_BVH8_Q16, BVH_LAYOUT_AABB2};
            if (leaf_size <= 15) {  // u4 leaf count
                layouts.push_back(BVH_LAYOUT_PBRT_Q16);
                layouts.push_back(BVH_LAYOUT_SG_EQ);
            }
        }
        if (sd.stack_lds > 0) sls.push_back(sd.stack_lds);
        else sls = {16, 8, 32};
        int64_t np = probe_default;
        const bvh_ray *probe = nullptr;
        if (opts && opts->probe) {
            np = std::min<int64_t>(np, opts->probe_offsets[i + 1] - opts->probe_offsets[i]);
            probe = opts->probe + opts->probe_offsets[i];
        }
        const bool choose = layouts.size() * sls.size() > 1 && sd.n_tris > 0 && np > 0;
        bvh_handle_s *best = nullptr;
        float best_ms = INFINITY;
        int ncand = 0;
        // stage 1: every candidate layout at the first stack depth; stage 2:
        // the other stack depths on the winning layout
        const int sl0 = sls[0];
        for (int layout : (choose ? layouts : std::vector<int>{layouts[0]})) {
            bvh_handle_s *h = nullptr;
            rc = build_handle(sd.verts, sd.n_verts, sd.tris, sd.n_tris, layout, leaf_size,
                              BVH_LEAF_COMPACT, sl0, BVH_BUILDER_LBVH, s, &h);
            if (rc != BVH_OK) break;
            if (!choose) {
                best = h;
                h->stack_lds = (sls.size() == 1) ? sl0 : 16;
                break;
            }
            if (!probe) {
                if (!gen) {
                    rc = set_error(BVH_EHIP, "bvh_batch_create: no probe buffer");
                    bvh_destroy(h);
                    break;
                }
                k_probe_rays<<<(unsigned)((np + 255) / 256), 256, 0, s>>>(
                    gen, (uint32_t)np, h->scene_lo[0], h->scene_lo[1], h->scene_lo[2], h->scene_hi[0],
                    h->scene_hi[1], h->scene_hi[2], 0x5EEDu + (uint32_t)i);
                probe = gen;
            }
            float ms = 0.0f;
            rc = time_trace(h, probe, (uint64_t)np, hits, s, e0, e1, &ms);
            if (rc != BVH_OK) {
                bvh_destroy(h);
                break;
            }
            ncand++;
            if (ms < best_ms) {
                best_ms = ms;
                if (best) bvh_destroy(best);
                best = h;
            } else {
                bvh_destroy(h);
            }
        }
        if (rc == BVH_OK && choose && best) {
            int keep_sl = sl0;
            for (size_t k = 1; k < sls.size(); k++) {
                best->stack_lds = sls[k];
                float ms = 0.0f;
                rc = time_trace(best, probe, (uint64_t)np, hits, s, e0, e1, &ms);
                if (rc != BVH_OK) break;
                ncand++;
                if (ms < best_ms) {
                    best_ms = ms;
                    keep_sl = sls[k];
                }
            }
            best->stack_lds = keep_sl;
        }
        if (rc != BVH_OK) {
            if (best) bvh_destroy(best);
            break;
        }
        b->handles[i] = best;
        bvh_batch_scene_info &inf = b->info[i];
        inf.layout = best->layout;
        inf.stack_lds = best->stack_lds;
        inf.candidates = choose ? ncand : 1;
        inf.probe_ns_per_ray = choose ? (float)(best_ms * 1e6 / (double)np) : 0.0f;
        inf.n_nodes = best->n_nodes;
        inf.bvh_bytes = best->n_nodes * best->node_bytes + best->n_tris * (int64_t)sizeof(bvh_tri);
    }
    cleanup();
    if (rc == BVH_OK) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = set_error(BVH_EHIP, "bvh_batch_create: %s", hipGetErrorString(e));
    }
    return rc;
}

template <typename T>
int32_t upload(bvh_batch_s *b, const std::vector<T> &v, T **out) {
    void *p = nullptr;
    BVH_HIP_TRY(hipMalloc(&p, std::max<size_t>(v.size(), 1) * sizeof(T)));
    b->g_mem.push_back(p);
    if (!v.empty()) BVH_HIP_TRY(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    *out = static_cast<T *>(p);
    return BVH_OK;
}

// Builds and instantiates the graph for one argument set: a counter-reset
// kernel, then per (layout, stack) variant its persistent kernel and its
// fallback pass, the variants one after another (each fills the GPU, and
// they share one per-lane stack spill area).
int32_t make_graph(bvh_batch_s *b, const bvh_ray *rays, const int64_t *offsets, bvh_hit *hits) {
    b->drop_graph();
    const int n = (int)b->handles.size();
    std::map<std::pair<int, int>, std::vector<int>> groups;
    for (int i = 0; i < n; i++) {
        const int64_t cnt = offsets[i + 1] - offsets[i];
        if (cnt <= 0) continue;
        groups[{b->handles[i]->layout, b->handles[i]->stack_lds}].push_back(i);
    }
    int n_cu = 0;
    BVH_HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, b->device));
    // counters[g]: work queue of group g; counters[ngroups + g]: its fallback count
    const int ngroups = (int)groups.size();
    uint32_t *counters = nullptr;
    BVH_TRY(upload(b, std::vector<uint32_t>(std::max<size_t>(2 * groups.size(), 1), 0u), &counters));
    BVH_HIP_TRY(hipGraphCreate(&b->graph, 0));
    hipGraphNode_t reset;
    {
        int nctr = 2 * ngroups;
        void *args[] = {&counters, &nctr};
        hipKernelNodeParams p{};
        p.func = reinterpret_cast<void *>(&k_reset_counters);
        p.gridDim = dim3((unsigned)((2 * ngroups + 255) / 256 + 1));
        p.blockDim = dim3(256);
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        BVH_HIP_TRY(hipGraphAddKernelNode(&reset, b->graph, nullptr, 0, &p));
    }
    int g = 0;
    hipGraphNode_t prev = reset;
    void *spill = nullptr;
    uint32_t spill_lanes = 0;
    for (auto &kv : groups) {
        std::vector<BatchScene> sc;
        std::vector<uint32_t> toff(1, 0);
        for (int i : kv.second) {
            const bvh_handle_s *h = b->handles[i];
            const int64_t cnt = offsets[i + 1] - offsets[i];
            if (cnt > 0xFFFFFFFFll) return set_error(BVH_EUNSUPPORTED, "bvh_batch_trace: scene ray count");
            sc.push_back(BatchScene{h->nodes, h->n_nodes, h->leaf, (uint64_t)offsets[i],
                                    (uint32_t)h->n_tris, (uint32_t)cnt, h->coord_max(),
                                    {h->frame_origin[0], h->frame_origin[1], h->frame_origin[2]},
                                    {h->frame_scale[0], h->frame_scale[1], h->frame_scale[2]},
                                    {h->frame_top[0], h->frame_top[1], h->frame_top[2]},
                                    topo_of(h->nodes, h->n_nodes, h->layout)});
            const uint64_t tiles = ((uint64_t)cnt + kTile - 1) / kTile;
            if (toff.back() + tiles > 0xFFFFFFFFull)
                return set_error(BVH_EUNSUPPORTED, "bvh_batch_trace: too many rays");
            toff.push_back(toff.back() + (uint32_t)tiles);
        }
        BatchScene *d_sc = nullptr;
        uint32_t *d_toff = nullptr;
        BVH_TRY(upload(b, sc, &d_sc));
        BVH_TRY(upload(b, toff, &d_toff));
        const KernelFn fn = kernel_for(kv.first.first, kv.first.second);
        int per_cu = 0;
        BVH_TRY(blocks_per_cu(reinterpret_cast<const void *>(fn), b->device, per_cu));
        const uint32_t total = toff.back();
        const uint32_t waves_per_block = kTraceBlock / 64;
        uint64_t group_rays = 0;
        for (const BatchScene &x : sc) group_rays += x.ray_count;
        // the groups run one after another, each on the whole GPU
        const uint64_t resident = (uint64_t)std::max(per_cu, 1) * (uint64_t)n_cu;
        uint32_t grid = (uint32_t)std::min<uint64_t>(resident, (total + waves_per_block - 1) / waves_per_block);
        grid = std::max<uint32_t>(grid, 1);
        uint32_t nsc = (uint32_t)sc.size();
        uint32_t *ctr = counters + g;
        const bvh_ray *r = rays;
        bvh_hit *hh = hits;
        // fallback work area of this group (list sized for all its rays),
        // then the per-lane stack spill area of its grid
        const uint32_t lanes = grid * kTraceBlock;
        void *ws = nullptr;
        BVH_HIP_TRY(hipMalloc(&ws, fallback_bytes(group_rays)));
        b->g_mem.push_back(ws);
        Fallback fb = fallback_view(ws, group_rays);
        fb.count = counters + ngroups + g;
        if (lanes > spill_lanes) {  // the shared spill area, sized for the largest grid
            spill_lanes = n_cu * 32u * 64u;  // every lane the GPU can hold
            BVH_HIP_TRY(hipMalloc(&spill, (size_t)spill_lanes * kBatchSpillCap * 8));
            b->g_mem.push_back(spill);
        }
        SpillArea sa;
        sa.ent = static_cast<uint2 *>(spill);
        sa.lanes = lanes;
        sa.cap = kBatchSpillCap;
        void *args[] = {&d_sc, &d_toff, &nsc, (void *)&total, &ctr, &r, &hh, &fb, &sa};
        hipKernelNodeParams p{};
        p.func = reinterpret_cast<void *>(fn);
        p.gridDim = dim3(grid);
        p.blockDim = dim3(kTraceBlock);
        p.sharedMemBytes = 0;
        p.kernelParams = args;
        p.extra = nullptr;
        hipGraphNode_t node;
        BVH_HIP_TRY(hipGraphAddKernelNode(&node, b->graph, &prev, 1, &p));
        void *fargs[] = {&d_sc, &nsc, &r, &hh, &fb};
        hipKernelNodeParams q{};
        q.func = reinterpret_cast<void *>(fallback_for(kv.first.first));
        q.gridDim = dim3(kFallbackBlocks);
        q.blockDim = dim3(kTraceBlock);
        q.sharedMemBytes = 0;
        q.kernelParams = fargs;
        q.extra = nullptr;
        hipGraphNode_t fnode;
        BVH_HIP_TRY(hipGraphAddKernelNode(&fnode, b->graph, &node, 1, &q));
        prev = fnode;
        g++;
    }
    BVH_HIP_TRY(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->g_rays = rays;
    b->g_hits = hits;
    b->g_offsets.assign(offsets, offsets + n + 1);
    return BVH_OK;
}

}  // namespace
}  // namespace bvhlib

extern "C" int32_t bvh_batch_create(const bvh_scene_desc *scenes, int32_t n_scenes,
                                    const bvh_tune_opts *opts, void *stream, bvh_batch_t *out) {
    if (!out) return set_error(BVH_EINVAL, "bvh_batch_create: out is null");
    *out = nullptr;
    if (n_scenes < 1 || !scenes) return set_error(BVH_EINVAL, "bvh_batch_create: no scenes");
    if (opts) {
        for (int k = 0; k < 4; k++)
            if (opts->reserved[k]) return set_error(BVH_EINVAL, "bvh_batch_create: reserved option set");
        if (opts->probe_rays < 0) return set_error(BVH_EINVAL, "bvh_batch_create: probe_rays < 0");
        if (opts->leaf_size < 0 || opts->leaf_size > kMaxLeafSize)
            return set_error(BVH_EINVAL, "bvh_batch_create: leaf_size %d", opts->leaf_size);
        if (opts->probe && !opts->probe_offsets)
            return set_error(BVH_EINVAL, "bvh_batch_create: probe without probe_offsets");
        if (opts->probe)
            for (int i = 0; i < n_scenes; i++)
                if (opts->probe_offsets[i + 1] < opts->probe_offsets[i] || opts->probe_offsets[0] < 0)
                    return set_error(BVH_EINVAL, "bvh_batch_create: probe_offsets not non-decreasing");
    }
    for (int i = 0; i < n_scenes; i++) {
        const bvh_scene_desc &sd = scenes[i];
        if (sd.n_tris < 0 || sd.n_verts < 0 || (sd.n_tris > 0 && (!sd.verts || !sd.tris)) ||
            (sd.n_tris > 0 && sd.n_verts == 0))
            return set_error(BVH_EINVAL, "bvh_batch_create: bad mesh for scene %d", i);
        if (sd.layout < -1 || sd.layout >= BVH_NUM_LAYOUTS)
            return set_error(BVH_EINVAL, "bvh_batch_create: bad layout for scene %d", i);
        if (sd.layout == BVH_LAYOUT_SHARED_SLAB)
            return set_error(BVH_EUNSUPPORTED,
                             "bvh_batch_create: scene %d: the shared-slab layout is not batched", i);
        if (sd.stack_lds != 0 && sd.stack_lds != 8 && sd.stack_lds != 16 && sd.stack_lds != 32)
            return set_error(BVH_EINVAL, "bvh_batch_create: bad stack_lds for scene %d", i);
        if (sd.reserved[0] || sd.reserved[1])
            return set_error(BVH_EINVAL, "bvh_batch_create: reserved field set for scene %d", i);
        if (sd.n_tris > kMaxTris)
            return set_error(BVH_EUNSUPPORTED, "bvh_batch_create: scene %d too large", i);
    }
    BVH_TRY(require_device());
    bvh_batch_s *b = new bvh_batch_s;
    if (hipGetDevice(&b->device) != hipSuccess) {
        delete b;
        return set_error(BVH_ENODEV, "bvh_batch_create: no device");
    }
    const int32_t rc = create_impl(scenes, n_scenes, opts, static_cast<hipStream_t>(stream), b);
    if (rc != BVH_OK) {
        std::string msg = bvh_last_error();
        bvh_batch_destroy(b);
        return set_error(rc, "%s", msg.c_str());
    }
    *out = b;
    return BVH_OK;
}

extern "C" int32_t bvh_batch_get_scene_info(bvh_batch_t b, int32_t scene, bvh_batch_scene_info *out) {
    if (!b || !out || scene < 0 || scene >= (int32_t)b->info.size())
        return set_error(BVH_EINVAL, "bvh_batch_get_scene_info: bad argument");
    *out = b->info[scene];
    return BVH_OK;
}

extern "C" int32_t bvh_batch_scene_handle(bvh_batch_t b, int32_t scene, bvh_handle_t *out) {
    if (!b || !out || scene < 0 || scene >= (int32_t)b->handles.size())
        return set_error(BVH_EINVAL, "bvh_batch_scene_handle: bad argument");
    *out = b->handles[scene];
    return BVH_OK;
}

extern "C" int32_t bvh_batch_trace(bvh_batch_t b, const bvh_ray *rays, const int64_t *ray_offsets,
                                   bvh_hit *hits, void *stream) {
    if (!b || !ray_offsets) return set_error(BVH_EINVAL, "bvh_batch_trace: null argument");
    const int n = (int)b->handles.size();
    if (ray_offsets[0] < 0) return set_error(BVH_EINVAL, "bvh_batch_trace: negative offset");
    for (int i = 0; i < n; i++)
        if (ray_offsets[i + 1] < ray_offsets[i])
            return set_error(BVH_EINVAL, "bvh_batch_trace: ray_offsets not non-decreasing");
    if (ray_offsets[n] > ray_offsets[0] && (!rays || !hits))
        return set_error(BVH_EINVAL, "bvh_batch_trace: null ray or hit buffer");
    if (ray_offsets[n] == ray_offsets[0]) return BVH_OK;
    if (ray_offsets[n] > (int64_t)0xFFFFFFFFll)
        return set_error(BVH_EUNSUPPORTED, "bvh_batch_trace: more than 2^32 - 1 rays");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != b->device)
        return set_error(BVH_EINVAL, "bvh_batch_trace: batch belongs to another device");
    const bool same = b->exec && b->g_rays == rays && b->g_hits == hits &&
                      std::equal(b->g_offsets.begin(), b->g_offsets.end(), ray_offsets);
    if (!same) BVH_TRY(make_graph(b, rays, ray_offsets, hits));
    BVH_HIP_TRY(hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream)));
    return BVH_OK;
}

extern "C" int32_t bvh_batch_destroy(bvh_batch_t b) {
    if (!b) return BVH_OK;
    (void)hipDeviceSynchronize();
    b->drop_graph();
    for (bvh_handle_s *h : b->handles)
        if (h) bvh_destroy(h);
    delete b;
    return BVH_OK;
}
