// Internal definitions shared by the library's HIP sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <algorithm>
#include <vector>

#include "bvh.h"

namespace bvhlib {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
int32_t set_error(int32_t code, const char *fmt, ...);

#define BVH_HIP_TRY(expr)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) {                                                             \
            if (e_ == hipErrorOutOfMemory)                                                  \
                return ::bvhlib::set_error(BVH_ENOMEM, "%s: %s", #expr, hipGetErrorString(e_)); \
            return ::bvhlib::set_error(BVH_EHIP, "%s: %s", #expr, hipGetErrorString(e_));   \
        }                                                                                   \
    } while (0)

#define BVH_TRY(expr)                       \
    do {                                    \
        int32_t rc_ = (expr);               \
        if (rc_ != BVH_OK) return rc_;      \
    } while (0)

// Fails with ENODEV when no HIP device is present.
int32_t require_device();



// ---------------------------------------------------------------------------
// Limits shared by build and trace
// ---------------------------------------------------------------------------
constexpr int kMaxLeafSize = 16;
constexpr int64_t kMaxTris = (int64_t(1) << 27) - 1;   // leaf ref has 27 offset bits
// Traversal stack bound: the fast pass keeps 8, 16 or 32 entries per lane in
// LDS; rays that need more are re-traced with a deep stack of kStackMax
// entries, so a tree's worst-case stack need must not exceed it.
constexpr int kStackMax = 256;

// ---------------------------------------------------------------------------
// Handle
// ---------------------------------------------------------------------------
}  // namespace bvhlib

struct bvh_handle_s {
    int device = 0;
    int32_t layout = 0;
    int32_t leaf_mode = 0;
    int32_t leaf_size = 4;
    int32_t stack_lds = 16;
    bool stack_lds_default = false;  // stack_lds left to the build's default
    int32_t builder = BVH_BUILDER_LBVH;
    int32_t arity = 2;
    int64_t n_tris = 0;
    int64_t n_verts = 0;
    int64_t n_nodes = 0;
    int64_t n_leaves = 0;
    int64_t node_bytes = 0;
    int32_t depth = 0;
    int32_t max_stack = 0;
    float scene_lo[3] = {0, 0, 0};
    float scene_hi[3] = {0, 0, 0};
    float frame_origin[3] = {0, 0, 0};  // PBRT_Q16, SG_EQ: lo = fmaf(q, frame_scale, frame_origin)
    float frame_scale[3] = {0, 0, 0};
    float frame_top[3] = {0, 0, 0};     // SG_EQ: hi = fmaf(-q, frame_scale, frame_top)
    void *block = nullptr;       // device allocation of leaf, verts and tris
    void *node_block = nullptr;  // device allocation of the node records
    uint32_t node_block_cap = 0; // records node_block holds
    void *nodes = nullptr;       // node records
    void *leaf = nullptr;        // bvh_tri[n_tris] or int32 prim id[n_tris]
    float *verts = nullptr;      // INDEXED: own copy of the vertices
    int32_t *tris = nullptr;     // INDEXED: own copy of the triangle indices

    // Largest coordinate magnitude of the scene box (+inf for an empty or
    // non-finite scene): decides which slab-distance form the kernels use.
    float coord_max() const {
        float m = 0.0f;
        for (int a = 0; a < 3; a++) {
            const float l = scene_lo[a] < 0 ? -scene_lo[a] : scene_lo[a];
            const float u = scene_hi[a] < 0 ? -scene_hi[a] : scene_hi[a];
            m = l > m ? l : m;
            m = u > m ? u : m;
            if (!(scene_lo[a] <= scene_hi[a])) return __builtin_inff();
        }
        return n_tris > 0 ? m : __builtin_inff();
    }
};

namespace bvhlib {

inline int64_t node_record_bytes(int32_t layout) {
    switch (layout) {
        case BVH_LAYOUT_AABB2: return sizeof(bvh_node_aabb2);
        case BVH_LAYOUT_BVH4: return sizeof(bvh_node_bvh4);
        case BVH_LAYOUT_BVH8_Q8: return sizeof(bvh_node_bvh8_q8);
        case BVH_LAYOUT_BVH8_Q16: return sizeof(bvh_node_bvh8_q16);
        case BVH_LAYOUT_PBRT_Q16: return sizeof(bvh_node_pbrt_q16);
        case BVH_LAYOUT_SG_EQ: return sizeof(bvh_node_sg_eq);
        case BVH_LAYOUT_PBRT_SOAOS: return sizeof(bvh_node_box_f32) + sizeof(bvh_node_topo);
        case BVH_LAYOUT_PBRT_Q16_SOAOS: return sizeof(bvh_node_box_q16) + sizeof(uint32_t);
        case BVH_LAYOUT_SG_EQ_A16: return sizeof(bvh_node_sg_eq_a16);
        case BVH_LAYOUT_SHARED_SLAB: return sizeof(bvh_node_slab);
        default: return 0;
    }
}

inline int32_t layout_arity(int32_t layout) {
    switch (layout) {
        case BVH_LAYOUT_AABB2: return 2;
        case BVH_LAYOUT_PBRT_Q16: return 2;
        case BVH_LAYOUT_SG_EQ: return 2;
        case BVH_LAYOUT_PBRT_SOAOS: return 2;
        case BVH_LAYOUT_PBRT_Q16_SOAOS: return 2;
        case BVH_LAYOUT_SG_EQ_A16: return 2;
        case BVH_LAYOUT_SHARED_SLAB: return 2;
        case BVH_LAYOUT_BVH4: return 4;
        default: return 8;
    }
}

// EINVAL unless the calling thread's current device is the handle's device.
int32_t check_handle_device(const bvh_handle_s *h, const char *who);

// Builds one BVH (bvh_build after argument checks); used by the batch path.
int32_t build_handle(const float *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                     int32_t layout, int32_t leaf_size, int32_t leaf_mode, int32_t stack_lds,
                     int32_t builder, hipStream_t s, bvh_handle_s **out);

// bvh_trace without argument checks (closest or any hit, no counters).
int32_t trace_launch(const bvh_handle_s *h, const bvh_ray *rays, uint64_t n, bvh_hit *hits,
                     int32_t mode, hipStream_t s);

// ---------------------------------------------------------------------------
// Device work areas (workspace.hip): grow-only, one per (device, stream,
// purpose), kept until the process ends.  Callers that use one stream from
// several host threads must serialise those calls themselves.
// ---------------------------------------------------------------------------
enum AreaPurpose {
    kAreaBuild = 0,
    kAreaBuildWide = 1,
    kAreaTrace = 2,
    kAreaTune = 3,
    kAreaSah = 4,
    kAreaBackward = 5
};
int32_t stream_workspace(hipStream_t s, int purpose, size_t bytes, void **out);

// Carves several device buffers out of one work area: request() them all,
// then bind() once.
class Arena {
  public:
    template <typename T>
    void request(T **slot, size_t count) {
        reqs_.push_back(Req{reinterpret_cast<void **>(slot), total_});
        total_ += (std::max<size_t>(count, 1) * sizeof(T) + 255) & ~size_t(255);
    }
    int32_t bind(hipStream_t s, int purpose) {
        void *base = nullptr;
        int32_t rc = stream_workspace(s, purpose, total_, &base);
        if (rc != 0) return rc;
        for (const Req &r : reqs_) *r.slot = static_cast<char *>(base) + r.offset;
        return 0;
    }
    size_t bytes() const { return total_; }

  private:
    struct Req {
        void **slot;
        size_t offset;
    };
    std::vector<Req> reqs_;
    size_t total_ = 0;
};

static_assert(sizeof(bvh_ray) == 32, "bvh_ray");
static_assert(sizeof(bvh_hit) == 16, "bvh_hit");
static_assert(sizeof(bvh_point_query) == 16, "bvh_point_query");
static_assert(sizeof(bvh_closest) == 16, "bvh_closest");
static_assert(sizeof(bvh_tri) == 48, "bvh_tri");
static_assert(sizeof(bvh_node_aabb2) == 32, "aabb2 node");
static_assert(sizeof(bvh_node_pbrt_q16) == 16, "pbrt-q16 node");
static_assert(sizeof(bvh_node_sg_eq) == 12, "sg-eq node");
static_assert(sizeof(bvh_node_box_f32) == 24 && sizeof(bvh_node_topo) == 8, "pbrt-soaos arrays");
static_assert(sizeof(bvh_node_box_q16) == 12, "pbrt-q16-soaos boxes");
static_assert(sizeof(bvh_node_sg_eq_a16) == 16, "sg-eq-align16 node");
static_assert(sizeof(bvh_node_slab) == 16, "shared-slab node");

// Layouts whose node buffer is a box array followed by a topology array, and
// the bytes of one box entry.
inline bool layout_split(int32_t layout) {
    return layout == BVH_LAYOUT_PBRT_SOAOS || layout == BVH_LAYOUT_PBRT_Q16_SOAOS;
}
inline int64_t split_box_bytes(int32_t layout) {
    return layout == BVH_LAYOUT_PBRT_SOAOS ? (int64_t)sizeof(bvh_node_box_f32)
                                           : (int64_t)sizeof(bvh_node_box_q16);
}
// The topology array of a split layout (after the n_nodes box entries).
inline const void *topo_of(const void *nodes, int64_t n_nodes, int32_t layout) {
    return layout_split(layout)
               ? static_cast<const char *>(nodes) + split_box_bytes(layout) * n_nodes
               : nullptr;
}
// Scene-frame quantised layouts (PBRT_Q16, SG_EQ and their variants).
inline bool layout_scene_frame(int32_t layout) {
    return layout == BVH_LAYOUT_PBRT_Q16 || layout == BVH_LAYOUT_SG_EQ ||
           layout == BVH_LAYOUT_PBRT_Q16_SOAOS || layout == BVH_LAYOUT_SG_EQ_A16;
}
inline bool layout_sg_eq(int32_t layout) {
    return layout == BVH_LAYOUT_SG_EQ || layout == BVH_LAYOUT_SG_EQ_A16;
}
static_assert(sizeof(bvh_node_bvh4) == 128, "bvh4 node");
static_assert(sizeof(bvh_node_bvh8_q8) == 128, "bvh8 q8 node");
static_assert(sizeof(bvh_node_bvh8_q16) == 160, "bvh8 q16 node");

// Child reference encoding (see bvh.h).
__host__ __device__ inline uint32_t ref_interior(uint32_t node) { return (node << 1) | 1u; }
__host__ __device__ inline uint32_t ref_leaf(uint32_t first, uint32_t n) {
    return (first << 5) | ((n - 1u) << 1);
}
constexpr uint32_t kRefEmpty = 0xFFFFFFFFu;

}  // namespace bvhlib
