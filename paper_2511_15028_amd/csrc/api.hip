// Handle management, errors and introspection calls of the C ABI.
#include <cstring>
#include <string>

#include "internal.h"

namespace bvhlib {

static thread_local std::string g_last_error;

int32_t set_error(int32_t code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int32_t require_device() {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return set_error(BVH_ENODEV, "no HIP device available");
    }
    return BVH_OK;
}

}  // namespace bvhlib

using namespace bvhlib;

extern "C" const char *bvh_last_error(void) { return g_last_error.c_str(); }

extern "C" int32_t bvh_version(void) { return 1; }

extern "C" int32_t bvh_destroy(bvh_handle_t h) {
    if (!h) return BVH_OK;
    int prev = 0;
    bool have_prev = hipGetDevice(&prev) == hipSuccess;
    if (hipSetDevice(h->device) == hipSuccess) {
        (void)hipDeviceSynchronize();
        if (h->block) (void)hipFree(h->block);
        if (h->node_block) (void)hipFree(h->node_block);
    }
    if (have_prev) (void)hipSetDevice(prev);
    delete h;
    return BVH_OK;
}

static int64_t leaf_buffer_bytes(const bvh_handle_s *h) {
    return h->leaf_mode == BVH_LEAF_COMPACT ? h->n_tris * (int64_t)sizeof(bvh_tri)
                                            : h->n_tris * (int64_t)sizeof(int32_t);
}

extern "C" int32_t bvh_get_stats(bvh_handle_t h, bvh_stats *out) {
    if (!h || !out) return set_error(BVH_EINVAL, "bvh_get_stats: null argument");
    std::memset(out, 0, sizeof(*out));
    out->layout = h->layout;
    out->leaf_mode = h->leaf_mode;
    out->arity = h->arity;
    out->leaf_size = h->leaf_size;
    out->n_tris = h->n_tris;
    out->n_nodes = h->n_nodes;
    out->n_leaves = h->n_leaves;
    out->node_bytes = h->node_bytes;
    out->nodes_buffer_bytes = h->n_nodes * h->node_bytes;
    out->leaf_buffer_bytes = leaf_buffer_bytes(h);
    out->extra_bytes = h->leaf_mode == BVH_LEAF_INDEXED
                           ? h->n_verts * 12 + h->n_tris * 12
                           : 0;
    out->depth = h->depth;
    out->max_stack = h->max_stack;
    for (int a = 0; a < 3; a++) {
        out->scene_lo[a] = h->scene_lo[a];
        out->scene_hi[a] = h->scene_hi[a];
    }
    out->stack_lds = h->stack_lds;
    out->builder = h->builder;
    for (int a = 0; a < 3; a++) {
        out->frame_origin[a] = h->frame_origin[a];
        out->frame_scale[a] = h->frame_scale[a];
        out->frame_top[a] = h->frame_top[a];
    }
    return BVH_OK;
}

extern "C" int32_t bvh_read_buffer(bvh_handle_t h, int32_t which, void *host_dst,
                                   int64_t capacity, int64_t *bytes_total) {
    if (!h) return set_error(BVH_EINVAL, "bvh_read_buffer: null handle");
    if (capacity < 0 || (capacity > 0 && !host_dst))
        return set_error(BVH_EINVAL, "bvh_read_buffer: bad destination");
    const void *src = nullptr;
    int64_t size = 0;
    if (which == BVH_BUF_NODES) {
        src = h->nodes;
        size = h->n_nodes * h->node_bytes;
    } else if (which == BVH_BUF_LEAF) {
        src = h->leaf;
        size = leaf_buffer_bytes(h);
    } else {
        return set_error(BVH_EINVAL, "bvh_read_buffer: unknown buffer %d", which);
    }
    if (bytes_total) *bytes_total = size;
    int64_t nbytes = capacity < size ? capacity : size;
    if (nbytes > 0 && src) {
        BVH_TRY(require_device());
        BVH_HIP_TRY(hipSetDevice(h->device));
        BVH_HIP_TRY(hipDeviceSynchronize());
        BVH_HIP_TRY(hipMemcpy(host_dst, src, (size_t)nbytes, hipMemcpyDeviceToHost));
    }
    return BVH_OK;
}
