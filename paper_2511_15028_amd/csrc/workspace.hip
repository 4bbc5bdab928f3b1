// Grow-only device work areas, one per (device, stream, purpose), kept until
// the process ends.  Builds and traces on one stream are ordered by that
// stream, so they can reuse its area; work on different streams gets
// different areas.  In steady state no call allocates or frees device memory
// (stream-ordered frees cost up to milliseconds each on this platform).
#include <map>
#include <mutex>
#include <tuple>

#include "internal.h"

namespace bvhlib {
namespace {

struct Area {
    void *ptr = nullptr;
    size_t bytes = 0;
};

std::mutex g_mutex;
std::map<std::tuple<int, hipStream_t, int>, Area> g_areas;

}  // namespace

int32_t stream_workspace(hipStream_t s, int purpose, size_t bytes, void **out) {
    *out = nullptr;
    int dev = 0;
    BVH_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_mutex);
    Area &a = g_areas[std::make_tuple(dev, s, purpose)];
    if (a.bytes < bytes) {
        if (a.ptr) {
            // the old area may still be in use by queued work on this stream
            BVH_HIP_TRY(hipStreamSynchronize(s));
            BVH_HIP_TRY(hipFree(a.ptr));
            a.ptr = nullptr;
            a.bytes = 0;
        }
        const size_t grow = bytes + bytes / 4;  // headroom against repeated growth
        hipError_t e = hipMalloc(&a.ptr, grow);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            a.ptr = nullptr;
            return set_error(BVH_ENOMEM, "work area of %zu bytes: %s", grow, hipGetErrorString(e));
        }
        a.bytes = grow;
    }
    *out = a.ptr;
    return BVH_OK;
}

}  // namespace bvhlib
