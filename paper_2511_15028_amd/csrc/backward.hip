// Backward pass of closest-hit tracing with the hit primitive held fixed.
//
// The hit point obeys F = o + t d - (1-u-v) p0 - u p1 - v p2 = 0 (the
// barycentric form of App. G's Moller-Trumbore result).  With
// J = dF/d(t,u,v) = [d | p0-p1 | p0-p2] and g = dL/d(t,u,v), the solution of
// J^T lam = g gives dL/dx = -lam^T dF/dx for every input x:
//   dL/do = -lam, dL/dd = -t lam, dL/dp0 = (1-u-v) lam, dL/dp1 = u lam,
//   dL/dp2 = v lam.
// lam comes from Cramer's rule with the rows a = d, b = p0-p1, c = p0-p2 of
// J^T: lam = (g_t (b x c) + g_u (c x a) + g_v (a x b)) / (a . (b x c)).
#include "internal.h"

namespace bvhlib {
namespace {

constexpr int kBlock = 256;

__global__ __launch_bounds__(kBlock) void k_backward(const float *verts, int64_t n_verts,
                                                     const int32_t *tris, int64_t n_tris,
                                                     const bvh_ray *rays, uint64_t n,
                                                     const bvh_hit *hits, const float *grad_hits,
                                                     float *grad_verts, float *grad_rays) {
    const uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    float out[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const int4 hw = reinterpret_cast<const int4 *>(hits)[i];
    const int32_t prim = hw.x;
    bool ok = prim >= 0 && (int64_t)prim < n_tris;
    int32_t idx[3] = {0, 0, 0};
    if (ok) {
        for (int k = 0; k < 3; k++) {
            idx[k] = tris[3 * (size_t)prim + k];
            ok = ok && idx[k] >= 0 && (int64_t)idx[k] < n_verts;
        }
    }
    if (ok) {
        const float t = __int_as_float(hw.y), u = __int_as_float(hw.z), v = __int_as_float(hw.w);
        const float4 *rp = reinterpret_cast<const float4 *>(rays + i);
        const float4 ra = rp[0], rb = rp[1];
        const float *q0 = verts + 3 * (size_t)idx[0];
        const float *q1 = verts + 3 * (size_t)idx[1];
        const float *q2 = verts + 3 * (size_t)idx[2];
        const float ax = rb.x, ay = rb.y, az = rb.z;                       // d
        const float bx = q0[0] - q1[0], by = q0[1] - q1[1], bz = q0[2] - q1[2];  // p0 - p1
        const float cx = q0[0] - q2[0], cy = q0[1] - q2[1], cz = q0[2] - q2[2];  // p0 - p2
        const float bcx = by * cz - bz * cy, bcy = bz * cx - bx * cz, bcz = bx * cy - by * cx;
        const float cax = cy * az - cz * ay, cay = cz * ax - cx * az, caz = cx * ay - cy * ax;
        const float abx = ay * bz - az * by, aby = az * bx - ax * bz, abz = ax * by - ay * bx;
        const float det = ax * bcx + ay * bcy + az * bcz;
        (void)ra;
        if (det != 0.0f) {
            const float gt = grad_hits[3 * i], gu = grad_hits[3 * i + 1], gv = grad_hits[3 * i + 2];
            const float inv = 1.0f / det;
            const float lx = (gt * bcx + gu * cax + gv * abx) * inv;
            const float ly = (gt * bcy + gu * cay + gv * aby) * inv;
            const float lz = (gt * bcz + gu * caz + gv * abz) * inv;
            out[0] = -lx; out[1] = -ly; out[2] = -lz;
            out[3] = -t * lx; out[4] = -t * ly; out[5] = -t * lz;
            const float w[3] = {1.0f - u - v, u, v};
            for (int k = 0; k < 3; k++) {
                float *g = grad_verts + 3 * (size_t)idx[k];
                unsafeAtomicAdd(g + 0, w[k] * lx);
                unsafeAtomicAdd(g + 1, w[k] * ly);
                unsafeAtomicAdd(g + 2, w[k] * lz);
            }
        }
    }
    float *gr = grad_rays + 6 * i;
    for (int k = 0; k < 6; k++) gr[k] = out[k];
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
    const unsigned grid = (unsigned)(((uint64_t)n + kBlock - 1) / kBlock);
    k_backward<<<grid, kBlock, 0, static_cast<hipStream_t>(stream)>>>(
        verts, n_verts, tris, n_tris, rays, (uint64_t)n, hits, grad_hits, grad_verts, grad_rays);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(BVH_EHIP, "bvh_trace_backward: launch failed: %s", hipGetErrorString(e));
    return BVH_OK;
}
