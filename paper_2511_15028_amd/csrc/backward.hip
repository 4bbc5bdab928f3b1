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

// lam and the ray gradient of ray i; false for a miss, an out-of-range
// primitive or vertex index, or a singular system.
__device__ inline bool ray_grad(const float *verts, int64_t n_verts, const int32_t *tris,
                                int64_t n_tris, const bvh_ray *rays, const bvh_hit *hits,
                                const float *grad_hits, uint64_t i, float *out, int32_t *idx,
                                float *w, float *lam) {
    const int4 hw = reinterpret_cast<const int4 *>(hits)[i];
    const int32_t prim = hw.x;
    if (prim < 0 || (int64_t)prim >= n_tris) return false;
    for (int k = 0; k < 3; k++) {
        idx[k] = tris[3 * (size_t)prim + k];
        if (idx[k] < 0 || (int64_t)idx[k] >= n_verts) return false;
    }
    const float t = __int_as_float(hw.y), u = __int_as_float(hw.z), v = __int_as_float(hw.w);
    const float4 rb = reinterpret_cast<const float4 *>(rays + i)[1];
    const float *q0 = verts + 3 * (size_t)idx[0];
    const float *q1 = verts + 3 * (size_t)idx[1];
    const float *q2 = verts + 3 * (size_t)idx[2];
    const float ax = rb.x, ay = rb.y, az = rb.z;                              // d
    const float bx = q0[0] - q1[0], by = q0[1] - q1[1], bz = q0[2] - q1[2];  // p0 - p1
    const float cx = q0[0] - q2[0], cy = q0[1] - q2[1], cz = q0[2] - q2[2];  // p0 - p2
    const float bcx = by * cz - bz * cy, bcy = bz * cx - bx * cz, bcz = bx * cy - by * cx;
    const float cax = cy * az - cz * ay, cay = cz * ax - cx * az, caz = cx * ay - cy * ax;
    const float abx = ay * bz - az * by, aby = az * bx - ax * bz, abz = ax * by - ay * bx;
    const float det = ax * bcx + ay * bcy + az * bcz;
    if (det == 0.0f) return false;
    const float gt = grad_hits[3 * i], gu = grad_hits[3 * i + 1], gv = grad_hits[3 * i + 2];
    const float inv = 1.0f / det;
    lam[0] = (gt * bcx + gu * cax + gv * abx) * inv;
    lam[1] = (gt * bcy + gu * cay + gv * aby) * inv;
    lam[2] = (gt * bcz + gu * caz + gv * abz) * inv;
    for (int k = 0; k < 3; k++) {
        out[k] = -lam[k];
        out[3 + k] = -t * lam[k];
    }
    w[0] = 1.0f - u - v;
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
