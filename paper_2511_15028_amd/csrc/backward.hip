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
