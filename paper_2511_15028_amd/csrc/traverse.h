// Device-side traversal shared by the per-scene and the batched kernels.
//
// One traversal routine per node family (binary nodes that carry their own
// box; wide nodes that carry their children's boxes), each instantiated with a
// layout decoder, so the search order and culling logic are written once and
// the node format is a type parameter: the decoupling of traversal from
// layout argued in Sec. 3-4 of the paper.
#pragma once

#include <cmath>

#include "internal.h"

namespace bvhlib {


// Traversal kernels run 256 threads (four wave64) per block; the per-lane
// LDS stack columns are indexed by threadIdx.x with this stride.
constexpr int kTraceBlock = 256;

// Slab-test widening: far distances are scaled by 1 + 2^-21, above the
// 1 + 2 gamma_3 bound on the relative rounding error of (plane - o) * (1/d)
// (Ize 2013), so a box that the exact ray enters before the current best
// distance is never culled.
constexpr float kFarScale = 1.000000476837158203125f;

struct Ray {
    float ox, oy, oz;
    float dx, dy, dz;
    float rx, ry, rz;  // 1/d, IEEE (+-inf for +-0)
    float tmax;
    bool nx, ny, nz;   // sign bits of d
};

__device__ inline Ray load_ray(const bvh_ray *rays, uint64_t i) {
    const float4 *p = reinterpret_cast<const float4 *>(rays + i);
    const float4 a = p[0], b = p[1];
    Ray r;
    r.ox = a.x; r.oy = a.y; r.oz = a.z;
    r.dx = b.x; r.dy = b.y; r.dz = b.z;
    r.tmax = b.w;
    r.rx = 1.0f / r.dx;
    r.ry = 1.0f / r.dy;
    r.rz = 1.0f / r.dz;
    r.nx = signbit(r.dx);
    r.ny = signbit(r.dy);
    r.nz = signbit(r.dz);
    return r;
}

// Ray/box test of App. G (intersectsp_ray_aabb) with the node cull folded
// in: the far end is clipped at tcur (the best hit so far, or tmax).
// Returns the entry distance, or +inf when the box is culled.
__device__ inline float slab(const Ray &r, float lox, float loy, float loz, float hix, float hiy,
                             float hiz, float tcur) {
    const float nx = r.nx ? hix : lox, fx = r.nx ? lox : hix;
    const float ny = r.ny ? hiy : loy, fy = r.ny ? loy : hiy;
    const float nz = r.nz ? hiz : loz, fz = r.nz ? loz : hiz;
    const float tnx = (nx - r.ox) * r.rx, tfx = (fx - r.ox) * r.rx;
    const float tny = (ny - r.oy) * r.ry, tfy = (fy - r.oy) * r.ry;
    const float tnz = (nz - r.oz) * r.rz, tfz = (fz - r.oz) * r.rz;
    const float t_near = fmaxf(0.0f, fmaxf(tnx, fmaxf(tny, tnz)));
    const float t_far = fminf(tcur, fminf(tfx, fminf(tfy, tfz)));
    return (t_near <= t_far * kFarScale) ? t_near : INFINITY;
}

// Moller-Trumbore of App. G (intersectsp_ray_tri_mt), operation for
// operation: e1 = p0-p1, e2 = p2-p0, ng = e2 x e1, c = p0-o, r = c x d,
// D = ng.d, U/V/T sign-folded by D, edges inclusive, 0 < t <= tmax,
// t, u, v = (T, U, V) * (1/|D|).  Built without FMA contraction.
__device__ inline bool mt(const Ray &r, float p0x, float p0y, float p0z, float p1x, float p1y,
                          float p1z, float p2x, float p2y, float p2z, float &t, float &u,
                          float &v) {
    const float e1x = p0x - p1x, e1y = p0y - p1y, e1z = p0z - p1z;
    const float e2x = p2x - p0x, e2y = p2y - p0y, e2z = p2z - p0z;
    const float ngx = e2y * e1z - e2z * e1y;
    const float ngy = e2z * e1x - e2x * e1z;
    const float ngz = e2x * e1y - e2y * e1x;
    const float cx = p0x - r.ox, cy = p0y - r.oy, cz = p0z - r.oz;
    const float rrx = cy * r.dz - cz * r.dy;
    const float rry = cz * r.dx - cx * r.dz;
    const float rrz = cx * r.dy - cy * r.dx;
    const float D = (ngx * r.dx + ngy * r.dy) + ngz * r.dz;
    if (D == 0.0f) return false;
    const float absD = fabsf(D);
    const uint32_t sgn = __float_as_uint(D) & 0x80000000u;
    const float U = __uint_as_float(__float_as_uint((rrx * e2x + rry * e2y) + rrz * e2z) ^ sgn);
    const float V = __uint_as_float(__float_as_uint((rrx * e1x + rry * e1y) + rrz * e1z) ^ sgn);
    if (!(U >= 0.0f && V >= 0.0f && U + V <= absD)) return false;
    const float T = __uint_as_float(__float_as_uint((ngx * cx + ngy * cy) + ngz * cz) ^ sgn);
    if (!(absD * 0.0f < T && T <= absD * r.tmax)) return false;
    const float inv = 1.0f / absD;
    t = T * inv;
    u = U * inv;
    v = V * inv;
    return true;
}

struct Best {
    float t, u, v;
    uint32_t id;  // 0xFFFFFFFF = none (compares above every valid id)
};

// (t, id) lexicographic improvement: lower t, then lower primitive id.
__device__ inline void consider(Best &b, float t, float u, float v, uint32_t id) {
    if (t < b.t || (t == b.t && id < b.id)) {
        b.t = t;
        b.u = u;
        b.v = v;
        b.id = id;
    }
}

// Leaf storage: COMPACT reads 48-B triangle records in leaf order; INDEXED
// reads a primitive id, its three vertex indices and three vertices.
struct LeafData {
    const void *leaf;
    const float *verts;
    const int32_t *tris;
    uint32_t n_tris;
};

template <int LeafMode>
__device__ inline void fetch_tri(const LeafData &ld, uint32_t k, float *p, uint32_t &id) {
    if (LeafMode == BVH_LEAF_COMPACT) {
        const float4 *q = static_cast<const float4 *>(ld.leaf) + 3 * (size_t)k;
        const float4 a = q[0], b = q[1], c = q[2];
        p[0] = a.x; p[1] = a.y; p[2] = a.z;
        p[3] = a.w; p[4] = b.x; p[5] = b.y;
        p[6] = b.z; p[7] = b.w; p[8] = c.x;
        id = __float_as_uint(c.y);
    } else {
        id = (uint32_t)static_cast<const int32_t *>(ld.leaf)[k];
        const int32_t *tv = ld.tris + 3 * (size_t)id;
        for (int j = 0; j < 3; j++) {
            const float *vp = ld.verts + 3 * (size_t)tv[j];
            p[3 * j] = vp[0];
            p[3 * j + 1] = vp[1];
            p[3 * j + 2] = vp[2];
        }
    }
}

// Tests triangles [first, first+n) of the leaf order.  Returns true when an
// any-hit query is satisfied.
template <int LeafMode, int Mode>
__device__ inline bool test_leaf(const LeafData &ld, const Ray &r, uint32_t first, uint32_t n,
                                 Best &best, uint32_t &ntri) {
    const uint32_t end = min(first + n, ld.n_tris);  // bounds guard; a valid tree never clips
    for (uint32_t k = first; k < end; k++) {
        float p[9];
        uint32_t id;
        fetch_tri<LeafMode>(ld, k, p, id);
        ntri++;
        float t, u, v;
        if (mt(r, p[0], p[1], p[2], p[3], p[4], p[5], p[6], p[7], p[8], t, u, v)) {
            consider(best, t, u, v, id);
            if (Mode == BVH_TRACE_ANY) return true;
        }
    }
    return false;
}

// ---------------------------------------------------------------------------
// Traversal stacks.  The fast path keeps SL entries per lane in LDS (one
// column per lane, so lanes never share a bank) and has no overflow area: a
// push beyond SL fails, the ray stops and is re-traced by the fallback pass,
// which keeps a deep stack (kStackMax entries, the build's bound) in a
// global-memory workspace.  No private (scratch) memory is used.
// ---------------------------------------------------------------------------
template <bool WithT, int SL>
struct LdsStack {
    uint32_t *lds_ref;  // [SL][kTraceBlock]
    float *lds_t;
    uint32_t sp = 0;
    __device__ LdsStack(uint32_t *r, float *t) : lds_ref(r), lds_t(t) {}
    __device__ bool push(uint32_t ref, float t) {
        if (sp >= (uint32_t)SL) return false;
        const uint32_t slot = sp * kTraceBlock + threadIdx.x;
        lds_ref[slot] = ref;
        if (WithT) lds_t[slot] = t;
        sp++;
        return true;
    }
    __device__ uint32_t pop(float &t) {
        sp--;
        const uint32_t slot = sp * kTraceBlock + threadIdx.x;
        t = WithT ? lds_t[slot] : 0.0f;
        return lds_ref[slot];
    }
};

// Deep stack of one lane in global memory: ref[kStackMax], t[kStackMax].
template <bool WithT>
struct GlobalStack {
    uint32_t *ref;
    float *tt;
    uint32_t sp = 0;
    __device__ GlobalStack(uint32_t *r, float *t) : ref(r), tt(t) {}
    __device__ bool push(uint32_t r, float t) {
        if (sp >= (uint32_t)kStackMax) return false;  // the build bounds the depth by kStackMax
        ref[sp] = r;
        if (WithT) tt[sp] = t;
        sp++;
        return true;
    }
    __device__ uint32_t pop(float &t) {
        sp--;
        t = WithT ? tt[sp] : 0.0f;
        return ref[sp];
    }
};

__device__ inline void store_hit(bvh_hit *hits, uint64_t i, const Best &b) {
    int4 w;
    w.x = (b.id == 0xFFFFFFFFu) ? -1 : (int)b.id;
    w.y = __float_as_int(b.id == 0xFFFFFFFFu ? INFINITY : b.t);
    w.z = __float_as_int(b.id == 0xFFFFFFFFu ? 0.0f : b.u);
    w.w = __float_as_int(b.id == 0xFFFFFFFFu ? 0.0f : b.v);
    reinterpret_cast<int4 *>(hits)[i] = w;
}


// ---------------------------------------------------------------------------
// Binary layout with the box in the node (AABB2): pop a node, test its own
// box against the current best, descend near child first (split axis and
// ray direction sign), push the far child.  s_ref: [SL][kTraceBlock] LDS.
// ---------------------------------------------------------------------------
template <int LeafMode, int Mode, class Stack>
__device__ inline Best trace_aabb2(const bvh_node_aabb2 *nodes, int64_t n_nodes, const LeafData &ld,
                                   const Ray &r, Stack &st, uint32_t &nfetch, uint32_t &ntri,
                                   bool &incomplete) {
    Best best{INFINITY, 0.0f, 0.0f, 0xFFFFFFFFu};
    uint32_t node = 0;
    bool active = n_nodes > 0;
    while (active) {
        if (node >= (uint64_t)n_nodes) break;  // bounds guard; a valid tree never takes it
        const float4 *np = reinterpret_cast<const float4 *>(nodes + node);
        const float4 a = np[0], b = np[1];
        nfetch++;
        const float tcur = (Mode == BVH_TRACE_ANY) ? r.tmax : fminf(best.t, r.tmax);
        const float tn = slab(r, a.x, a.y, a.z, a.w, b.x, b.y, tcur);
        if (tn != INFINITY) {
            const uint32_t off = __float_as_uint(b.z), meta = __float_as_uint(b.w);
            const uint32_t np_ = meta & 0xFFFFu;
            if (np_ > 0) {
                if (test_leaf<LeafMode, Mode>(ld, r, off, np_, best, ntri)) break;
            } else {
                const uint32_t axis = (meta >> 16) & 3u;
                const bool neg = axis == 0 ? r.nx : (axis == 1 ? r.ny : r.nz);
                const uint32_t left = node + 1, right = node + off;
                if (!st.push(neg ? left : right, 0.0f)) {
                    incomplete = true;
                    break;
                }
                node = neg ? right : left;
                continue;
            }
        }
        if (st.sp == 0) break;
        float unused;
        node = st.pop(unused);
    }
    return best;
}

// ---------------------------------------------------------------------------
// Wide layouts: the node holds its children's boxes.  Decoders expose
//   K                      arity
//   test(node ptr, ray, tcur, tn[K], ref[K])
// writing the entry distance of every child the ray meets (+inf otherwise).
// ---------------------------------------------------------------------------
struct DecodeBVH4 {
    static constexpr int K = 4;
    __device__ static void test(const void *base, uint32_t node, const Ray &r, float tcur,
                                float *tn, uint32_t *ref) {
        const float4 *p = static_cast<const float4 *>(base) + 8 * (size_t)node;
        const float4 lx = p[0], ly = p[1], lz = p[2], hx = p[3], hy = p[4], hz = p[5];
        const uint4 ch = reinterpret_cast<const uint4 *>(p)[6];
        const float lxs[4] = {lx.x, lx.y, lx.z, lx.w}, lys[4] = {ly.x, ly.y, ly.z, ly.w};
        const float lzs[4] = {lz.x, lz.y, lz.z, lz.w}, hxs[4] = {hx.x, hx.y, hx.z, hx.w};
        const float hys[4] = {hy.x, hy.y, hy.z, hy.w}, hzs[4] = {hz.x, hz.y, hz.z, hz.w};
        const uint32_t chs[4] = {ch.x, ch.y, ch.z, ch.w};
#pragma unroll
        for (int c = 0; c < 4; c++) {
            tn[c] = slab(r, lxs[c], lys[c], lzs[c], hxs[c], hys[c], hzs[c], tcur);
            ref[c] = chs[c];
        }
    }
};

// Byte c of the 8 packed bytes held in words (w0, w1).
__device__ inline uint32_t byte_of(uint32_t w0, uint32_t w1, int c) {
    return ((c < 4 ? w0 : w1) >> (8 * (c & 3))) & 0xFFu;
}
__device__ inline uint32_t half_of(const uint32_t *w, int c) {
    return (w[c >> 1] >> (16 * (c & 1))) & 0xFFFFu;
}

struct DecodeBVH8Q8 {
    static constexpr int K = 8;
    __device__ static void test(const void *base, uint32_t node, const Ray &r, float tcur,
                                float *tn, uint32_t *ref) {
        const uint4 *p = static_cast<const uint4 *>(base) + 8 * (size_t)node;
        uint32_t w[28];
#pragma unroll
        for (int k = 0; k < 7; k++) {
            const uint4 q = p[k];
            w[4 * k] = q.x; w[4 * k + 1] = q.y; w[4 * k + 2] = q.z; w[4 * k + 3] = q.w;
        }
        const float ox = __uint_as_float(w[0]), oy = __uint_as_float(w[1]), oz = __uint_as_float(w[2]);
        const float sx = __uint_as_float(w[3]), sy = __uint_as_float(w[4]), sz = __uint_as_float(w[5]);
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const float lox = fmaf((float)byte_of(w[6], w[7], c), sx, ox);
            const float loy = fmaf((float)byte_of(w[8], w[9], c), sy, oy);
            const float loz = fmaf((float)byte_of(w[10], w[11], c), sz, oz);
            const float hix = fmaf((float)byte_of(w[12], w[13], c), sx, ox);
            const float hiy = fmaf((float)byte_of(w[14], w[15], c), sy, oy);
            const float hiz = fmaf((float)byte_of(w[16], w[17], c), sz, oz);
            const bool valid = (uint32_t)c < w[26];
            tn[c] = valid ? slab(r, lox, loy, loz, hix, hiy, hiz, tcur) : INFINITY;
            ref[c] = w[18 + c];
        }
    }
};

struct DecodeBVH8Q16 {
    static constexpr int K = 8;
    __device__ static void test(const void *base, uint32_t node, const Ray &r, float tcur,
                                float *tn, uint32_t *ref) {
        const uint4 *p = static_cast<const uint4 *>(base) + 10 * (size_t)node;
        uint32_t w[40];
#pragma unroll
        for (int k = 0; k < 10; k++) {
            const uint4 q = p[k];
            w[4 * k] = q.x; w[4 * k + 1] = q.y; w[4 * k + 2] = q.z; w[4 * k + 3] = q.w;
        }
        const float ox = __uint_as_float(w[0]), oy = __uint_as_float(w[1]), oz = __uint_as_float(w[2]);
        const float sx = __uint_as_float(w[3]), sy = __uint_as_float(w[4]), sz = __uint_as_float(w[5]);
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const float lox = fmaf((float)half_of(w + 6, c), sx, ox);
            const float loy = fmaf((float)half_of(w + 10, c), sy, oy);
            const float loz = fmaf((float)half_of(w + 14, c), sz, oz);
            const float hix = fmaf((float)half_of(w + 18, c), sx, ox);
            const float hiy = fmaf((float)half_of(w + 22, c), sy, oy);
            const float hiz = fmaf((float)half_of(w + 26, c), sz, oz);
            const bool valid = (uint32_t)c < w[38];
            tn[c] = valid ? slab(r, lox, loy, loz, hix, hiy, hiz, tcur) : INFINITY;
            ref[c] = w[30 + c];
        }
    }
};

__device__ inline void cswap(float *t, uint32_t *r, int a, int b) {
    const bool sw = t[b] < t[a];
    const float ta = t[a], tb = t[b];
    const uint32_t ra = r[a], rb = r[b];
    t[a] = sw ? tb : ta;
    t[b] = sw ? ta : tb;
    r[a] = sw ? rb : ra;
    r[b] = sw ? ra : rb;
}

// Ascending sort by entry distance (sorting networks: 5 and 19 exchanges).
template <int K>
__device__ inline void sort_children(float *t, uint32_t *r) {
    if (K == 4) {
        cswap(t, r, 0, 1); cswap(t, r, 2, 3);
        cswap(t, r, 0, 2); cswap(t, r, 1, 3);
        cswap(t, r, 1, 2);
    } else {
        cswap(t, r, 0, 2); cswap(t, r, 1, 3); cswap(t, r, 4, 6); cswap(t, r, 5, 7);
        cswap(t, r, 0, 4); cswap(t, r, 1, 5); cswap(t, r, 2, 6); cswap(t, r, 3, 7);
        cswap(t, r, 0, 1); cswap(t, r, 2, 3); cswap(t, r, 4, 5); cswap(t, r, 6, 7);
        cswap(t, r, 2, 4); cswap(t, r, 3, 5);
        cswap(t, r, 1, 4); cswap(t, r, 3, 6);
        cswap(t, r, 1, 2); cswap(t, r, 3, 4); cswap(t, r, 5, 6);
    }
}


// Wide-node traversal: test all children of the current node, sort the hit
// ones near-first, continue with the nearest and push the rest with their
// entry distances; popped entries are re-culled against the current best.
// s_ref, s_t: [SL][kTraceBlock] LDS.
template <class Dec, int LeafMode, int Mode, class Stack>
__device__ inline Best trace_wide(const void *nodes, int64_t n_nodes, const LeafData &ld,
                                  const Ray &r, Stack &st, uint32_t &nfetch, uint32_t &ntri,
                                  bool &incomplete) {
    constexpr int K = Dec::K;
    Best best{INFINITY, 0.0f, 0.0f, 0xFFFFFFFFu};
    uint32_t cur = n_nodes > 0 ? ref_interior(0) : kRefEmpty;
    while (cur != kRefEmpty) {
        const float tcur = (Mode == BVH_TRACE_ANY) ? r.tmax : fminf(best.t, r.tmax);
        if (cur & 1u) {
            if ((cur >> 1) >= (uint64_t)n_nodes) break;  // bounds guard; never taken on a valid tree
            float tn[K];
            uint32_t ref[K];
            Dec::test(nodes, cur >> 1, r, tcur, tn, ref);
            nfetch++;
            sort_children<K>(tn, ref);
            bool ok = true;
#pragma unroll
            for (int c = K - 1; c >= 1; c--)
                if (tn[c] != INFINITY) ok = st.push(ref[c], tn[c]) && ok;
            if (!ok) {
                incomplete = true;
                break;
            }
            if (tn[0] != INFINITY) {
                cur = ref[0];
                continue;
            }
        } else {
            const uint32_t first = cur >> 5, cnt = ((cur >> 1) & 0xFu) + 1u;
            if (test_leaf<LeafMode, Mode>(ld, r, first, cnt, best, ntri)) break;
        }
        // pop the next entry that the current best has not culled
        cur = kRefEmpty;
        const float tb = (Mode == BVH_TRACE_ANY) ? r.tmax : fminf(best.t, r.tmax);
        while (st.sp > 0) {
            float t;
            const uint32_t ref = st.pop(t);
            if (t <= tb * kFarScale) {
                cur = ref;
                break;
            }
        }
    }
    return best;
}

// Work area of the fallback pass: a counter and list of rays that
// overflowed the LDS stack, and one deep stack per fallback lane.
constexpr int kFallbackBlocks = 128;
constexpr int kFallbackLanes = kFallbackBlocks * kTraceBlock;
struct Fallback {
    uint32_t *count;     // rays appended by the fast pass
    uint32_t *list;      // ray indices (capacity: rays of the launch)
    uint32_t *stack_ref; // [kFallbackLanes][kStackMax]
    float *stack_t;      // [kFallbackLanes][kStackMax]
};

inline size_t fallback_bytes(uint64_t n_rays) {
    return 256 + n_rays * 4 + (size_t)kFallbackLanes * kStackMax * 8;
}

// Carves the work area out of one allocation of fallback_bytes(n_rays).
inline Fallback fallback_view(void *base, uint64_t n_rays) {
    char *p = static_cast<char *>(base);
    Fallback f;
    f.count = reinterpret_cast<uint32_t *>(p);
    f.list = reinterpret_cast<uint32_t *>(p + 256);
    f.stack_ref = reinterpret_cast<uint32_t *>(p + 256 + n_rays * 4);
    f.stack_t = reinterpret_cast<float *>(p + 256 + n_rays * 4 + (size_t)kFallbackLanes * kStackMax * 4);
    return f;
}

__device__ inline void fallback_append(const Fallback &fb, uint32_t ray) {
    const uint32_t k = atomicAdd(fb.count, 1u);
    fb.list[k] = ray;
}

}  // namespace bvhlib
