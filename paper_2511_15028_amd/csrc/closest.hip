// Closest-point query (App. G "Closest Point Query"; evaluated on the same
// layouts as ray traversal in Sec. 9.2.3 and 9.3.2) and the
// bvh_closest_point / bvh_closest_point_counts entry points.
//
// Per query: the triangle at the smallest squared distance d2 <= r2 from the
// point, ties to the lowest primitive id.  Children are visited nearest box
// first (the listing's distance-based child sorting); a node or stacked entry
// whose box lies farther than the best distance so far is skipped.  The
// point-triangle distance is Ericson's Voronoi-region method (Real-Time
// Collision Detection 5.1.5), the one the paper's listing uses.
//
// Scheduling follows the persistent ray kernel: a grid of resident blocks,
// lanes refilled from their wave's pool of claimed queries, per-lane stacks
// in an LDS ring over a global spill area, and a fallback pass with a deep
// stack for the few queries that outgrow both.
#include <algorithm>

#include "traverse.h"

namespace bvhlib {
namespace {

// Box distances are scaled by 1 - 2^-21 before the cull: the rounding of the
// three gaps, their squares and the two sums (at most five roundings, each
// within 2^-24 relative) cannot lift the computed value above the exact
// squared distance divided by that factor, so a box that holds a triangle
// at least as near as the best one is never skipped.
constexpr float kNearScale = 0.999999523162841796875f;  // 1 - 2^-21

struct CpqBest {
    float d2, u, v;
    uint32_t id;
};

// (d2, id) lexicographic improvement; the initial best is (r2, none), so a
// triangle at exactly d2 == r2 is accepted.
__device__ inline void cp_consider(CpqBest &b, float d2, float u, float v, uint32_t id) {
    if (d2 < b.d2 || (d2 == b.d2 && id < b.id)) {
        b.d2 = d2;
        b.u = u;
        b.v = v;
        b.id = id;
    }
}

// A query: the point and squared radius; `live` is false for a point with a
// non-finite coordinate (such a query returns no triangle).
struct Query {
    float x, y, z, r2;
    bool live;
};

__device__ inline Query load_query(const bvh_point_query *qs, uint64_t i) {
    const float4 w = reinterpret_cast<const float4 *>(qs)[i];
    Query q{w.x, w.y, w.z, w.w, false};
    q.live = isfinite(w.x) && isfinite(w.y) && isfinite(w.z) && w.w >= 0.0f;
    return q;
}

__device__ inline float box_d2(const Query &q, float lox, float loy, float loz, float hix,
                               float hiy, float hiz) {
    const float gx = fmaxf(fmaxf(lox - q.x, q.x - hix), 0.0f);
    const float gy = fmaxf(fmaxf(loy - q.y, q.y - hiy), 0.0f);
    const float gz = fmaxf(fmaxf(loz - q.z, q.z - hiz), 0.0f);
    return fmaf(gx, gx, fmaf(gy, gy, gz * gz)) * kNearScale;
}

__device__ inline float dot3(float ax, float ay, float az, float bx, float by, float bz) {
    return (ax * bx + ay * by) + az * bz;
}

// Nearest point of the segment a + s (b - a), s in [0, 1], to p (offset
// vectors relative to a): returns s.
__device__ inline float seg_s(float px, float py, float pz, float dx, float dy, float dz) {
    const float len2 = dot3(dx, dy, dz, dx, dy, dz);
    const float s = len2 > 0.0f ? dot3(px, py, pz, dx, dy, dz) / len2 : 0.0f;
    return fminf(fmaxf(s, 0.0f), 1.0f);
}

// Squared distance of the point a + u ab + v ac from p, given ap = p - a.
__device__ inline float cp_dist2(float apx, float apy, float apz, float abx, float aby, float abz,
                                 float acx, float acy, float acz, float u, float v) {
    const float x = fmaf(-acx, v, fmaf(-abx, u, apx));
    const float y = fmaf(-acy, v, fmaf(-aby, u, apy));
    const float z = fmaf(-acz, v, fmaf(-abz, u, apz));
    return dot3(x, y, z, x, y, z);
}

// Ericson's closest point on triangle (a, b, c) to p, from ap = p - a and the
// edges ab = b - a, ac = c - a.  The Voronoi regions are tested in the
// listing's order (vertex a, vertex b, edge ab, vertex c, edge ac, edge bc,
// face); the first that holds decides, and all are evaluated without
// branches so the lanes of a wave stay together.  Returns d2 and the
// barycentrics (u of b, v of c).  A degenerate triangle (no positive face
// denominator) or a face result outside the triangle takes the nearest of the
// three edge projections instead.
__device__ inline float cp_tri(float apx, float apy, float apz, float abx, float aby, float abz,
                               float acx, float acy, float acz, float &u, float &v) {
    const float d1 = dot3(abx, aby, abz, apx, apy, apz);
    const float d2 = dot3(acx, acy, acz, apx, apy, apz);
    const float bpx = apx - abx, bpy = apy - aby, bpz = apz - abz;  // p - b
    const float d3 = dot3(abx, aby, abz, bpx, bpy, bpz);
    const float d4 = dot3(acx, acy, acz, bpx, bpy, bpz);
    const float cpx = apx - acx, cpy = apy - acy, cpz = apz - acz;  // p - c
    const float d5 = dot3(abx, aby, abz, cpx, cpy, cpz);
    const float d6 = dot3(acx, acy, acz, cpx, cpy, cpz);
    const float vc = d1 * d4 - d3 * d2;
    const float vb = d5 * d2 - d1 * d6;
    const float va = d3 * d6 - d5 * d4;
    const bool in_a = d1 <= 0.0f && d2 <= 0.0f;
    const bool in_b = d3 >= 0.0f && d4 <= d3;
    const bool in_ab = vc <= 0.0f && d1 >= 0.0f && d3 <= 0.0f;
    const bool in_c = d6 >= 0.0f && d5 <= d6;
    const bool in_ac = vb <= 0.0f && d2 >= 0.0f && d6 <= 0.0f;
    const bool in_bc = va <= 0.0f && (d4 - d3) >= 0.0f && (d5 - d6) >= 0.0f;
    // the one division of the chosen region, s = num / den, as num times the
    // hardware reciprocal of den (within one ulp)
    float num = 1.0f, den = va + vb + vc;  // face: 1 / (va + vb + vc)
    if (in_bc) { num = d4 - d3; den = (d4 - d3) + (d5 - d6); }
    if (in_ac) { num = d2; den = d2 - d6; }
    if (in_ab) { num = d1; den = d1 - d3; }
    const float s = num * __builtin_amdgcn_rcpf(den);
    float uu = vb * s, vv = vc * s;  // face
    if (in_bc) { uu = 1.0f - s; vv = s; }
    if (in_ac) { uu = 0.0f; vv = s; }
    if (in_c) { uu = 0.0f; vv = 1.0f; }
    if (in_ab) { uu = s; vv = 0.0f; }
    if (in_b) { uu = 1.0f; vv = 0.0f; }
    if (in_a) { uu = 0.0f; vv = 0.0f; }
    const bool face = !(in_a || in_b || in_ab || in_c || in_ac || in_bc);
    if (face && !(den > 0.0f && uu >= -1e-3f && vv >= -1e-3f && uu + vv <= 1.001f)) {
        // degenerate or ill-conditioned: the nearest point of the boundary
        const float s01 = seg_s(apx, apy, apz, abx, aby, abz);
        const float s02 = seg_s(apx, apy, apz, acx, acy, acz);
        const float s12 = seg_s(bpx, bpy, bpz, acx - abx, acy - aby, acz - abz);
        float best = cp_dist2(apx, apy, apz, abx, aby, abz, acx, acy, acz, s01, 0.0f);
        uu = s01;
        vv = 0.0f;
        const float e02 = cp_dist2(apx, apy, apz, abx, aby, abz, acx, acy, acz, 0.0f, s02);
        if (e02 < best) { best = e02; uu = 0.0f; vv = s02; }
        const float e12 = cp_dist2(apx, apy, apz, abx, aby, abz, acx, acy, acz, 1.0f - s12, s12);
        if (e12 < best) { best = e12; uu = 1.0f - s12; vv = s12; }
        u = uu;
        v = vv;
        return best;
    }
    u = uu;
    v = vv;
    return cp_dist2(apx, apy, apz, abx, aby, abz, acx, acy, acz, uu, vv);
}

// Triangles [first, first + n) of the leaf order.  Compacted records give
// p0 and e1 = p1 - p0, e2 = p2 - p0, which are ab and ac exactly as the
// indexed path computes them from the vertices (both leaf modes give
// bit-identical distances).
template <int LeafMode>
__device__ inline void cp_leaf(const SceneData &ld, const Query &q, uint32_t first, uint32_t n,
                               CpqBest &best, uint32_t &ntri) {
    const uint32_t end = min(first + n, ld.n_tris);  // bounds guard; a valid tree never clips
    if (LeafMode == BVH_LEAF_COMPACT) {
        const float4 *base = static_cast<const float4 *>(ld.leaf);
        for (uint32_t k0 = first; k0 < end; k0 += kLeafBatch) {
            float4 qa[kLeafBatch], qb[kLeafBatch];
            float2 qc[kLeafBatch];
#pragma unroll
            for (uint32_t j = 0; j < kLeafBatch; j++) {
                if (k0 + j < end) {
                    const float4 *p = base + 3 * (size_t)(k0 + j);
                    qa[j] = p[0];
                    qb[j] = p[1];
                    qc[j] = *reinterpret_cast<const float2 *>(p + 2);
                }
            }
#pragma unroll
            for (uint32_t j = 0; j < kLeafBatch; j++) {
                if (k0 + j < end) {
                    ntri++;
                    const float4 a = qa[j], b = qb[j];
                    const float2 c = qc[j];
                    float u, v;
                    const float d2 = cp_tri(q.x - a.x, q.y - a.y, q.z - a.z, a.w, b.x, b.y, b.z,
                                            b.w, c.x, u, v);
                    cp_consider(best, d2, u, v, __float_as_uint(c.y));
                }
            }
        }
        return;
    }
    for (uint32_t k = first; k < end; k++) {
        const uint32_t id = (uint32_t) static_cast<const int32_t *>(ld.leaf)[k];
        const int32_t *tv = ld.tris + 3 * (size_t)id;
        const float *a = ld.verts + 3 * (size_t)tv[0];
        const float *b = ld.verts + 3 * (size_t)tv[1];
        const float *c = ld.verts + 3 * (size_t)tv[2];
        ntri++;
        float u, v;
        const float d2 = cp_tri(q.x - a[0], q.y - a[1], q.z - a[2], b[0] - a[0], b[1] - a[1],
                                b[2] - a[2], c[0] - a[0], c[1] - a[1], c[2] - a[2], u, v);
        cp_consider(best, d2, u, v, id);
    }
}

// ---------------------------------------------------------------------------
// Binary layouts (each node holds its own box): visiting an interior node
// loads both children, measures their boxes, continues with the nearer and
// stacks the farther (with its distance, so a later pop can skip it).
// ---------------------------------------------------------------------------
// Wave-level leaf batching for the closest-point query (the counterpart of
// wave_test_leaves for rays): the lanes that reach a leaf publish its
// triangles, and the wave tests the (query, triangle) pairs one per lane.
// The best of a leaf is the lexicographic minimum of (squared distance, id),
// taken per owner with an LDS 64-bit minimum of (distance bits << 32 | id)
// (squared distances are never negative, so the bits order like the values,
// and a NaN never beats a number); the lane holding the winning pair then
// stores its (u, v).  Each pair's arithmetic is cp_leaf's, so the results are
// the same bits as testing the leaf in one lane.  Called by every lane of
// the wave (converged).
template <int LeafMode>
__device__ inline void wave_cp_leaves(const SceneData &ld, const Query &q, bool want, uint32_t first,
                                      uint32_t cnt, CpqBest &best, uint32_t &ntri,
                                      WaveLeafLds *wl) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t c = want ? cnt : 0u;
    uint32_t pre = 0, total = 0;
#pragma unroll
    for (int b = 0; b < 5; b++) {  // leaf sizes are below 32
        const uint64_t m = __builtin_amdgcn_ballot_w64(((c >> b) & 1u) != 0u);
        pre += count_below(m) << b;
        total += (uint32_t)__builtin_popcountll(m) << b;
    }
    if (total == 0) return;
    ntri += c;
    for (uint32_t base = 0; base < total; base += 64u) {
        if (want) {
            const uint32_t lo = pre > base ? pre : base;
            const uint32_t hi = min(pre + c, base + 64u);
            for (uint32_t k = lo; k < hi; k++) wl->owner[k - base] = lane;
        }
        wl->key[lane] = ~0ull;
        wave_lds_sync();
        const uint32_t pair = base + lane;
        const bool act = pair < total;
        const uint32_t o = act ? wl->owner[lane] : lane;
        const float qx = lane_f(q.x, o), qy = lane_f(q.y, o), qz = lane_f(q.z, o);
        const uint32_t k = lane_u(first, o) + (pair - lane_u(pre, o));
        bool got = false;
        float d2 = 0.0f, u = 0.0f, v = 0.0f;
        uint32_t id = 0;
        if (act && k < ld.n_tris) {  // bounds guard; a valid tree never fails it
            got = true;
            if (LeafMode == BVH_LEAF_COMPACT) {
                const float4 *p = static_cast<const float4 *>(ld.leaf) + 3 * (size_t)k;
                const float4 a = p[0], b = p[1];
                const float2 cc = *reinterpret_cast<const float2 *>(p + 2);
                d2 = cp_tri(qx - a.x, qy - a.y, qz - a.z, a.w, b.x, b.y, b.z, b.w, cc.x, u, v);
                id = __float_as_uint(cc.y);
            } else {
                id = (uint32_t) static_cast<const int32_t *>(ld.leaf)[k];
                const int32_t *tv = ld.tris + 3 * (size_t)id;
                const float *a = ld.verts + 3 * (size_t)tv[0];
                const float *b = ld.verts + 3 * (size_t)tv[1];
                const float *cv = ld.verts + 3 * (size_t)tv[2];
                d2 = cp_tri(qx - a[0], qy - a[1], qz - a[2], b[0] - a[0], b[1] - a[1], b[2] - a[2],
                            cv[0] - a[0], cv[1] - a[1], cv[2] - a[2], u, v);
            }
        }
        const unsigned long long mine = ((unsigned long long)__float_as_uint(d2) << 32) | id;
        if (got) atomicMin(&wl->key[o], mine);
        wave_lds_sync();
        if (got && wl->key[o] == mine) wl->uv[o] = make_float2(u, v);
        wave_lds_sync();
        if (want) {
            const unsigned long long kb = wl->key[lane];
            if (kb != ~0ull) {
                const float2 w = wl->uv[lane];
                cp_consider(best, __uint_as_float((uint32_t)(kb >> 32)), w.x, w.y, (uint32_t)kb);
            }
        }
        wave_lds_sync();
    }
}

template <class Node>
struct CpqBin {
    struct State {
        CpqBest best;
        uint32_t cur;       // node to visit next (kRefEmpty: pop one)
        uint32_t cnt, off;  // its triangle count and offset (right-child delta or first triangle)
    };
    __device__ static State start(const void *nodes, int64_t n_nodes, const SceneData &ld,
                                  const Query &q, uint32_t &nfetch) {
        State s;
        s.best = CpqBest{q.r2, 0.0f, 0.0f, 0xFFFFFFFFu};
        s.cur = kRefEmpty;
        s.cnt = s.off = 0;
        if (q.live && n_nodes > 0) {
            float lo[3], hi[3];
            uint32_t cnt, off, axis;
            Node::load(nodes, 0, ld, lo, hi, cnt, off, axis);
            nfetch++;
            if (box_d2(q, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]) <= s.best.d2) {
                s.cur = 0;
                s.cnt = cnt;
                s.off = off;
            }
        }
        return s;
    }
    template <class Stack>
    __device__ static bool done(const State &s, const Stack &st) {
        return s.cur == kRefEmpty && st.sp == 0;
    }
    template <int LeafMode, class Stack>
    __device__ static void step(const void *nodes, const SceneData &ld, const Query &q, Stack &st,
                                State &s, uint32_t &nfetch, uint32_t &ntri, bool &incomplete) {
        if (s.cur == kRefEmpty) {
            while (st.sp > 0) {
                float d;
                const uint32_t i = st.pop(d);
                if (d <= s.best.d2) {
                    float lo[3], hi[3];
                    uint32_t axis;
                    Node::load(nodes, i, ld, lo, hi, s.cnt, s.off, axis);
                    nfetch++;
                    s.cur = i;
                    break;
                }
            }
            if (s.cur == kRefEmpty) return;
        }
        if (s.cnt > 0) {
            cp_leaf<LeafMode>(ld, q, s.off, s.cnt, s.best, ntri);
            s.cur = kRefEmpty;
            return;
        }
        const uint32_t li = s.cur + 1u, ri = s.cur + s.off;
        float llo[3], lhi[3], rlo[3], rhi[3];
        uint32_t lcnt, loff, rcnt, roff, axis;
        Node::load(nodes, li, ld, llo, lhi, lcnt, loff, axis);
        Node::load(nodes, ri, ld, rlo, rhi, rcnt, roff, axis);
        nfetch += 2;
        const float dl = box_d2(q, llo[0], llo[1], llo[2], lhi[0], lhi[1], lhi[2]);
        const float dr = box_d2(q, rlo[0], rlo[1], rlo[2], rhi[0], rhi[1], rhi[2]);
        const bool okl = dl <= s.best.d2, okr = dr <= s.best.d2;
        if (okl && okr) {
            const bool left_first = dl <= dr;
            if (!st.push(left_first ? ri : li, left_first ? dr : dl)) {
                incomplete = true;
                s.cur = kRefEmpty;
                return;
            }
            s.cur = left_first ? li : ri;
            s.cnt = left_first ? lcnt : rcnt;
            s.off = left_first ? loff : roff;
        } else if (okl || okr) {
            s.cur = okl ? li : ri;
            s.cnt = okl ? lcnt : rcnt;
            s.off = okl ? loff : roff;
        } else {
            s.cur = kRefEmpty;
        }
    }
    // The same step for the whole wave (every lane calls it; `act` lanes have
    // a query in progress): interior nodes per lane as in step, then the
    // leaves the lanes reached tested together (wave_cp_leaves).
    template <int LeafMode, class Stack>
    __device__ static void wave_step(const void *nodes, const SceneData &ld, const Query &q,
                                     Stack &st, State &s, uint32_t &nfetch, uint32_t &ntri,
                                     bool &incomplete, bool act, WaveLeafLds *wl) {
        bool want = false;
        uint32_t first = 0, cnt = 0;
        if (act) {
            if (s.cur == kRefEmpty) {
                while (st.sp > 0) {
                    float d;
                    const uint32_t i = st.pop(d);
                    if (d <= s.best.d2) {
                        float lo[3], hi[3];
                        uint32_t axis;
                        Node::load(nodes, i, ld, lo, hi, s.cnt, s.off, axis);
                        nfetch++;
                        s.cur = i;
                        break;
                    }
                }
            }
            if (s.cur != kRefEmpty) {
                if (s.cnt > 0) {  // a leaf: its triangles [off, off + cnt)
                    want = true;
                    first = s.off;
                    cnt = s.cnt;
                    s.cur = kRefEmpty;
                } else {
                    step<LeafMode>(nodes, ld, q, st, s, nfetch, ntri, incomplete);
                }
            }
        }
        wave_cp_leaves<LeafMode>(ld, q, want, first, cnt, s.best, ntri, wl);
    }
};

// ---------------------------------------------------------------------------
// Wide layouts (each node holds its children's boxes): the children's
// distances are measured, sorted ascending, the nearest is visited next and
// the others are stacked farthest first.
// ---------------------------------------------------------------------------
template <int Layout>
struct WideChildren;

template <>
struct WideChildren<BVH_LAYOUT_BVH4> {
    static constexpr int K = 4;
    __device__ static void measure(const void *base, uint32_t node, const Query &q, float *d,
                                   uint32_t *ref) {
        const float4 *p = static_cast<const float4 *>(base) + 8 * (size_t)node;
        const float4 lx = p[0], ly = p[1], lz = p[2], hx = p[3], hy = p[4], hz = p[5];
        const uint4 ch = *reinterpret_cast<const uint4 *>(p + 6);
        const uint32_t nc = *reinterpret_cast<const uint32_t *>(p + 7);
        d[0] = box_d2(q, lx.x, ly.x, lz.x, hx.x, hy.x, hz.x);
        d[1] = box_d2(q, lx.y, ly.y, lz.y, hx.y, hy.y, hz.y);
        d[2] = box_d2(q, lx.z, ly.z, lz.z, hx.z, hy.z, hz.z);
        d[3] = box_d2(q, lx.w, ly.w, lz.w, hx.w, hy.w, hz.w);
        ref[0] = ch.x;
        ref[1] = nc > 1 ? ch.y : kRefEmpty;
        ref[2] = nc > 2 ? ch.z : kRefEmpty;
        ref[3] = nc > 3 ? ch.w : kRefEmpty;
    }
};

template <>
struct WideChildren<BVH_LAYOUT_BVH8_Q8> {
    static constexpr int K = 8;
    __device__ static void measure(const void *base, uint32_t node, const Query &q, float *d,
                                   uint32_t *ref) {
        const uint4 *p = static_cast<const uint4 *>(base) + 8 * (size_t)node;
        uint32_t w[28];
#pragma unroll
        for (int k = 0; k < 7; k++) {
            const uint4 x = p[k];
            w[4 * k] = x.x; w[4 * k + 1] = x.y; w[4 * k + 2] = x.z; w[4 * k + 3] = x.w;
        }
        const float ox = __uint_as_float(w[0]), oy = __uint_as_float(w[1]), oz = __uint_as_float(w[2]);
        const float sx = __uint_as_float(w[3]), sy = __uint_as_float(w[4]), sz = __uint_as_float(w[5]);
        // words: lo_x 6-7, lo_y 8-9, lo_z 10-11, hi_x 12-13, hi_y 14-15, hi_z 16-17
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const float lx = fmaf((float)byte_of(w[6], w[7], c), sx, ox);
            const float ly = fmaf((float)byte_of(w[8], w[9], c), sy, oy);
            const float lz = fmaf((float)byte_of(w[10], w[11], c), sz, oz);
            const float hx = fmaf((float)byte_of(w[12], w[13], c), sx, ox);
            const float hy = fmaf((float)byte_of(w[14], w[15], c), sy, oy);
            const float hz = fmaf((float)byte_of(w[16], w[17], c), sz, oz);
            d[c] = box_d2(q, lx, ly, lz, hx, hy, hz);
            ref[c] = (uint32_t)c < w[26] ? w[18 + c] : kRefEmpty;
        }
    }
};

template <>
struct WideChildren<BVH_LAYOUT_BVH8_Q16> {
    static constexpr int K = 8;
    __device__ static void measure(const void *base, uint32_t node, const Query &q, float *d,
                                   uint32_t *ref) {
        const uint4 *p = static_cast<const uint4 *>(base) + 10 * (size_t)node;
        uint32_t w[40];
#pragma unroll
        for (int k = 0; k < 10; k++) {
            const uint4 x = p[k];
            w[4 * k] = x.x; w[4 * k + 1] = x.y; w[4 * k + 2] = x.z; w[4 * k + 3] = x.w;
        }
        const float ox = __uint_as_float(w[0]), oy = __uint_as_float(w[1]), oz = __uint_as_float(w[2]);
        const float sx = __uint_as_float(w[3]), sy = __uint_as_float(w[4]), sz = __uint_as_float(w[5]);
        // words: lo_x 6-9, lo_y 10-13, lo_z 14-17, hi_x 18-21, hi_y 22-25, hi_z 26-29
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const float lx = fmaf((float)half_of(w + 6, c), sx, ox);
            const float ly = fmaf((float)half_of(w + 10, c), sy, oy);
            const float lz = fmaf((float)half_of(w + 14, c), sz, oz);
            const float hx = fmaf((float)half_of(w + 18, c), sx, ox);
            const float hy = fmaf((float)half_of(w + 22, c), sy, oy);
            const float hz = fmaf((float)half_of(w + 26, c), sz, oz);
            d[c] = box_d2(q, lx, ly, lz, hx, hy, hz);
            ref[c] = (uint32_t)c < w[38] ? w[30 + c] : kRefEmpty;
        }
    }
};

template <int Layout>
struct CpqWide {
    using Ch = WideChildren<Layout>;
    static constexpr int K = Ch::K;
    struct State {
        CpqBest best;
        uint32_t cur;  // tagged child reference to visit next (kRefEmpty: pop one)
    };
    __device__ static State start(const void *, int64_t n_nodes, const SceneData &, const Query &q,
                                  uint32_t &) {
        State s;
        s.best = CpqBest{q.r2, 0.0f, 0.0f, 0xFFFFFFFFu};
        s.cur = (q.live && n_nodes > 0) ? ref_interior(0) : kRefEmpty;
        return s;
    }
    template <class Stack>
    __device__ static bool done(const State &s, const Stack &st) {
        return s.cur == kRefEmpty && st.sp == 0;
    }
    template <int LeafMode, class Stack>
    __device__ static void step(const void *nodes, const SceneData &ld, const Query &q, Stack &st,
                                State &s, uint32_t &nfetch, uint32_t &ntri, bool &incomplete) {
        if (s.cur == kRefEmpty) {
            while (st.sp > 0) {
                float d;
                const uint32_t r = st.pop(d);
                if (d <= s.best.d2) {
                    s.cur = r;
                    break;
                }
            }
            if (s.cur == kRefEmpty) return;
        }
        if ((s.cur & 1u) == 0u) {  // a leaf: first triangle and count in the reference
            cp_leaf<LeafMode>(ld, q, s.cur >> 5, ((s.cur >> 1) & 0xFu) + 1u, s.best, ntri);
            s.cur = kRefEmpty;
            return;
        }
        float d[K];
        uint32_t ref[K];
        Ch::measure(nodes, s.cur >> 1, q, d, ref);
        nfetch++;
#pragma unroll
        for (int c = 0; c < K; c++) {
            const bool keep = ref[c] != kRefEmpty && d[c] <= s.best.d2;
            d[c] = keep ? d[c] : INFINITY;
            ref[c] = keep ? ref[c] : kRefEmpty;
        }
        sort_children<K>(d, ref);
        // culled entries sort last (infinite distance) or tie with a genuine
        // infinite distance; the reference tells them apart
#pragma unroll
        for (int c = K - 1; c >= 1; c--) {
            if (ref[c] != kRefEmpty && !st.push(ref[c], d[c])) {
                incomplete = true;
                s.cur = kRefEmpty;
                return;
            }
        }
        s.cur = ref[0];
    }
    // The same step for the whole wave (every lane calls it; `act` lanes have
    // a query in progress): interior nodes per lane as in step, then the
    // leaves the lanes reached tested together (wave_cp_leaves).
    template <int LeafMode, class Stack>
    __device__ static void wave_step(const void *nodes, const SceneData &ld, const Query &q,
                                     Stack &st, State &s, uint32_t &nfetch, uint32_t &ntri,
                                     bool &incomplete, bool act, WaveLeafLds *wl) {
        bool want = false;
        uint32_t first = 0, cnt = 0;
        if (act) {
            if (s.cur == kRefEmpty) {
                while (st.sp > 0) {
                    float d;
                    const uint32_t r = st.pop(d);
                    if (d <= s.best.d2) {
                        s.cur = r;
                        break;
                    }
                }
            }
            if (s.cur != kRefEmpty) {
                if ((s.cur & 1u) == 0u) {  // a leaf: first triangle and count in the reference
                    want = true;
                    first = s.cur >> 5;
                    cnt = ((s.cur >> 1) & 0xFu) + 1u;
                    s.cur = kRefEmpty;
                } else {
                    step<LeafMode>(nodes, ld, q, st, s, nfetch, ntri, incomplete);
                }
            }
        }
        wave_cp_leaves<LeafMode>(ld, q, want, first, cnt, s.best, ntri, wl);
    }
};

template <int Layout>
struct CpqFor;
template <> struct CpqFor<BVH_LAYOUT_AABB2> { using type = CpqBin<BinAABB2>; };
template <> struct CpqFor<BVH_LAYOUT_PBRT_Q16> { using type = CpqBin<BinPbrtQ16>; };
template <> struct CpqFor<BVH_LAYOUT_SG_EQ> { using type = CpqBin<BinSgEq>; };
template <> struct CpqFor<BVH_LAYOUT_PBRT_SOAOS> { using type = CpqBin<BinPbrtSoAoS>; };
template <> struct CpqFor<BVH_LAYOUT_PBRT_Q16_SOAOS> { using type = CpqBin<BinPbrtQ16SoAoS>; };
template <> struct CpqFor<BVH_LAYOUT_SG_EQ_A16> { using type = CpqBin<BinSgEqA16>; };
template <> struct CpqFor<BVH_LAYOUT_BVH4> { using type = CpqWide<BVH_LAYOUT_BVH4>; };
template <> struct CpqFor<BVH_LAYOUT_BVH8_Q8> { using type = CpqWide<BVH_LAYOUT_BVH8_Q8>; };
template <> struct CpqFor<BVH_LAYOUT_BVH8_Q16> { using type = CpqWide<BVH_LAYOUT_BVH8_Q16>; };

__device__ inline void store_closest(bvh_closest *out, uint64_t i, const CpqBest &b) {
    const bool none = b.id == 0xFFFFFFFFu;
    int4 w;
    w.x = none ? -1 : (int)b.id;
    w.y = __float_as_int(none ? INFINITY : b.d2);
    w.z = __float_as_int(none ? 0.0f : b.u);
    w.w = __float_as_int(none ? 0.0f : b.v);
    reinterpret_cast<int4 *>(out)[i] = w;
}

constexpr uint32_t kNoQuery = 0xFFFFFFFFu;
constexpr uint32_t kCpqRefill = 16;  // idle lanes of a wave that trigger a refill
constexpr uint32_t kCpqClaim = 64;   // queries claimed per chunk

// Persistent kernel: lanes take query after query.  A wave hands new queries
// to its idle lanes once kCpqRefill of them are idle, from its pool of
// claimed queries; the first three quarters of the queries are dealt to the
// waves round-robin in 64-query chunks, the rest is claimed from a queue.
// Every wave leaves once the queue is drained and its lanes are idle.
template <int Layout, int LeafMode, bool Count, int SL>
__global__ __launch_bounds__(kTraceBlock) void k_cpq_persist(const void *nodes, int64_t n_nodes,
                                                             SceneData ld,
                                                             const bvh_point_query *qs,
                                                             uint64_t n, bvh_closest *out,
                                                             uint32_t *counts, Fallback fb,
                                                             SpillArea sa) {
    using Wk = typename CpqFor<Layout>::type;
    __shared__ uint32_t s_ref[SL * kTraceBlock];
    __shared__ float s_d[SL * kTraceBlock];
    __shared__ WaveLeafLds s_wl[kWavesPerBlock];
    const uint32_t lane = threadIdx.x & 63u;
    WaveLeafLds *const wl = s_wl + (threadIdx.x >> 6);
    SpillStack<true, SL> st(s_ref, s_d, sa);
    uint32_t qi = kNoQuery;
    Query q{};
    typename Wk::State ws{};
    uint32_t nfetch = 0, ntri = 0;
    bool incomplete = false;
    uint64_t pool = 0, pool_end = 0;  // wave-uniform pool of claimed queries
    bool drained = false;
    const uint32_t waves = gridDim.x * (kTraceBlock / 64u);
    const uint32_t wave =
        blockIdx.x * (kTraceBlock / 64u) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint64_t static_rounds = (n * 3u / 4u) / ((uint64_t)waves * kCpqClaim);
    const uint64_t static_end = static_rounds * waves * kCpqClaim;
    uint64_t round = 0;
    uint32_t queue = wave % kQueues;  // the wave's current dynamic queue (wave-uniform)
    for (;;) {
        const uint64_t idle = __builtin_amdgcn_ballot_w64(qi == kNoQuery);
        const uint32_t nidle = (uint32_t)__builtin_popcountll(idle);
        if (nidle >= kCpqRefill && !(drained && pool == pool_end)) {
            const uint32_t avail = (uint32_t)(pool_end - pool);
            uint64_t fresh = 0, fresh_end = 0;  // a newly claimed range
            if (avail < nidle && !drained) {
                if (round < static_rounds) {
                    fresh = (round * waves + wave) * kCpqClaim;
                    fresh_end = fresh + kCpqClaim;
                    round++;
                } else if (!claim_dynamic(fb, static_end, n, kCpqClaim,
                                          (uint32_t)__builtin_ctzll(idle), queue, fresh,
                                          fresh_end)) {
                    drained = true;
                }
            }
            const uint32_t fresh_n = (uint32_t)(fresh_end - fresh);
            if (qi == kNoQuery) {
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                    (uint32_t)(idle >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
                uint64_t my = kNoQuery;
                if (rank < avail) my = pool + rank;
                else if (rank - avail < fresh_n) my = fresh + (rank - avail);
                if (my != kNoQuery) {
                    qi = (uint32_t)my;
                    q = load_query(qs, my);
                    st.reset();
                    nfetch = ntri = 0;
                    incomplete = false;
                    ws = Wk::start(nodes, n_nodes, ld, q, nfetch);
                }
            }
            if (avail >= nidle) {
                pool += nidle;
            } else if (fresh_n > 0) {
                pool = fresh + min(nidle - avail, fresh_n);
                pool_end = fresh + fresh_n;
            } else {
                pool = pool_end;
            }
        }
        const uint64_t busy = __builtin_amdgcn_ballot_w64(qi != kNoQuery);
        if (busy == 0) {
            if (drained && pool == pool_end) break;
            continue;
        }
        {  // every lane: the wave's leaves are tested together
            const bool act = qi != kNoQuery && !Wk::done(ws, st);
            Wk::template wave_step<LeafMode>(nodes, ld, q, st, ws, nfetch, ntri, incomplete, act, wl);
        }
        if (qi != kNoQuery) {
            if (incomplete) {
                fallback_append(fb, qi);
                st.reset();
                qi = kNoQuery;
            } else if (Wk::done(ws, st)) {
                store_closest(out, qi, ws.best);
                if (Count) {
                    counts[2 * (size_t)qi] = nfetch;
                    counts[2 * (size_t)qi + 1] = ntri;
                }
                qi = kNoQuery;
            }
        }
    }
}

// Fallback pass: the listed queries from the root with a deep stack in
// global memory (the build bounds the stack a query needs by kStackMax).
template <int Layout, int LeafMode, bool Count>
__global__ __launch_bounds__(kTraceBlock) void k_cpq_fallback(const void *nodes, int64_t n_nodes,
                                                              SceneData ld,
                                                              const bvh_point_query *qs,
                                                              bvh_closest *out, uint32_t *counts,
                                                              Fallback fb) {
    using Wk = typename CpqFor<Layout>::type;
    const uint32_t lane = blockIdx.x * kTraceBlock + threadIdx.x;
    const uint32_t total = *fb.count;
    for (uint32_t k = lane; k < total; k += kFallbackLanes) {
        const uint32_t i = fb.list[k];
        const Query q = load_query(qs, i);
        uint32_t nfetch = 0, ntri = 0;
        bool incomplete = false;
        GlobalStack<true> st(fb.stack_ref + (size_t)lane * kStackMax,
                             fb.stack_t + (size_t)lane * kStackMax);
        typename Wk::State ws = Wk::start(nodes, n_nodes, ld, q, nfetch);
        while (!Wk::done(ws, st) && !incomplete)
            Wk::template step<LeafMode>(nodes, ld, q, st, ws, nfetch, ntri, incomplete);
        store_closest(out, i, ws.best);
        if (Count) {
            counts[2 * (size_t)i] = nfetch;
            counts[2 * (size_t)i + 1] = ntri;
        }
    }
}

// Shared-slab layout: each stack entry carries its node's own box (the
// inherited box with the node's slab) and that box's distance.  Visiting an
// interior node loads both children's slabs, forms their boxes and continues
// with the nearer; grid-stride over the queries.
template <int LeafMode, bool Count>
__global__ __launch_bounds__(kTraceBlock) void k_cpq_slab(const bvh_node_slab *nodes,
                                                          int64_t n_nodes, SceneData ld,
                                                          const bvh_point_query *qs, uint64_t n,
                                                          bvh_closest *out, uint32_t *counts,
                                                          CarriedStack cs) {
    const uint32_t lane = blockIdx.x * kTraceBlock + threadIdx.x;
    for (uint64_t i = lane; i < n; i += cs.lanes) {
        const Query q = load_query(qs, i);
        CpqBest best{q.r2, 0.0f, 0.0f, 0xFFFFFFFFu};
        uint32_t nfetch = 0, ntri = 0, sp = 0;
        uint32_t cur = kRefEmpty, cnt = 0, off = 0, split = 0;
        float lo[3], hi[3];  // the current node's own box
        if (q.live && n_nodes > 0) {
            const bvh_node_slab r0 = nodes[0];
            nfetch++;
            const uint32_t sa = (r0.meta >> 16) & 3u;
            for (int k = 0; k < 3; k++) {
                lo[k] = (uint32_t)k == sa ? r0.slo : ld.fo[k];
                hi[k] = (uint32_t)k == sa ? r0.shi : ld.ft[k];
            }
            if (box_d2(q, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]) <= best.d2) {
                cur = 0;
                cnt = r0.meta & 0xFFFFu;
                off = r0.offset;
                split = (r0.meta >> 18) & 3u;
            }
        }
        for (;;) {
            if (cur == kRefEmpty) {
                while (sp > 0) {
                    sp--;
                    const float d = cs.box[((size_t)sp * 7 + 6) * cs.lanes + lane];
                    if (d <= best.d2) {
                        cur = cs.ref[(size_t)sp * cs.lanes + lane];
                        for (int k = 0; k < 3; k++) {
                            lo[k] = cs.box[((size_t)sp * 7 + k) * cs.lanes + lane];
                            hi[k] = cs.box[((size_t)sp * 7 + 3 + k) * cs.lanes + lane];
                        }
                        break;
                    }
                }
                if (cur == kRefEmpty || cur >= (uint64_t)n_nodes) break;
                const bvh_node_slab nd = nodes[cur];
                nfetch++;
                cnt = nd.meta & 0xFFFFu;
                off = nd.offset;
                split = (nd.meta >> 18) & 3u;
            }
            if (cnt > 0) {
                cp_leaf<LeafMode>(ld, q, off, cnt, best, ntri);
                cur = kRefEmpty;
                continue;
            }
            const uint32_t ci[2] = {cur + 1u, cur + off};
            if (ci[1] >= (uint64_t)n_nodes) break;  // bounds guard; a valid tree never takes it
            const bvh_node_slab c0 = nodes[ci[0]], c1 = nodes[ci[1]];
            nfetch += 2;
            float clo[2][3], chi[2][3], d[2];
            const bvh_node_slab cr[2] = {c0, c1};
            for (int c = 0; c < 2; c++) {
                const uint32_t sa = (cr[c].meta >> 16) & 3u;
                for (int k = 0; k < 3; k++) {
                    clo[c][k] = (uint32_t)k == sa ? cr[c].slo : lo[k];
                    chi[c][k] = (uint32_t)k == sa ? cr[c].shi : hi[k];
                }
                d[c] = box_d2(q, clo[c][0], clo[c][1], clo[c][2], chi[c][0], chi[c][1], chi[c][2]);
            }
            const bool ok0 = d[0] <= best.d2, ok1 = d[1] <= best.d2;
            int next = -1;
            if (ok0 && ok1) {
                const int nr = d[0] <= d[1] ? 0 : 1, fr = 1 - nr;
                if (sp < cs.cap) {  // the build bounds the pushes per path by cap - 1
                    cs.ref[(size_t)sp * cs.lanes + lane] = ci[fr];
                    for (int k = 0; k < 3; k++) {
                        cs.box[((size_t)sp * 7 + k) * cs.lanes + lane] = clo[fr][k];
                        cs.box[((size_t)sp * 7 + 3 + k) * cs.lanes + lane] = chi[fr][k];
                    }
                    cs.box[((size_t)sp * 7 + 6) * cs.lanes + lane] = d[fr];
                    sp++;
                }
                next = nr;
            } else if (ok0 || ok1) {
                next = ok0 ? 0 : 1;
            }
            if (next < 0) {
                cur = kRefEmpty;
                continue;
            }
            cur = ci[next];
            cnt = cr[next].meta & 0xFFFFu;
            off = cr[next].offset;
            split = (cr[next].meta >> 18) & 3u;
            for (int k = 0; k < 3; k++) {
                lo[k] = clo[next][k];
                hi[k] = chi[next][k];
            }
        }
        (void)split;
        store_closest(out, i, best);
        if (Count) {
            counts[2 * (size_t)i] = nfetch;
            counts[2 * (size_t)i + 1] = ntri;
        }
    }
}

template <int Layout, int LeafMode, bool Count, int SL>
int32_t launch_layout(const bvh_handle_s *h, const SceneData &ld, const bvh_point_query *qs,
                      uint64_t n, bvh_closest *out, uint32_t *counts, hipStream_t s) {
    auto kernel = k_cpq_persist<Layout, LeafMode, Count, SL>;
    unsigned resident = 0;
    BVH_TRY(resident_blocks(kernel, resident));
    const uint64_t need = (n + kTraceBlock - 1) / kTraceBlock;
    const unsigned grid = (unsigned)std::min<uint64_t>(resident, need);
    TraceArea ta;
    BVH_TRY(trace_area(s, n, grid * kTraceBlock, ta));
    kernel<<<grid, kTraceBlock, 0, s>>>(h->nodes, h->n_nodes, ld, qs, n, out, counts, ta.fb, ta.sa);
    k_cpq_fallback<Layout, LeafMode, Count><<<kFallbackBlocks, kTraceBlock, 0, s>>>(
        h->nodes, h->n_nodes, ld, qs, out, counts, ta.fb);
    return BVH_OK;
}

template <int LeafMode, bool Count, int SL>
int32_t launch_sl(const bvh_handle_s *h, const SceneData &ld, const bvh_point_query *qs, uint64_t n,
                  bvh_closest *out, uint32_t *counts, hipStream_t s) {
    switch (h->layout) {
        case BVH_LAYOUT_AABB2:
            return launch_layout<BVH_LAYOUT_AABB2, LeafMode, Count, SL>(h, ld, qs, n, out, counts, s);
        case BVH_LAYOUT_BVH4:
            return launch_layout<BVH_LAYOUT_BVH4, LeafMode, Count, SL>(h, ld, qs, n, out, counts, s);
        case BVH_LAYOUT_BVH8_Q8:
            return launch_layout<BVH_LAYOUT_BVH8_Q8, LeafMode, Count, SL>(h, ld, qs, n, out, counts, s);
        case BVH_LAYOUT_PBRT_Q16:
            return launch_layout<BVH_LAYOUT_PBRT_Q16, LeafMode, Count, SL>(h, ld, qs, n, out, counts, s);
        case BVH_LAYOUT_SG_EQ:
            return launch_layout<BVH_LAYOUT_SG_EQ, LeafMode, Count, SL>(h, ld, qs, n, out, counts, s);
        case BVH_LAYOUT_PBRT_SOAOS:
            return launch_layout<BVH_LAYOUT_PBRT_SOAOS, LeafMode, Count, SL>(h, ld, qs, n, out, counts, s);
        case BVH_LAYOUT_PBRT_Q16_SOAOS:
            return launch_layout<BVH_LAYOUT_PBRT_Q16_SOAOS, LeafMode, Count, SL>(h, ld, qs, n, out,
                                                                                counts, s);
        case BVH_LAYOUT_SG_EQ_A16:
            return launch_layout<BVH_LAYOUT_SG_EQ_A16, LeafMode, Count, SL>(h, ld, qs, n, out, counts, s);
        default:
            return launch_layout<BVH_LAYOUT_BVH8_Q16, LeafMode, Count, SL>(h, ld, qs, n, out, counts, s);
    }
}

template <int LeafMode, bool Count>
int32_t launch_mode(const bvh_handle_s *h, const bvh_point_query *qs, uint64_t n, bvh_closest *out,
                    uint32_t *counts, hipStream_t s) {
    const SceneData ld = scene_data(h);
    int32_t rc;
    if (h->layout == BVH_LAYOUT_SHARED_SLAB) {
        CarriedStack cs;
        unsigned grid = 0;
        rc = carried_stack(s, n, h->max_stack, 7, cs, grid);
        if (rc == BVH_OK)
            k_cpq_slab<LeafMode, Count><<<grid, kTraceBlock, 0, s>>>(
                static_cast<const bvh_node_slab *>(h->nodes), h->n_nodes, ld, qs, n, out, counts, cs);
    } else {
        // every stack entry carries a distance, so the LDS ring holds at most
        // 16 entries per lane (32 would halve the resident waves); left at its
        // default, the wide layouts (whose kernel also holds the batched leaf
        // state in LDS) take 8, one more resident block per CU: 3-6 % faster
        // than 16 on the terrain and the spheres scene
        const bool eight = h->stack_lds == 8 || (h->stack_lds_default && h->arity > 2);
        rc = eight ? launch_sl<LeafMode, Count, 8>(h, ld, qs, n, out, counts, s)
                   : launch_sl<LeafMode, Count, 16>(h, ld, qs, n, out, counts, s);
    }
    if (rc != BVH_OK) return rc;
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(BVH_EHIP, "bvh_closest_point: launch failed: %s", hipGetErrorString(e));
    return BVH_OK;
}

template <bool Count>
int32_t launch(const bvh_handle_s *h, const bvh_point_query *qs, uint64_t n, bvh_closest *out,
               uint32_t *counts, hipStream_t s) {
    if (h->leaf_mode == BVH_LEAF_COMPACT)
        return launch_mode<BVH_LEAF_COMPACT, Count>(h, qs, n, out, counts, s);
    return launch_mode<BVH_LEAF_INDEXED, Count>(h, qs, n, out, counts, s);
}

int32_t validate(bvh_handle_t h, const bvh_point_query *qs, int64_t n, bvh_closest *out,
                 const char *who) {
    if (!h) return set_error(BVH_EINVAL, "%s: null handle", who);
    if (n < 0) return set_error(BVH_EINVAL, "%s: negative query count", who);
    if (n > 0 && (!qs || !out)) return set_error(BVH_EINVAL, "%s: null query or result buffer", who);
    if ((uint64_t)n > (uint64_t)0xFFFFFFFFu)
        return set_error(BVH_EUNSUPPORTED, "%s: more than 2^32 - 1 queries", who);
    return BVH_OK;
}

}  // namespace
}  // namespace bvhlib

using namespace bvhlib;

extern "C" int32_t bvh_closest_point(bvh_handle_t h, const bvh_point_query *queries, int64_t n,
                                     bvh_closest *out, void *stream) {
    BVH_TRY(validate(h, queries, n, out, "bvh_closest_point"));
    if (n == 0) return BVH_OK;
    BVH_TRY(check_handle_device(h, "bvh_closest_point"));
    return launch<false>(h, queries, (uint64_t)n, out, nullptr, static_cast<hipStream_t>(stream));
}

extern "C" int32_t bvh_closest_point_counts(bvh_handle_t h, const bvh_point_query *queries,
                                            int64_t n, bvh_closest *out, uint32_t *counts,
                                            void *stream) {
    BVH_TRY(validate(h, queries, n, out, "bvh_closest_point_counts"));
    if (n > 0 && !counts) return set_error(BVH_EINVAL, "bvh_closest_point_counts: null counts buffer");
    if (n == 0) return BVH_OK;
    BVH_TRY(check_handle_device(h, "bvh_closest_point_counts"));
    return launch<true>(h, queries, (uint64_t)n, out, counts, static_cast<hipStream_t>(stream));
}
