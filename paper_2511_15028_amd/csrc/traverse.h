// Device-side traversal shared by the per-scene and the batched kernels.
//
// One traversal routine per node family (binary nodes that carry their own
// box; wide nodes that carry their children's boxes), each instantiated with a
// layout decoder, so the search order and culling logic are written once and
// the node format is a type parameter: the decoupling of traversal from
// layout argued in Sec. 3-4 of the paper.
#pragma once

#include <cmath>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

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
    float knx, kny, knz;  // -(o * rdir) rounded up / down, for the one-FMA slab
    float kfx, kfy, kfz;  // distances (see slab_nf)
    bool nx, ny, nz;   // sign bits of d
    bool fast;         // the one-FMA slab distances are valid for this ray
};

// Scenes whose coordinates exceed this magnitude, and rays whose origin or
// 1/d components lie outside [2^-60, 2^60] in magnitude, use the two-rounding
// slab distances; everything else uses the one-FMA form.
constexpr float kFastLimit = 1.152921504606846976e18f;  // 2^60

// o * rdir moved outward by at least one ulp: the returned pair (lo, hi)
// brackets the exact product.
__device__ inline void bracket_product(float o, float rd, float &lo, float &hi) {
    const float c = o * rd;
    const float delta = fabsf(c) * 2.384185791015625e-07f + 2.350988701644575e-38f;  // 2^-22, 2^-125
    lo = c - delta;
    hi = c + delta;
}

// coord_max: largest coordinate magnitude of the scene (or +inf).
__device__ inline Ray load_ray(const bvh_ray *rays, uint64_t i, float coord_max) {
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
    float lo, hi;
    bracket_product(r.ox, r.rx, lo, hi);
    r.knx = -hi; r.kfx = -lo;
    bracket_product(r.oy, r.ry, lo, hi);
    r.kny = -hi; r.kfy = -lo;
    bracket_product(r.oz, r.rz, lo, hi);
    r.knz = -hi; r.kfz = -lo;
    const float rmax = fmaxf(fabsf(r.rx), fmaxf(fabsf(r.ry), fabsf(r.rz)));
    const float rmin = fminf(fabsf(r.rx), fminf(fabsf(r.ry), fabsf(r.rz)));
    const float omax = fmaxf(fabsf(r.ox), fmaxf(fabsf(r.oy), fabsf(r.oz)));
    r.fast = rmax <= kFastLimit && rmin >= 1.0f / kFastLimit && omax <= kFastLimit &&
             coord_max <= kFastLimit;  // false for NaN as well
    return r;
}

// True when every active lane's ray can use the one-FMA slab distances (a
// wave-uniform value, so the choice costs one scalar branch).
__device__ inline bool wave_fast(const Ray &r) {
    return __builtin_amdgcn_ballot_w64(!r.fast) == 0;
}

// True when the rays of the lanes in `mask` (those with `has` set) all point
// into the same octant.  Called by every lane of the wave, so the result is
// wave-uniform.
__device__ inline bool rays_share_octant(const Ray &r, bool has, uint64_t mask) {
    const uint64_t nx = __builtin_amdgcn_ballot_w64(has && r.nx);
    const uint64_t ny = __builtin_amdgcn_ballot_w64(has && r.ny);
    const uint64_t nz = __builtin_amdgcn_ballot_w64(has && r.nz);
    return (nx == 0 || nx == mask) && (ny == 0 || ny == mask) && (nz == 0 || nz == mask);
}

// True when the active lanes' rays all point into the same octant (a cheap
// wave-uniform coherence test: camera rays of neighbouring pixels pass it,
// scattered secondary rays do not).
__device__ inline bool wave_coherent(const Ray &r) {
    return rays_share_octant(r, true, __builtin_amdgcn_ballot_w64(true));
}

// Ray/box test (the slab method of Kay and Kajiya; the paper's traversal
// tests node boxes with it, App. G) on planes already ordered by the ray:
// (nx, ny, nz) are the planes the ray enters through (the lower plane of an
// axis where d >= +0, the upper where d <= -0), (fx, fy, fz) the planes it
// leaves through.  The node cull is folded in: the far end is
// clipped at tcur (the best hit so far, or tmax).  Returns the entry
// distance, or +inf when the box is culled.
//
// Plane distances: the two-rounding form (plane - o) * rdir, or, when Fast, one FMA plane * rdir - o * rdir with the product o * rdir
// bracketed outward (entry planes subtract an upper bound, exit planes a
// lower bound), so the computed entry distance never exceeds
// (plane - o) * rdir by more than one rounding and the exit distance never
// falls short of it by more than one rounding.  Either way the relative
// error of each distance against the exact (plane - o) / d stays below the
// far-distance widening, so no box that the ray meets before tcur is culled.
template <bool Fast>
__device__ inline float slab_nf(const Ray &r, float nx, float ny, float nz, float fx, float fy,
                                float fz, float tcur) {
    float tnx, tny, tnz, tfx, tfy, tfz;
    if (Fast) {
        tnx = fmaf(nx, r.rx, r.knx); tfx = fmaf(fx, r.rx, r.kfx);
        tny = fmaf(ny, r.ry, r.kny); tfy = fmaf(fy, r.ry, r.kfy);
        tnz = fmaf(nz, r.rz, r.knz); tfz = fmaf(fz, r.rz, r.kfz);
    } else {
        tnx = (nx - r.ox) * r.rx; tfx = (fx - r.ox) * r.rx;
        tny = (ny - r.oy) * r.ry; tfy = (fy - r.oy) * r.ry;
        tnz = (nz - r.oz) * r.rz; tfz = (fz - r.oz) * r.rz;
    }
    const float t_near = fmaxf(0.0f, fmaxf(tnx, fmaxf(tny, tnz)));
    const float t_far = fminf(tcur, fminf(tfx, fminf(tfy, tfz)));
    return (t_near <= t_far * kFarScale) ? t_near : INFINITY;
}

// The same test on a box given as (lo, hi): the entry and exit planes are
// chosen by the sign bit of each direction component.
template <bool Fast>
__device__ inline float slab(const Ray &r, float lox, float loy, float loz, float hix, float hiy,
                             float hiz, float tcur) {
    return slab_nf<Fast>(r, r.nx ? hix : lox, r.ny ? hiy : loy, r.nz ? hiz : loz,
                         r.nx ? lox : hix, r.ny ? loy : hiy, r.nz ? loz : hiz, tcur);
}

// Ray/triangle test: Moller and Trumbore (1997), with App. G's acceptance
// intervals (u, v >= 0 and u + v <= 1 inclusive, both faces; 0 < t <= tmax).
// Given p0 and the edges e1 = p1 - p0, e2 = p2 - p0 (as stored in a
// compacted leaf record), the hit o + t d = p0 + u e1 + v e2 is solved by
// Cramer's rule through P = d x e2, det = e1 . P, S = o - p0, Q = S x e1:
// U = S . P, V = d . Q, T = e2 . Q are u, v, t times det.  The interval
// tests run on those numerators with det's sign bit moved onto them (exact),
// against |det|, so only an accepted hit pays for the one correctly rounded
// division: t, u, v = (T, U, V) * (1 / |det|).  Every cross-product
// component is one product and one fused multiply-add, every dot product
// one product and two fused multiply-adds, in a fixed order, so the results
// are a fixed function of the f32 inputs (30 VALU operations up to the
// tests).
struct TriNum {
    float U, V, T, adet;
};

// The numerators and |det| of the test (no acceptance decision).
__device__ inline TriNum tri_numerators(const Ray &r, float p0x, float p0y, float p0z, float e1x,
                                        float e1y, float e1z, float e2x, float e2y, float e2z) {
    const float px = fmaf(r.dy, e2z, -(r.dz * e2y));
    const float py = fmaf(r.dz, e2x, -(r.dx * e2z));
    const float pz = fmaf(r.dx, e2y, -(r.dy * e2x));
    const float det = fmaf(e1z, pz, fmaf(e1y, py, e1x * px));
    const uint32_t sgn = __float_as_uint(det) & 0x80000000u;
    const float sx = r.ox - p0x, sy = r.oy - p0y, sz = r.oz - p0z;
    const float qx = fmaf(sy, e1z, -(sz * e1y));
    const float qy = fmaf(sz, e1x, -(sx * e1z));
    const float qz = fmaf(sx, e1y, -(sy * e1x));
    TriNum n;
    n.U = __uint_as_float(__float_as_uint(fmaf(sz, pz, fmaf(sy, py, sx * px))) ^ sgn);
    n.V = __uint_as_float(__float_as_uint(fmaf(r.dz, qz, fmaf(r.dy, qy, r.dx * qx))) ^ sgn);
    n.T = __uint_as_float(__float_as_uint(fmaf(e2z, qz, fmaf(e2y, qy, e2x * qx))) ^ sgn);
    n.adet = fabsf(det);
    return n;
}

__device__ inline bool tri_accept(const TriNum &n, float tmax) {
    return n.adet > 0.0f && n.adet < INFINITY && n.U >= 0.0f && n.V >= 0.0f &&
           n.U + n.V <= n.adet && n.T > 0.0f && n.T <= n.adet * tmax;
}

__device__ inline bool mt_edges(const Ray &r, float p0x, float p0y, float p0z, float e1x,
                                float e1y, float e1z, float e2x, float e2y, float e2z, float &t,
                                float &u, float &v) {
    const TriNum n = tri_numerators(r, p0x, p0y, p0z, e1x, e1y, e1z, e2x, e2y, e2z);
    if (!tri_accept(n, r.tmax)) return false;
    const float inv = 1.0f / n.adet;
    t = n.T * inv;
    u = n.U * inv;
    v = n.V * inv;
    return true;
}

// The same test from the three vertices.
__device__ inline bool mt(const Ray &r, float p0x, float p0y, float p0z, float p1x, float p1y,
                          float p1z, float p2x, float p2y, float p2z, float &t, float &u,
                          float &v) {
    return mt_edges(r, p0x, p0y, p0z, p1x - p0x, p1y - p0y, p1z - p0z, p2x - p0x, p2y - p0y,
                    p2z - p0z, t, u, v);
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

// Per-scene data the kernels need besides the node buffer.  Leaf storage:
// COMPACT reads 48-B records {p0, e1 = p1 - p0, e2 = p2 - p0, prim id} in
// leaf order; INDEXED
// reads a primitive id, its three vertex indices and three vertices.
struct SceneData {
    const void *leaf;
    const float *verts;
    const int32_t *tris;
    uint32_t n_tris;
    float coord_max;  // largest coordinate magnitude of the scene (selects the slab form)
    float fo[3], fs[3];  // PBRT_Q16, SG_EQ: lower plane = fmaf(q, fs[a], fo[a])
    float ft[3];         // SG_EQ: upper plane = fmaf(-q, fs[a], ft[a])
    const void *topo;    // split layouts: the topology array after the boxes
};

// Compacted leaves: triangles are fetched in batches of kLeafBatch (all loads
// issued before the first test, so their latencies overlap).
constexpr uint32_t kLeafBatch = 4;

// Tests triangles [first, first+n) of the leaf order.  Returns true when an
// any-hit query is satisfied.
template <int LeafMode, int Mode>
__device__ inline bool test_leaf(const SceneData &ld, const Ray &r, uint32_t first, uint32_t n,
                                 Best &best, uint32_t &ntri) {
    const uint32_t end = min(first + n, ld.n_tris);  // bounds guard; a valid tree never clips
    if (LeafMode == BVH_LEAF_COMPACT) {
        const float4 *base = static_cast<const float4 *>(ld.leaf);
        for (uint32_t k0 = first; k0 < end; k0 += kLeafBatch) {
            float4 qa[kLeafBatch], qb[kLeafBatch];
            float2 qc[kLeafBatch];  // e2.z and the prim id (the record's padding is not read)
#pragma unroll
            for (uint32_t j = 0; j < kLeafBatch; j++) {
                if (k0 + j < end) {
                    const float4 *p = base + 3 * (size_t)(k0 + j);
                    qa[j] = p[0];
                    qb[j] = p[1];
                    qc[j] = *reinterpret_cast<const float2 *>(p + 2);
                }
            }
            bool found = false;
#pragma unroll
            for (uint32_t j = 0; j < kLeafBatch; j++) {
                if (k0 + j < end && !found) {
                    ntri++;
                    float t, u, v;
                    const float4 a = qa[j], b = qb[j];
                    const float2 c = qc[j];
                    if (mt_edges(r, a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, t, u, v)) {
                        consider(best, t, u, v, __float_as_uint(c.y));
                        found = Mode == BVH_TRACE_ANY;
                    }
                }
            }
            if (found) return true;
        }
        return false;
    }
    for (uint32_t k = first; k < end; k++) {
        const uint32_t id = (uint32_t) static_cast<const int32_t *>(ld.leaf)[k];
        const int32_t *tv = ld.tris + 3 * (size_t)id;
        const float *a = ld.verts + 3 * (size_t)tv[0];
        const float *b = ld.verts + 3 * (size_t)tv[1];
        const float *c = ld.verts + 3 * (size_t)tv[2];
        ntri++;
        float t, u, v;
        if (mt(r, a[0], a[1], a[2], b[0], b[1], b[2], c[0], c[1], c[2], t, u, v)) {
            consider(best, t, u, v, id);
            if (Mode == BVH_TRACE_ANY) return true;
        }
    }
    return false;
}

// ---------------------------------------------------------------------------
// Wave-level leaf batching: the lanes of a wave that hold a leaf to test
// publish its triangles, and the wave tests the (ray, triangle) pairs one per
// lane, so a leaf phase costs one triangle test per 64 pairs instead of one
// per triangle of the largest leaf.  Per round of up to 64 pairs:
//   * pair slots are assigned by an exclusive prefix sum of the leaf sizes
//     over the lanes (five ballots: leaf sizes are below 32);
//   * each leaf lane writes its lane number into the slots of its pairs (an
//     LDS table), each pair lane reads its owner and fetches the owner's ray
//     and leaf start from the owner's registers (ds_bpermute);
//   * hits are reduced per owner with an LDS 64-bit minimum of
//     (t bits << 32 | primitive id): t > 0, so the bits order like the
//     values, and the minimum is the (t, id) lexicographic best; the lane
//     holding that pair then stores its (u, v) for the owner.
// The arithmetic of each test is exactly that of test_leaf, so the hits are
// the same bits.
// ---------------------------------------------------------------------------
struct WaveLeafLds {
    unsigned long long key[64];  // per owner lane: best (t bits, id) of the round
    float2 uv[64];               // per owner lane: (u, v) of that best
    uint32_t owner[64];          // per pair slot of the round: owner lane
};
constexpr int kWavesPerBlock = kTraceBlock / 64;

// Orders the calling wave's LDS accesses on either side (a wave executes
// its LDS instructions in order; this keeps the compiler from moving them).
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Set bits of m below the calling lane.
__device__ inline uint32_t count_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ inline float lane_f(float x, uint32_t src) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute((int)(src << 2), __float_as_int(x)));
}
__device__ inline uint32_t lane_u(uint32_t x, uint32_t src) {
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src << 2), (int)x);
}

// Called by every lane of the wave (converged).  Lanes with `want` set test
// triangles [first, first + cnt) of the leaf order against their ray; their
// best is updated and their triangle counter advanced.  Returns true in a
// want lane whose any-hit query was satisfied.
template <int LeafMode, int Mode>
__device__ inline bool wave_test_leaves(const SceneData &ld, const Ray &r, bool want,
                                        uint32_t first, uint32_t cnt, Best &best, uint32_t &ntri,
                                        WaveLeafLds *wl) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t c = want ? cnt : 0u;
    uint32_t pre = 0, total = 0;
#pragma unroll
    for (int b = 0; b < 5; b++) {
        const uint64_t m = __builtin_amdgcn_ballot_w64(((c >> b) & 1u) != 0u);
        pre += count_below(m) << b;
        total += (uint32_t)__builtin_popcountll(m) << b;
    }
    if (total == 0) return false;
    ntri += c;
    bool ended = false;
    for (uint32_t base = 0; base < total; base += 64u) {
        if (want) {
            const uint32_t lo = pre > base ? pre : base;
            const uint32_t hi = min(pre + c, base + 64u);
            for (uint32_t q = lo; q < hi; q++) wl->owner[q - base] = lane;
        }
        wl->key[lane] = ~0ull;
        wave_lds_sync();
        const uint32_t pair = base + lane;
        const bool act = pair < total;
        const uint32_t o = act ? wl->owner[lane] : lane;
        Ray ro;
        ro.ox = lane_f(r.ox, o); ro.oy = lane_f(r.oy, o); ro.oz = lane_f(r.oz, o);
        ro.dx = lane_f(r.dx, o); ro.dy = lane_f(r.dy, o); ro.dz = lane_f(r.dz, o);
        ro.tmax = lane_f(r.tmax, o);
        const uint32_t k = lane_u(first, o) + (pair - lane_u(pre, o));
        bool hit = false;
        float t = 0.0f, u = 0.0f, v = 0.0f;
        uint32_t id = 0;
        if (act && k < ld.n_tris) {  // bounds guard; a valid tree never fails it
            if (LeafMode == BVH_LEAF_COMPACT) {
                const float4 *p = static_cast<const float4 *>(ld.leaf) + 3 * (size_t)k;
                const float4 a = p[0], b = p[1];
                const float2 cc = *reinterpret_cast<const float2 *>(p + 2);
                hit = mt_edges(ro, a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, cc.x, t, u, v);
                id = __float_as_uint(cc.y);
            } else {
                id = (uint32_t) static_cast<const int32_t *>(ld.leaf)[k];
                const int32_t *tv = ld.tris + 3 * (size_t)id;
                const float *a = ld.verts + 3 * (size_t)tv[0];
                const float *b = ld.verts + 3 * (size_t)tv[1];
                const float *cv = ld.verts + 3 * (size_t)tv[2];
                hit = mt(ro, a[0], a[1], a[2], b[0], b[1], b[2], cv[0], cv[1], cv[2], t, u, v);
            }
        }
        const unsigned long long mine = ((unsigned long long)__float_as_uint(t) << 32) | id;
        if (hit) atomicMin(&wl->key[o], mine);
        wave_lds_sync();
        if (hit && wl->key[o] == mine) wl->uv[o] = make_float2(u, v);
        wave_lds_sync();
        if (want) {
            const unsigned long long kb = wl->key[lane];
            if (kb != ~0ull) {
                const float2 q = wl->uv[lane];
                consider(best, __uint_as_float((uint32_t)(kb >> 32)), q.x, q.y, (uint32_t)kb);
                if (Mode == BVH_TRACE_ANY) ended = true;
            }
        }
        wave_lds_sync();
    }
    return ended;
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

// Stack of one lane of a persistent kernel: a ring of SL entries in LDS
// (one column per lane) over a spill area in global memory that belongs to
// the lane for the whole launch.  When the ring is full, a push first moves
// its oldest half to the spill area; when it is empty, a pop first brings the
// newest spilled half back.  Entries [0, lo) live in the spill area, entries
// [lo, sp) in the ring (entry e in slot e mod SL).  A push fails only when
// the spill area (cap entries) is full.  A lane's spill entries are
// contiguous (reference and entry distance side by side), so moving half a
// ring writes or reads one run of SL/2 * 8 bytes (a 64-byte line for SL = 16)
// instead of SL scattered words.
struct SpillArea {
    uint2 *ent;       // [lanes][cap]: (reference, entry-distance bits)
    uint32_t lanes;   // lanes of the launch (the grid's threads)
    uint32_t cap;     // spill entries per lane (a multiple of SL / 2)
};

template <bool WithT, int SL>
struct SpillStack {
    static_assert((SL & (SL - 1)) == 0 && SL >= 2, "ring size must be a power of two");
    uint32_t *lds_ref;  // [SL][kTraceBlock]
    float *lds_t;       // [SL][kTraceBlock] when WithT
    SpillArea area;     // uniform across the launch
    uint32_t sp = 0, lo = 0;
    __device__ SpillStack(uint32_t *r, float *t, const SpillArea &a) : lds_ref(r), lds_t(t), area(a) {}
    __device__ void reset() { sp = lo = 0; }
    __device__ static uint32_t slot(uint32_t e) { return (e & (SL - 1)) * kTraceBlock + threadIdx.x; }
    // entry e of this lane's spill run (the lane's index in the grid)
    __device__ size_t spill_index(uint32_t e) const {
        return ((size_t)blockIdx.x * kTraceBlock + threadIdx.x) * area.cap + e;
    }
    __device__ bool push(uint32_t ref, float t) {
        if (sp - lo == (uint32_t)SL) {
            constexpr uint32_t H = SL / 2;
            if (lo + H > area.cap) return false;
            for (uint32_t e = lo; e < lo + H; e++)
                area.ent[spill_index(e)] =
                    make_uint2(lds_ref[slot(e)], WithT ? __float_as_uint(lds_t[slot(e)]) : 0u);
            lo += H;
        }
        lds_ref[slot(sp)] = ref;
        if (WithT) lds_t[slot(sp)] = t;
        sp++;
        return true;
    }
    __device__ uint32_t pop(float &t) {  // requires sp > 0
        if (sp == lo) {
            const uint32_t n = lo < (uint32_t)(SL / 2) ? lo : (uint32_t)(SL / 2);
            for (uint32_t e = lo - n; e < lo; e++) {
                const uint2 x = area.ent[spill_index(e)];
                lds_ref[slot(e)] = x.x;
                if (WithT) lds_t[slot(e)] = __uint_as_float(x.y);
            }
            lo -= n;
        }
        sp--;
        t = WithT ? lds_t[slot(sp)] : 0.0f;
        return lds_ref[slot(sp)];
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


// The best-hit bound that culls nodes: the best hit so far (closest-hit
// queries) or tmax.
template <int Mode>
__device__ inline float best_bound(const Ray &r, const Best &b) {
    return (Mode == BVH_TRACE_ANY) ? r.tmax : fminf(b.t, r.tmax);
}

// ---------------------------------------------------------------------------
// Binary layout with the box in the node (AABB2): visit a node by testing its
// own box against the current best; a leaf's triangles are then tested, an
// interior node continues with the near child (split axis and ray direction
// sign) and pushes the far child.
// ---------------------------------------------------------------------------
struct BinState {
    Best best;
    uint32_t node;  // next node to visit; kRefEmpty when no node is left
    uint32_t leaf;  // leaf parked by the two-phase order (kRefEmpty: none)
    uint32_t hold;  // a second leaf met while one is parked
};

__device__ inline BinState bin_start(int64_t n_nodes) {
    BinState s;
    s.best = Best{INFINITY, 0.0f, 0.0f, 0xFFFFFFFFu};
    s.node = n_nodes > 0 ? 0u : kRefEmpty;
    s.leaf = s.hold = kRefEmpty;
    return s;
}

template <class Stack>
__device__ inline uint32_t bin_pop(Stack &st) {
    float unused;
    return st.sp > 0 ? st.pop(unused) : kRefEmpty;
}

// Binary node formats: load node i as its box, triangle count (0 for an
// interior node), offset (right-child delta or first triangle) and split
// axis (3 when unknown).
struct BinAABB2 {
    static constexpr bool kSplit = false;
    __device__ static void load(const void *nodes, uint32_t i, const SceneData &, float *lo,
                                float *hi, uint32_t &cnt, uint32_t &off, uint32_t &axis) {
        const float4 *np = reinterpret_cast<const float4 *>(static_cast<const bvh_node_aabb2 *>(nodes) + i);
        const float4 a = np[0], b = np[1];
        lo[0] = a.x; lo[1] = a.y; lo[2] = a.z;
        hi[0] = a.w; hi[1] = b.x; hi[2] = b.y;
        off = __float_as_uint(b.z);
        const uint32_t meta = __float_as_uint(b.w);
        cnt = meta & 0xFFFFu;
        axis = (meta >> 16) & 3u;
    }
};

// pbrt-q16: one 16-B load; planes dequantised in the scene frame.
struct BinPbrtQ16 {
    static constexpr bool kSplit = false;
    __device__ static void load(const void *nodes, uint32_t i, const SceneData &sd, float *lo,
                                float *hi, uint32_t &cnt, uint32_t &off, uint32_t &axis) {
        const uint4 w = reinterpret_cast<const uint4 *>(nodes)[i];
        const uint32_t q[6] = {w.x & 0xFFFFu, w.x >> 16, w.y & 0xFFFFu,
                               w.y >> 16,     w.z & 0xFFFFu, w.z >> 16};
#pragma unroll
        for (int a = 0; a < 3; a++) {
            lo[a] = fmaf((float)q[a], sd.fs[a], sd.fo[a]);
            hi[a] = fmaf((float)q[3 + a], sd.fs[a], sd.fo[a]);
        }
        cnt = w.w & 0xFu;
        off = w.w >> 4;
        axis = (q[0] & 1u) | ((q[1] & 1u) << 1);
    }
};

// sg-eq: one 12-B load; 10-bit planes counted up from the frame origin
// (lower) and down from the frame top (upper).
struct BinSgEq {
    static constexpr bool kSplit = false;
    __device__ static void load(const void *nodes, uint32_t i, const SceneData &sd, float *lo,
                                float *hi, uint32_t &cnt, uint32_t &off, uint32_t &axis) {
        const uint32_t *p = static_cast<const uint32_t *>(nodes) + 3 * (size_t)i;
        const uint32_t ql = p[0], qh = p[1], w = p[2];
        const uint32_t qlo[3] = {(ql >> 20) & 1023u, (ql >> 10) & 1023u, ql & 1023u};
        const uint32_t qhi[3] = {(qh >> 20) & 1023u, (qh >> 10) & 1023u, qh & 1023u};
#pragma unroll
        for (int a = 0; a < 3; a++) {
            lo[a] = fmaf((float)qlo[a], sd.fs[a], sd.fo[a]);
            hi[a] = fmaf(-(float)qhi[a], sd.fs[a], sd.ft[a]);
        }
        cnt = (ql >> 30) | ((qh >> 30) << 2);
        off = w & 0x3FFFFFFFu;
        axis = cnt > 0 ? 3u : (w >> 30);
    }
};

// Split layouts (box array, then topology array): load_box fetches only the
// box, load_meta the topology word(s), so a node whose box the query misses
// costs one fetch; load fetches both.
struct BinPbrtSoAoS {
    static constexpr bool kSplit = true;
    __device__ static void load_box(const void *nodes, uint32_t i, const SceneData &, float *lo,
                                    float *hi) {
        const float2 *p = static_cast<const float2 *>(nodes) + 3 * (size_t)i;
        const float2 a = p[0], b = p[1], c = p[2];
        lo[0] = a.x; lo[1] = a.y; lo[2] = b.x;
        hi[0] = b.y; hi[1] = c.x; hi[2] = c.y;
    }
    __device__ static void load_meta(uint32_t i, const SceneData &sd, uint32_t &cnt, uint32_t &off,
                                     uint32_t &axis) {
        const uint2 t = static_cast<const uint2 *>(sd.topo)[i];
        off = t.x;
        cnt = t.y & 0xFFFFu;
        axis = (t.y >> 16) & 3u;
    }
    __device__ static void load(const void *nodes, uint32_t i, const SceneData &sd, float *lo,
                                float *hi, uint32_t &cnt, uint32_t &off, uint32_t &axis) {
        load_box(nodes, i, sd, lo, hi);
        load_meta(i, sd, cnt, off, axis);
    }
};

struct BinPbrtQ16SoAoS {
    static constexpr bool kSplit = true;
    // boxes are 12 B: entry i starts at word 3 i (u16 pairs lo_x|lo_y, lo_z|hi_x, hi_y|hi_z)
    __device__ static void load_box_q(const void *nodes, uint32_t i, uint32_t *q) {
        const uint32_t *p = static_cast<const uint32_t *>(nodes) + 3 * (size_t)i;
        const uint32_t w0 = p[0], w1 = p[1], w2 = p[2];
        q[0] = w0 & 0xFFFFu; q[1] = w0 >> 16; q[2] = w1 & 0xFFFFu;
        q[3] = w1 >> 16;     q[4] = w2 & 0xFFFFu; q[5] = w2 >> 16;
    }
    __device__ static void load_box(const void *nodes, uint32_t i, const SceneData &sd, float *lo,
                                    float *hi) {
        uint32_t q[6];
        load_box_q(nodes, i, q);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            lo[a] = fmaf((float)q[a], sd.fs[a], sd.fo[a]);
            hi[a] = fmaf((float)q[3 + a], sd.fs[a], sd.fo[a]);
        }
    }
    // the split axis lives in the box (lowest bits of lo_x and lo_y)
    __device__ static void load_meta_axis(const void *nodes, uint32_t i, const SceneData &sd,
                                          uint32_t &cnt, uint32_t &off, uint32_t &axis) {
        const uint32_t m = static_cast<const uint32_t *>(sd.topo)[i];
        cnt = m & 0xFu;
        off = m >> 4;
        const uint32_t w0 = static_cast<const uint32_t *>(nodes)[3 * (size_t)i];
        axis = (w0 & 1u) | ((w0 >> 16) & 1u) << 1;
    }
    __device__ static void load(const void *nodes, uint32_t i, const SceneData &sd, float *lo,
                                float *hi, uint32_t &cnt, uint32_t &off, uint32_t &axis) {
        uint32_t q[6];
        load_box_q(nodes, i, q);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            lo[a] = fmaf((float)q[a], sd.fs[a], sd.fo[a]);
            hi[a] = fmaf((float)q[3 + a], sd.fs[a], sd.fo[a]);
        }
        const uint32_t m = static_cast<const uint32_t *>(sd.topo)[i];
        cnt = m & 0xFu;
        off = m >> 4;
        axis = (q[0] & 1u) | ((q[1] & 1u) << 1);
    }
};

// sg-eq records padded to 16 B: one aligned 16-byte fetch.
struct BinSgEqA16 {
    static constexpr bool kSplit = false;
    __device__ static void load(const void *nodes, uint32_t i, const SceneData &sd, float *lo,
                                float *hi, uint32_t &cnt, uint32_t &off, uint32_t &axis) {
        const uint4 r = static_cast<const uint4 *>(nodes)[i];
        const uint32_t ql = r.x, qh = r.y, w = r.z;
        const uint32_t qlo[3] = {(ql >> 20) & 1023u, (ql >> 10) & 1023u, ql & 1023u};
        const uint32_t qhi[3] = {(qh >> 20) & 1023u, (qh >> 10) & 1023u, qh & 1023u};
#pragma unroll
        for (int a = 0; a < 3; a++) {
            lo[a] = fmaf((float)qlo[a], sd.fs[a], sd.fo[a]);
            hi[a] = fmaf(-(float)qhi[a], sd.fs[a], sd.ft[a]);
        }
        cnt = (ql >> 30) | ((qh >> 30) << 2);
        off = w & 0x3FFFFFFFu;
        axis = cnt > 0 ? 3u : (w >> 30);
    }
};

// Split-layout meta fetch (the pbrt-q16 variant re-reads the box's first word
// for the axis bits, a cache hit after the box fetch).
template <class Node>
__device__ inline void split_meta(const void *nodes, uint32_t i, const SceneData &sd, uint32_t &cnt,
                                  uint32_t &off, uint32_t &axis) {
    if constexpr (std::is_same_v<Node, BinPbrtQ16SoAoS>)
        Node::load_meta_axis(nodes, i, sd, cnt, off, axis);
    else
        Node::load_meta(i, sd, cnt, off, axis);
}

// Visits bs.node; returns the leaf reference when the node is a leaf whose
// box the ray meets (kRefEmpty otherwise).  bs.node moves on to the next node.
template <class Node, int Mode, class Stack>
__device__ inline uint32_t bin_visit(const void *nodes, int64_t n_nodes, const SceneData &sd,
                                     const Ray &r, bool fast, Stack &st, BinState &bs,
                                     uint32_t &nfetch, bool &incomplete) {
    if (bs.node >= (uint64_t)n_nodes) {  // bounds guard; a valid tree never takes it
        bs.node = bs.leaf = bs.hold = kRefEmpty;
        return kRefEmpty;
    }
    float lo[3], hi[3];
    uint32_t cnt = 0, off = 0, axis = 0;
    if constexpr (Node::kSplit)
        Node::load_box(nodes, bs.node, sd, lo, hi);
    else
        Node::load(nodes, bs.node, sd, lo, hi, cnt, off, axis);
    nfetch++;
    const float tcur = best_bound<Mode>(r, bs.best);
    const float tn = fast ? slab<true>(r, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], tcur)
                          : slab<false>(r, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], tcur);
    if (tn != INFINITY) {
        if constexpr (Node::kSplit) split_meta<Node>(nodes, bs.node, sd, cnt, off, axis);
        if (cnt > 0) {
            bs.node = bin_pop(st);
            return ref_leaf(off, cnt);
        }
        const bool neg = axis == 0 ? r.nx : (axis == 1 ? r.ny : (axis == 2 ? r.nz : false));
        const uint32_t left = bs.node + 1, right = bs.node + off;
        if (!st.push(neg ? left : right, 0.0f)) {
            incomplete = true;
            bs.node = bs.leaf = bs.hold = kRefEmpty;
            return kRefEmpty;
        }
        bs.node = neg ? right : left;
        return kRefEmpty;
    }
    bs.node = bin_pop(st);
    return kRefEmpty;
}

// Tests the triangles of a leaf reference; a satisfied any-hit query ends
// the ray.
template <int LeafMode, int Mode>
__device__ inline bool bin_test_leaf(const SceneData &ld, const Ray &r, uint32_t leaf,
                                     BinState &bs, uint32_t &ntri) {
    const uint32_t first = leaf >> 5, cnt = ((leaf >> 1) & 0xFu) + 1u;
    if (test_leaf<LeafMode, Mode>(ld, r, first, cnt, bs.best, ntri)) {
        bs.node = bs.leaf = bs.hold = kRefEmpty;
        return true;
    }
    return false;
}

// ---------------------------------------------------------------------------
// Wide layouts: the node holds its children's boxes.  Decoders expose
//   K                      arity
//   Prep prep(ray)         per-ray constants (which plane arrays are near/far)
//   test(node ptr, node, ray, prep, tcur, tn[K], ref[K])
// writing the entry distance of every child the ray meets (+inf otherwise).
// ---------------------------------------------------------------------------

// BVH4: the near and far plane arrays of an axis are picked by address (the
// sign of the direction component decides whether lo_a or hi_a is entered
// first), so the per-child slab test needs no plane selects.
struct DecodeBVH4 {
    static constexpr int K = 4;
    // scattered waves end a round's interior phase at <= kStall progressing
    // lanes (terrain bounce rays: 0.674 ms with the single-loop order and
    // batched leaves; 0.616 / 0.600 / 0.577 / 0.559 / 0.563 / 0.585 / 0.646
    // ms at 8 / 16 / 24 / 32 / 40 / 48 / 56)
    static constexpr uint32_t kStall = 32;
    struct Prep {
        // byte offsets of the entry-plane arrays in a node; the exit-plane
        // array of an axis is the other one of the pair (lo_a, hi_a), at
        // (lo_a + hi_a offsets) - entry offset
        uint32_t nx, ny, nz;
    };
    __device__ static Prep prep(const Ray &r) {
        Prep p;
        p.nx = r.nx ? 48u : 0u;
        p.ny = r.ny ? 64u : 16u;
        p.nz = r.nz ? 80u : 32u;
        return p;
    }
    template <bool Fast>
    __device__ static void test(const void *base, uint32_t node, const Ray &r, const Prep &pp,
                                float tcur, float *tn, uint32_t *ref) {
        // 32-bit byte offsets from the buffer base (the builder keeps wide
        // node buffers below 4 GiB), so each fetch is base + one offset
        const char *b = static_cast<const char *>(base);
        const uint32_t o = node * 128u;
        const float4 nx = *reinterpret_cast<const float4 *>(b + (o + pp.nx));
        const float4 ny = *reinterpret_cast<const float4 *>(b + (o + pp.ny));
        const float4 nz = *reinterpret_cast<const float4 *>(b + (o + pp.nz));
        const float4 fx = *reinterpret_cast<const float4 *>(b + ((o + 48u) - pp.nx));
        const float4 fy = *reinterpret_cast<const float4 *>(b + ((o + 80u) - pp.ny));
        const float4 fz = *reinterpret_cast<const float4 *>(b + ((o + 112u) - pp.nz));
        const uint4 ch = *reinterpret_cast<const uint4 *>(b + (o + 96u));
        tn[0] = slab_nf<Fast>(r, nx.x, ny.x, nz.x, fx.x, fy.x, fz.x, tcur);
        tn[1] = slab_nf<Fast>(r, nx.y, ny.y, nz.y, fx.y, fy.y, fz.y, tcur);
        tn[2] = slab_nf<Fast>(r, nx.z, ny.z, nz.z, fx.z, fy.z, fz.z, tcur);
        tn[3] = slab_nf<Fast>(r, nx.w, ny.w, nz.w, fx.w, fy.w, fz.w, tcur);
        ref[0] = ch.x;
        ref[1] = ch.y;
        ref[2] = ch.z;
        ref[3] = ch.w;
    }
};

// Byte c of the 8 packed bytes held in words (w0, w1).
__device__ inline uint32_t byte_of(uint32_t w0, uint32_t w1, int c) {
    return ((c < 4 ? w0 : w1) >> (8 * (c & 3))) & 0xFFu;
}
__device__ inline uint32_t half_of(const uint32_t *w, int c) {
    return (w[c >> 1] >> (16 * (c & 1))) & 0xFFFFu;
}

// Quantised layouts: the near/far choice is made once per packed word (four
// u8 or two u16 planes at a time) before dequantising.
struct SignPrep {
    bool nx, ny, nz;
};

struct DecodeBVH8Q8 {
    static constexpr int K = 8;
    // as DecodeBVH4::kStall (terrain bounce rays: 0.668 ms single-loop;
    // 0.705 / 0.653 / 0.620 / 0.632 / 0.665 ms at 16 / 32 / 40 / 48 / 56)
    static constexpr uint32_t kStall = 40;
    using Prep = SignPrep;
    __device__ static Prep prep(const Ray &r) { return Prep{r.nx, r.ny, r.nz}; }
    template <bool Fast>
    __device__ static void test(const void *base, uint32_t node, const Ray &r, const Prep &,
                                float tcur, float *tn, uint32_t *ref) {
        const uint4 *p = static_cast<const uint4 *>(base) + 8 * (size_t)node;
        uint32_t w[28];
#pragma unroll
        for (int k = 0; k < 7; k++) {
            const uint4 q = p[k];
            w[4 * k] = q.x; w[4 * k + 1] = q.y; w[4 * k + 2] = q.z; w[4 * k + 3] = q.w;
        }
        const float ox = __uint_as_float(w[0]), oy = __uint_as_float(w[1]), oz = __uint_as_float(w[2]);
        const float sx = __uint_as_float(w[3]), sy = __uint_as_float(w[4]), sz = __uint_as_float(w[5]);
        // words: lo_x 6-7, lo_y 8-9, lo_z 10-11, hi_x 12-13, hi_y 14-15, hi_z 16-17
        uint32_t n[6], f[6];
#pragma unroll
        for (int k = 0; k < 2; k++) {
            n[k] = r.nx ? w[12 + k] : w[6 + k];
            f[k] = r.nx ? w[6 + k] : w[12 + k];
            n[2 + k] = r.ny ? w[14 + k] : w[8 + k];
            f[2 + k] = r.ny ? w[8 + k] : w[14 + k];
            n[4 + k] = r.nz ? w[16 + k] : w[10 + k];
            f[4 + k] = r.nz ? w[10 + k] : w[16 + k];
        }
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const float nxp = fmaf((float)byte_of(n[0], n[1], c), sx, ox);
            const float nyp = fmaf((float)byte_of(n[2], n[3], c), sy, oy);
            const float nzp = fmaf((float)byte_of(n[4], n[5], c), sz, oz);
            const float fxp = fmaf((float)byte_of(f[0], f[1], c), sx, ox);
            const float fyp = fmaf((float)byte_of(f[2], f[3], c), sy, oy);
            const float fzp = fmaf((float)byte_of(f[4], f[5], c), sz, oz);
            const bool valid = (uint32_t)c < w[26];
            tn[c] = valid ? slab_nf<Fast>(r, nxp, nyp, nzp, fxp, fyp, fzp, tcur) : INFINITY;
            ref[c] = w[18 + c];
        }
    }
};

struct DecodeBVH8Q16 {
    static constexpr int K = 8;
    static constexpr uint32_t kStall = 40;  // 0.642 ms at 40 (0.688 single-loop)
    using Prep = SignPrep;
    __device__ static Prep prep(const Ray &r) { return Prep{r.nx, r.ny, r.nz}; }
    template <bool Fast>
    __device__ static void test(const void *base, uint32_t node, const Ray &r, const Prep &,
                                float tcur, float *tn, uint32_t *ref) {
        const uint4 *p = static_cast<const uint4 *>(base) + 10 * (size_t)node;
        uint32_t w[40];
#pragma unroll
        for (int k = 0; k < 10; k++) {
            const uint4 q = p[k];
            w[4 * k] = q.x; w[4 * k + 1] = q.y; w[4 * k + 2] = q.z; w[4 * k + 3] = q.w;
        }
        const float ox = __uint_as_float(w[0]), oy = __uint_as_float(w[1]), oz = __uint_as_float(w[2]);
        const float sx = __uint_as_float(w[3]), sy = __uint_as_float(w[4]), sz = __uint_as_float(w[5]);
        // words: lo_x 6-9, lo_y 10-13, lo_z 14-17, hi_x 18-21, hi_y 22-25, hi_z 26-29
        uint32_t n[12], f[12];
#pragma unroll
        for (int k = 0; k < 4; k++) {
            n[k] = r.nx ? w[18 + k] : w[6 + k];
            f[k] = r.nx ? w[6 + k] : w[18 + k];
            n[4 + k] = r.ny ? w[22 + k] : w[10 + k];
            f[4 + k] = r.ny ? w[10 + k] : w[22 + k];
            n[8 + k] = r.nz ? w[26 + k] : w[14 + k];
            f[8 + k] = r.nz ? w[14 + k] : w[26 + k];
        }
#pragma unroll
        for (int c = 0; c < 8; c++) {
            const float nxp = fmaf((float)half_of(n, c), sx, ox);
            const float nyp = fmaf((float)half_of(n + 4, c), sy, oy);
            const float nzp = fmaf((float)half_of(n + 8, c), sz, oz);
            const float fxp = fmaf((float)half_of(f, c), sx, ox);
            const float fyp = fmaf((float)half_of(f + 4, c), sy, oy);
            const float fzp = fmaf((float)half_of(f + 8, c), sz, oz);
            const bool valid = (uint32_t)c < w[38];
            tn[c] = valid ? slab_nf<Fast>(r, nxp, nyp, nzp, fxp, fyp, fzp, tcur) : INFINITY;
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


// Pops stack entries until one is not culled by tb (the current best hit or
// tmax); returns kRefEmpty when the stack runs dry.
template <class Stack>
__device__ inline uint32_t pop_unculled(Stack &st, float tb, float &t_entry) {
    while (st.sp > 0) {
        float t;
        const uint32_t ref = st.pop(t);
        if (t <= tb * kFarScale) {
            t_entry = t;
            return ref;
        }
    }
    return kRefEmpty;
}

// Traversal state of one ray in a wide BVH.
struct WideState {
    Best best;
    uint32_t cur;    // entry to visit next; kRefEmpty once the ray is done
    float cur_t;     // entry distance of cur
    uint32_t leaf;   // leaf parked by the two-phase order (kRefEmpty: none)
};

__device__ inline WideState wide_start(int64_t n_nodes) {
    WideState ws;
    ws.best = Best{INFINITY, 0.0f, 0.0f, 0xFFFFFFFFu};
    ws.cur = n_nodes > 0 ? ref_interior(0) : kRefEmpty;
    ws.cur_t = 0.0f;
    ws.leaf = kRefEmpty;
    return ws;
}

// Visits the interior node ws.cur: tests all its children, sorts the hit ones
// near-first, pushes all but the nearest with their entry distances and
// continues with the nearest (or with the next unculled stack entry when no
// child is hit).  A failed push (stack full) ends the ray as incomplete.
template <class Dec, int Mode, class Stack>
__device__ inline void wide_visit_interior(const void *nodes, int64_t n_nodes, const Ray &r,
                                           const typename Dec::Prep &prep, bool fast, Stack &st,
                                           WideState &ws, uint32_t &nfetch, bool &incomplete) {
    constexpr int K = Dec::K;
    const float tcur = best_bound<Mode>(r, ws.best);
    if ((ws.cur >> 1) >= (uint64_t)n_nodes) {  // bounds guard; never taken on a valid tree
        ws.cur = kRefEmpty;
        ws.leaf = kRefEmpty;
        return;
    }
    float tn[K];
    uint32_t ref[K];
    if (fast)
        Dec::template test<true>(nodes, ws.cur >> 1, r, prep, tcur, tn, ref);
    else
        Dec::template test<false>(nodes, ws.cur >> 1, r, prep, tcur, tn, ref);
    nfetch++;
    sort_children<K>(tn, ref);
    bool ok = true;
#pragma unroll
    for (int c = K - 1; c >= 1; c--)
        if (tn[c] != INFINITY) ok = st.push(ref[c], tn[c]) && ok;
    if (!ok) {
        incomplete = true;
        ws.cur = kRefEmpty;
        ws.leaf = kRefEmpty;
    } else if (tn[0] != INFINITY) {
        ws.cur = ref[0];
        ws.cur_t = tn[0];
    } else {
        ws.cur = pop_unculled(st, tcur, ws.cur_t);
    }
}

// Tests the triangles of a leaf reference; an any-hit query that is
// satisfied ends the ray.
template <int LeafMode, int Mode>
__device__ inline bool wide_test_leaf(const SceneData &ld, const Ray &r, uint32_t leaf,
                                      WideState &ws, uint32_t &ntri) {
    const uint32_t first = leaf >> 5, cnt = ((leaf >> 1) & 0xFu) + 1u;
    if (test_leaf<LeafMode, Mode>(ld, r, first, cnt, ws.best, ntri)) {
        ws.cur = kRefEmpty;
        ws.leaf = kRefEmpty;
        return true;
    }
    return false;
}

// One step of the single-loop order: visit ws.cur (interior node or leaf),
// then take the next entry.  The best hit is updated as soon as a leaf is
// tested, which culls the most.
template <class Dec, int LeafMode, int Mode, class Stack>
__device__ inline void wide_step_single(const void *nodes, int64_t n_nodes, const SceneData &ld,
                                        const Ray &r, const typename Dec::Prep &prep, bool fast,
                                        Stack &st, WideState &ws, uint32_t &nfetch,
                                        uint32_t &ntri, bool &incomplete) {
    if (ws.cur & 1u) {
        wide_visit_interior<Dec, Mode>(nodes, n_nodes, r, prep, fast, st, ws, nfetch, incomplete);
        return;
    }
    if (wide_test_leaf<LeafMode, Mode>(ld, r, ws.cur, ws, ntri)) return;
    ws.cur = pop_unculled(st, best_bound<Mode>(r, ws.best), ws.cur_t);
}

// One round of the two-phase order (the while-while scheme of Aila and
// Laine 2009, with speculative traversal), wave-wide, so that the lanes test
// nodes together and triangles together instead of splitting every step
// between the two:
//   interior phase: lanes visit interior nodes; a lane that reaches a leaf
//     parks it (one at a time) and keeps descending; the phase ends when
//     every lane has a parked leaf or has no entry left;
//   leaf phase: every lane with a parked leaf tests its triangles.
// Every node that the current best does not cull is still visited, so the
// result equals the single-loop order's.
template <class Dec, int LeafMode, int Mode, class Stack>
__device__ inline void wide_round_two_phase(const void *nodes, int64_t n_nodes,
                                            const SceneData &ld, const Ray &r,
                                            const typename Dec::Prep &prep, bool fast,
                                            Stack &st, WideState &ws, uint32_t &nfetch,
                                            uint32_t &ntri, bool &incomplete) {
    for (;;) {
        if (ws.cur != kRefEmpty && (ws.cur & 1u))
            wide_visit_interior<Dec, Mode>(nodes, n_nodes, r, prep, fast, st, ws, nfetch,
                                           incomplete);
        if (ws.cur != kRefEmpty && !(ws.cur & 1u) && ws.leaf == kRefEmpty) {
            ws.leaf = ws.cur;
            ws.cur = pop_unculled(st, best_bound<Mode>(r, ws.best), ws.cur_t);
        }
        if (__builtin_amdgcn_ballot_w64(ws.leaf == kRefEmpty && ws.cur != kRefEmpty) == 0) break;
    }
    if (ws.leaf != kRefEmpty) {
        const uint32_t leaf = ws.leaf;
        ws.leaf = kRefEmpty;
        if (wide_test_leaf<LeafMode, Mode>(ld, r, leaf, ws, ntri)) return;
        // the entry taken before the leaf test may be culled by the new best
        const float tb = best_bound<Mode>(r, ws.best);
        if (ws.cur != kRefEmpty && !(ws.cur_t <= tb * kFarScale))
            ws.cur = pop_unculled(st, tb, ws.cur_t);
    }
}

// Two-phase round for scattered rays (called by every lane of the wave;
// `active` lanes have a ray): lanes visit interior nodes and park the first
// leaf they meet, continuing speculatively; a lane with a parked leaf whose
// next entry is a leaf waits.  The interior phase ends once at most `stall`
// lanes can still make progress (waiting for the last stragglers of an
// incoherent wave would idle the rest), and the parked leaves are then
// tested in one wave-batched leaf phase.  Nodes the best hit does not cull
// are all visited, so the result equals the single-loop order's.
template <class Dec, int LeafMode, int Mode, class Stack>
__device__ inline void wide_round_wave(const void *nodes, int64_t n_nodes, const SceneData &ld,
                                       const Ray &r, const typename Dec::Prep &prep, bool fast,
                                       Stack &st, WideState &ws, bool active, WaveLeafLds *wl,
                                       uint32_t stall, uint32_t &nfetch, uint32_t &ntri,
                                       bool &incomplete) {
    for (;;) {
        if (active && ws.cur != kRefEmpty && (ws.cur & 1u))
            wide_visit_interior<Dec, Mode>(nodes, n_nodes, r, prep, fast, st, ws, nfetch,
                                           incomplete);
        if (active && ws.cur != kRefEmpty && !(ws.cur & 1u) && ws.leaf == kRefEmpty) {
            ws.leaf = ws.cur;
            ws.cur = pop_unculled(st, best_bound<Mode>(r, ws.best), ws.cur_t);
        }
        const uint64_t prog = __builtin_amdgcn_ballot_w64(
            active && ws.cur != kRefEmpty && ((ws.cur & 1u) || ws.leaf == kRefEmpty));
        const uint64_t parked = __builtin_amdgcn_ballot_w64(active && ws.leaf != kRefEmpty);
        if (prog == 0 || ((uint32_t)__builtin_popcountll(prog) <= stall && parked != 0)) break;
    }
    const bool want = active && ws.leaf != kRefEmpty;
    const uint32_t first = ws.leaf >> 5, cnt = ((ws.leaf >> 1) & 0xFu) + 1u;
    const bool ended = wave_test_leaves<LeafMode, Mode>(ld, r, want, first, cnt, ws.best, ntri, wl);
    if (want) {
        ws.leaf = kRefEmpty;
        if (ended) {
            ws.cur = kRefEmpty;
        } else {
            const float tb = best_bound<Mode>(r, ws.best);
            if (ws.cur != kRefEmpty && !(ws.cur_t <= tb * kFarScale))
                ws.cur = pop_unculled(st, tb, ws.cur_t);
        }
    }
}

// ---------------------------------------------------------------------------
// Tracer policies: the per-layout state and steps behind one interface, so
// the kernels (one ray per lane, persistent, fallback, batched) are written
// once for all layouts.
//   kWithT              stack entries carry entry distances (pop-time cull)
//   Prep prep(ray)      per-ray layout constants
//   State start(nodes)  initial state;  done(state);  best(state)
//   step<LeafMode, Mode>(...)   one node or leaf of the single-loop order
//   kBatchLeaves, round_wave<LeafMode, Mode>(...)   (wide layouts) one round
//                       of the two-phase order with a wave-batched leaf phase
//   round<LeafMode, Mode>(...)  one round of the two-phase order (wave-wide)
// ---------------------------------------------------------------------------
template <class Dec>
struct WideTracer {
    static constexpr bool kWithT = true;
    // scattered waves batch their leaf tests across the wave (round_wave)
    static constexpr bool kBatchLeaves = true;
    using State = WideState;
    using Prep = typename Dec::Prep;
    __device__ static Prep prep(const Ray &r) { return Dec::prep(r); }
    __device__ static State start(int64_t n_nodes) { return wide_start(n_nodes); }
    __device__ static bool done(const State &s) { return s.cur == kRefEmpty; }
    template <int LeafMode, int Mode, class Stack>
    __device__ static void step(const void *nodes, int64_t n_nodes, const SceneData &ld,
                                const Ray &r, const Prep &prep, bool fast, Stack &st, State &s,
                                uint32_t &nfetch, uint32_t &ntri, bool &incomplete) {
        wide_step_single<Dec, LeafMode, Mode>(nodes, n_nodes, ld, r, prep, fast, st, s, nfetch,
                                              ntri, incomplete);
    }
    template <int LeafMode, int Mode, class Stack>
    __device__ static void round(const void *nodes, int64_t n_nodes, const SceneData &ld,
                                 const Ray &r, const Prep &prep, bool fast, Stack &st, State &s,
                                 uint32_t &nfetch, uint32_t &ntri, bool &incomplete) {
        wide_round_two_phase<Dec, LeafMode, Mode>(nodes, n_nodes, ld, r, prep, fast, st, s,
                                                  nfetch, ntri, incomplete);
    }
    // scattered waves: the two-phase round with a wave-batched leaf phase
    template <int LeafMode, int Mode, class Stack>
    __device__ static void round_wave(const void *nodes, int64_t n_nodes, const SceneData &ld,
                                      const Ray &r, const Prep &prep, bool fast, Stack &st,
                                      State &s, bool active, WaveLeafLds *wl, uint32_t &nfetch,
                                      uint32_t &ntri, bool &incomplete) {
        wide_round_wave<Dec, LeafMode, Mode>(nodes, n_nodes, ld, r, prep, fast, st, s, active, wl,
                                             Dec::kStall, nfetch, ntri, incomplete);
    }
};

template <class Node>
struct BinTracer {
    static constexpr bool kWithT = false;
    // a binary node visit is one box test, so a batched leaf phase per visit
    // costs more than it saves (measured 3-5 % slower on incoherent rays):
    // incoherent waves use the per-lane step
    static constexpr bool kBatchLeaves = false;
    using State = BinState;
    struct Prep {};
    __device__ static Prep prep(const Ray &) { return Prep{}; }
    __device__ static State start(int64_t n_nodes) { return bin_start(n_nodes); }
    __device__ static bool done(const State &s) {
        return s.node == kRefEmpty && s.leaf == kRefEmpty && s.hold == kRefEmpty;
    }
    // single-loop order: visit a node and test a leaf as soon as it is met.
    // A persistent wave can switch orders between rounds, so a leaf still
    // parked by the two-phase order is tested first.
    template <int LeafMode, int Mode, class Stack>
    __device__ static void step(const void *nodes, int64_t n_nodes, const SceneData &ld,
                                const Ray &r, const Prep &, bool fast, Stack &st, State &s,
                                uint32_t &nfetch, uint32_t &ntri, bool &incomplete) {
        if (s.leaf != kRefEmpty) {
            const uint32_t parked = s.leaf;
            s.leaf = s.hold;
            s.hold = kRefEmpty;
            bin_test_leaf<LeafMode, Mode>(ld, r, parked, s, ntri);
            return;
        }
        if (s.node == kRefEmpty) return;
        const uint32_t leaf =
            bin_visit<Node, Mode>(nodes, n_nodes, ld, r, fast, st, s, nfetch, incomplete);
        if (leaf != kRefEmpty) bin_test_leaf<LeafMode, Mode>(ld, r, leaf, s, ntri);
    }
    // two-phase order: lanes visit nodes and park the leaves they meet (one,
    // plus one held while the first is parked, after which the lane waits);
    // the phase ends when every lane has a parked leaf or no node left; then
    // the parked leaves are tested together.
    template <int LeafMode, int Mode, class Stack>
    __device__ static void round(const void *nodes, int64_t n_nodes, const SceneData &ld,
                                 const Ray &r, const Prep &, bool fast, Stack &st, State &s,
                                 uint32_t &nfetch, uint32_t &ntri, bool &incomplete) {
        for (;;) {
            if (s.node != kRefEmpty && s.hold == kRefEmpty) {
                const uint32_t leaf =
                    bin_visit<Node, Mode>(nodes, n_nodes, ld, r, fast, st, s, nfetch, incomplete);
                if (leaf != kRefEmpty) {
                    if (s.leaf == kRefEmpty) s.leaf = leaf;
                    else s.hold = leaf;
                }
            }
            if (__builtin_amdgcn_ballot_w64(s.leaf == kRefEmpty && s.node != kRefEmpty) == 0) break;
        }
        if (s.leaf != kRefEmpty) {
            const uint32_t leaf = s.leaf;
            s.leaf = s.hold;
            s.hold = kRefEmpty;
            bin_test_leaf<LeafMode, Mode>(ld, r, leaf, s, ntri);
        }
    }
};

template <int Layout>
struct TracerFor;
template <>
struct TracerFor<BVH_LAYOUT_AABB2> {
    using type = BinTracer<BinAABB2>;
};
template <>
struct TracerFor<BVH_LAYOUT_PBRT_Q16> {
    using type = BinTracer<BinPbrtQ16>;
};
template <>
struct TracerFor<BVH_LAYOUT_SG_EQ> {
    using type = BinTracer<BinSgEq>;
};
template <>
struct TracerFor<BVH_LAYOUT_PBRT_SOAOS> {
    using type = BinTracer<BinPbrtSoAoS>;
};
template <>
struct TracerFor<BVH_LAYOUT_PBRT_Q16_SOAOS> {
    using type = BinTracer<BinPbrtQ16SoAoS>;
};
template <>
struct TracerFor<BVH_LAYOUT_SG_EQ_A16> {
    using type = BinTracer<BinSgEqA16>;
};
template <>
struct TracerFor<BVH_LAYOUT_BVH4> {
    using type = WideTracer<DecodeBVH4>;
};
template <>
struct TracerFor<BVH_LAYOUT_BVH8_Q8> {
    using type = WideTracer<DecodeBVH8Q8>;
};
template <>
struct TracerFor<BVH_LAYOUT_BVH8_Q16> {
    using type = WideTracer<DecodeBVH8Q16>;
};

// Whole-ray traversal: waves of coherent rays use the two-phase order (their
// lanes reach nodes and leaves in step, so batching the phases pays); other
// waves use the single-loop order, which updates the best hit earliest.
template <int Layout, int LeafMode, int Mode, class Stack>
__device__ inline Best trace_ray(const void *nodes, int64_t n_nodes, const SceneData &ld,
                                 const Ray &r, Stack &st, uint32_t &nfetch, uint32_t &ntri,
                                 bool &incomplete) {
    using Tr = typename TracerFor<Layout>::type;
    const typename Tr::Prep prep = Tr::prep(r);
    const bool fast = wave_fast(r);
    typename Tr::State s = Tr::start(n_nodes);
    if (wave_coherent(r)) {
        while (!Tr::done(s))
            Tr::template round<LeafMode, Mode>(nodes, n_nodes, ld, r, prep, fast, st, s, nfetch,
                                               ntri, incomplete);
    } else {
        while (!Tr::done(s))
            Tr::template step<LeafMode, Mode>(nodes, n_nodes, ld, r, prep, fast, st, s, nfetch,
                                              ntri, incomplete);
    }
    return s.best;
}

// Work area of the fallback pass: a counter and list of rays that
// overflowed the LDS stack, and one deep stack per fallback lane.
constexpr int kFallbackBlocks = 128;
constexpr int kFallbackLanes = kFallbackBlocks * kTraceBlock;
// The dynamic part of a persistent launch is dealt by kQueues counters, each
// on a line of its own and each handing out one slice of the part: waves
// start at different queues, so their claims do not all serialise on one
// word (device-scope atomics on one address are ordered across the XCDs).
constexpr uint32_t kQueues = 8;
constexpr size_t kQueueStride = 256;  // bytes between two queue counters

struct Fallback {
    uint32_t *count;     // rays appended by the fast pass
    unsigned long long *queue;  // queue q's next unclaimed offset at queue + q * kQueueStride bytes
    uint32_t *list;      // ray indices (capacity: rays of the launch)
    uint32_t *stack_ref; // [kFallbackLanes][kStackMax]
    float *stack_t;      // [kFallbackLanes][kStackMax]
};

// Bytes of the header (counter line, queue lines) that must be zero before a launch.
constexpr size_t kFallbackHeaderBytes = kQueueStride * (1 + kQueues);

// Bytes of a work area for n_rays rays and `lanes` fallback lanes (the
// fallback grid's threads).
constexpr size_t fallback_bytes(uint64_t n_rays, size_t lanes = kFallbackLanes) {
    return kFallbackHeaderBytes + n_rays * 4 + lanes * kStackMax * 8;
}

// Carves the work area out of one allocation of fallback_bytes(n_rays, lanes).
inline Fallback fallback_view(void *base, uint64_t n_rays, size_t lanes = kFallbackLanes) {
    char *p = static_cast<char *>(base);
    Fallback f;
    f.count = reinterpret_cast<uint32_t *>(p);
    f.queue = reinterpret_cast<unsigned long long *>(p + kQueueStride);
    char *q = p + kFallbackHeaderBytes;
    f.list = reinterpret_cast<uint32_t *>(q);
    f.stack_ref = reinterpret_cast<uint32_t *>(q + n_rays * 4);
    f.stack_t = reinterpret_cast<float *>(q + n_rays * 4 + lanes * kStackMax * 4);
    return f;
}

// Claims the calling wave's next chunk of `claim` items of the dynamic part
// [static_end, n) (wave-uniform call; `leader` is an active lane): from queue
// q, then from the following queues as they run dry (q is updated).  Returns
// false once all are exhausted, else the chunk [fresh, fresh_end).
__device__ inline bool claim_dynamic(const Fallback &fb, uint64_t static_end, uint64_t n,
                                     uint32_t claim, uint32_t leader, uint32_t &q,
                                     uint64_t &fresh, uint64_t &fresh_end) {
    const uint64_t qlen = (n - static_end + kQueues - 1) / kQueues;
    for (uint32_t tries = 0; tries < kQueues; tries++) {
        const uint64_t qs = static_end + (uint64_t)q * qlen;
        const uint64_t qe = qs + qlen < n ? qs + qlen : n;
        uint32_t lo = 0xFFFFFFFFu, hi = 0x7FFFFFFFu;  // "exhausted" for an empty slice
        if ((threadIdx.x & 63u) == leader && qs < qe) {
            unsigned long long *w = reinterpret_cast<unsigned long long *>(
                reinterpret_cast<char *>(fb.queue) + (size_t)q * kQueueStride);
            const unsigned long long b = atomicAdd(w, (unsigned long long)claim);
            lo = (uint32_t)b;
            hi = (uint32_t)(b >> 32);
        }
        const uint64_t b = ((uint64_t)__builtin_amdgcn_readlane(hi, leader) << 32) |
                           __builtin_amdgcn_readlane(lo, leader);
        if (qs < qe && b < qe - qs) {
            fresh = qs + b;
            fresh_end = fresh + claim < qe ? fresh + claim : qe;
            return true;
        }
        q = (q + 1u) % kQueues;
    }
    return false;
}

__device__ inline void fallback_append(const Fallback &fb, uint32_t ray) {
    const uint32_t k = atomicAdd(fb.count, 1u);
    fb.list[k] = ray;
}

// ---------------------------------------------------------------------------
// Host-side launch helpers of the persistent kernels.
// ---------------------------------------------------------------------------
// Per-scene data of a handle for the traversal kernels.  SHARED_SLAB carries
// the scene box (the root's inherited box) in fo (lower) and ft (upper).
inline SceneData scene_data(const bvh_handle_s *h) {
    const bool slab = h->layout == BVH_LAYOUT_SHARED_SLAB;
    const float *lo = slab ? h->scene_lo : h->frame_origin;
    const float *top = slab ? h->scene_hi : h->frame_top;
    return SceneData{h->leaf, h->verts, h->tris, (uint32_t)h->n_tris, h->coord_max(),
                     {lo[0], lo[1], lo[2]},
                     {h->frame_scale[0], h->frame_scale[1], h->frame_scale[2]},
                     {top[0], top[1], top[2]},
                     topo_of(h->nodes, h->n_nodes, h->layout)};
}

// Per-lane stacks of the shared-slab kernels in a global work area: entry e
// of lane l is ref[e * lanes + l] and words box[(e * W + k) * lanes + l],
// k < W, of the box (and, for point queries, distance) it carries.
struct CarriedStack {
    uint32_t *ref;
    float *box;
    uint32_t lanes, cap;
};

// Launch shape of the shared-slab kernels: grid-stride over the queries with
// at most kSlabLanes lanes, each with a stack of cap entries of W words.
constexpr uint32_t kSlabLanes = 131072;
inline int32_t carried_stack(hipStream_t s, uint64_t n, int32_t max_stack, int words,
                             CarriedStack &cs, unsigned &grid) {
    const uint64_t need = (n + kTraceBlock - 1) / kTraceBlock;
    grid = (unsigned)std::min<uint64_t>(need, kSlabLanes / kTraceBlock);
    if (grid == 0) grid = 1;
    cs.lanes = grid * kTraceBlock;
    cs.cap = (uint32_t)(max_stack > 0 ? max_stack : 1) + 1u;
    const size_t ref_bytes = ((size_t)cs.lanes * cs.cap * 4 + 255) & ~(size_t)255;
    void *ws = nullptr;
    BVH_TRY(stream_workspace(s, kAreaTrace, ref_bytes + (size_t)cs.lanes * cs.cap * words * 4, &ws));
    cs.ref = static_cast<uint32_t *>(ws);
    cs.box = reinterpret_cast<float *>(static_cast<char *>(ws) + ref_bytes);
    return BVH_OK;
}
// Spill entries per lane of a persistent launch (beyond the LDS ring).
constexpr uint32_t kSpillCap = 64;

// Workgroups of a kernel resident on one CU at once: the runtime's occupancy
// figure, lowered so that the workgroups' static LDS stays strictly below the
// CU's capacity.  With the LDS of the runtime's figure filling the CU exactly
// (five 32 KiB workgroups in 160 KiB), a persistent grid of that size ran
// about a quarter slower than one a workgroup per CU smaller, as if the last
// workgroup of each CU started only once another had finished (the work
// dealt to it in advance then ends late).
inline int32_t blocks_per_cu(const void *kernel, int dev, int &per_cu) {
    BVH_HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kTraceBlock, 0));
    hipFuncAttributes attr;
    BVH_HIP_TRY(hipFuncGetAttributes(&attr, kernel));
    int lds_cu = 0;
    BVH_HIP_TRY(hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev));
    if (attr.sharedSizeBytes > 0 && lds_cu > 0) {
        const int cap = (int)((size_t)(lds_cu - 1) / attr.sharedSizeBytes);
        per_cu = per_cu < cap ? per_cu : cap;
    }
    if (per_cu < 1) per_cu = 1;
    return BVH_OK;
}

// Resident blocks of a kernel on the current device (cached per kernel).
template <typename K>
inline int32_t resident_blocks(K kernel, unsigned &blocks) {
    static std::mutex mu;
    static std::map<std::pair<const void *, int>, unsigned> cache;
    int dev = 0;
    BVH_HIP_TRY(hipGetDevice(&dev));
    const auto key = std::make_pair(reinterpret_cast<const void *>(kernel), dev);
    {
        std::lock_guard<std::mutex> lock(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            blocks = it->second;
            return BVH_OK;
        }
    }
    int per_cu = 0, n_cu = 0;
    BVH_TRY(blocks_per_cu(reinterpret_cast<const void *>(kernel), dev, per_cu));
    BVH_HIP_TRY(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
    blocks = (unsigned)per_cu * (unsigned)(n_cu > 0 ? n_cu : 1);
    std::lock_guard<std::mutex> lock(mu);
    cache[key] = blocks;
    return BVH_OK;
}

// Work area of one launch: the fallback header, list and deep stacks, then
// (persistent launches) the per-lane spill area.
struct TraceArea {
    Fallback fb;
    SpillArea sa;
};

inline int32_t trace_area(hipStream_t s, uint64_t n, uint32_t lanes, TraceArea &ta) {
    const size_t fb_bytes = (fallback_bytes(n) + 255) & ~(size_t)255;
    const size_t sp_bytes = (size_t)lanes * kSpillCap * 8;
    void *ws = nullptr;
    BVH_TRY(stream_workspace(s, kAreaTrace, fb_bytes + sp_bytes, &ws));
    ta.fb = fallback_view(ws, n);
    char *sp = static_cast<char *>(ws) + fb_bytes;
    ta.sa.ent = reinterpret_cast<uint2 *>(sp);
    ta.sa.lanes = lanes;
    ta.sa.cap = kSpillCap;
    BVH_HIP_TRY(hipMemsetAsync(ta.fb.count, 0, kFallbackHeaderBytes, s));
    return BVH_OK;
}

}  // namespace bvhlib
