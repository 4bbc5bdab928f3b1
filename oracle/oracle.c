/*
 * CPU oracle for closest-hit ray traversal of a triangle BVH.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU product path links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP library.
 *
 * What it computes (paper: "Decoupling Data Layouts from Bounding Volume
 * Hierarchies", PLDI 2026):
 *   - orc_mt_f32        ray/triangle test in FP32 (Moller-Trumbore, the test
 *                       of App. G, with App. G's acceptance intervals),
 *                       written from the 1997 vector formulation with fused
 *                       multiply-adds in a fixed order.
 *   - orc_mt_fixed      the same test of each ray against one given triangle
 *                       (checks a claimed hit without a search).
 *   - orc_brute_*       closest hit by exhaustive search over all triangles:
 *                       the plain definition of Fig. 4 / App. G closest_hit
 *                       (minimum t over every triangle the MT test accepts),
 *                       ties broken by lowest primitive id.
 *   - orc_bvh_*         a median-split BVH (top-down, largest-extent axis,
 *                       leaves of at most 4 triangles, the construction
 *                       pattern of Sec. 9.3.3 "Collision Detection") with a
 *                       scalar 64-entry stack traversal (Sec. 9.1) in three
 *                       modes: closest, top-2 (runner-up tracking for the
 *                       ambiguity mask) and any-hit.
 *   - orc_grad_f64      closed-form FP64 gradient of L = sum(w_t t + w_u u +
 *                       w_v v) with the hit primitive held fixed, from
 *                       implicit differentiation of the hit-point identity
 *                       o + t d = (1-u-v) p0 + u p1 + v p2 (App. G MT
 *                       parameterisation: u weights p1, v weights p2).
 *   - orc_tuv_f64       the same (t,u,v) at a fixed primitive in FP64, for
 *                       finite differences.
 *   - orc_sah_build     binned-SAH binary topology (32 bins, top-down,
 *                       Sec. 9.2.1), node list in preorder.
 *   - orc_*closest_point  closest-point query (App. G "Closest Point
 *                       Query"): the nearest triangle to a point within a
 *                       squared radius, its squared distance and the
 *                       barycentrics of the nearest point, in FP64, by
 *                       exhaustive search and through the median-split BVH;
 *                       orc_point_tri_f64 at fixed primitives.
 *
 * Parity status: every function here is pinned by the CPU test suite
 * (hand-built rays with exactly representable answers, FP64 linear solves,
 * brute force on small scenes, gradient identities and finite differences;
 * for the closest-point query: closed forms, the projection inequality,
 * dense sampling of the triangle, and BVH against exhaustive search).
 *
 * Build: gcc -O3 -fopenmp -ffp-contract=off (no FMA contraction: every FP32
 * product and sum rounds exactly as written; the fused multiply-adds of the
 * ray/triangle test are explicit fmaf calls, each correctly rounded).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* ------------------------------------------------------------------------ */
/* FP32 vector helpers.                                                      */
/* ------------------------------------------------------------------------ */
typedef struct { float x, y, z; } v3;

static inline v3 v3_load(const float *p) { v3 r = { p[0], p[1], p[2] }; return r; }
static inline v3 v3_sub(v3 a, v3 b) { v3 r = { a.x - b.x, a.y - b.y, a.z - b.z }; return r; }
/* a x b, each component as one product subtracted from a fused
 * multiply-add: x = fma(a.y, b.z, -(a.z b.y)), and cyclically. */
static inline v3 cross_fma(v3 a, v3 b) {
    v3 r;
    r.x = fmaf(a.y, b.z, -(a.z * b.y));
    r.y = fmaf(a.z, b.x, -(a.x * b.z));
    r.z = fmaf(a.x, b.y, -(a.y * b.x));
    return r;
}
/* a . b accumulated x, then y, then z: fma(a.z, b.z, fma(a.y, b.y, a.x b.x)). */
static inline float dot_fma(v3 a, v3 b) { return fmaf(a.z, b.z, fmaf(a.y, b.y, a.x * b.x)); }

static inline uint32_t f2u(float f) { uint32_t u; memcpy(&u, &f, 4); return u; }
static inline float u2f(uint32_t u) { float f; memcpy(&f, &u, 4); return f; }
/* x with the sign bit s (0 or 0x80000000) xor-ed in: x * (+-1), exactly. */
static inline float sign_xor(float x, uint32_t s) { return u2f(f2u(x) ^ s); }

/* ------------------------------------------------------------------------ */
/* Ray/triangle test (the intersection the paper's closest-hit search uses,  */
/* App. G, where it is Moller-Trumbore).  Written from Moller and Trumbore,  */
/* "Fast, Minimum Storage Ray/Triangle Intersection" (1997): with the edges   */
/* e1 = p1 - p0 and e2 = p2 - p0, the hit o + t d = p0 + u e1 + v e2 is a     */
/* 3x3 linear system whose Cramer solution shares two cross products,        */
/*   P = d x e2,  det = e1 . P,  S = o - p0,  Q = S x e1,                    */
/*   u det = S . P,   v det = d . Q,   t det = e2 . Q.                       */
/* Acceptance (App. G's intervals): u >= 0, v >= 0, u + v <= 1 (edges and     */
/* vertices count, both faces), and 0 < t <= tmax.  It is decided on the     */
/* numerators with the sign of det moved onto them (exact), against |det|,   */
/* so the single division happens only for an accepted hit:                 */
/*   t, u, v = (T, U, V) * (1 / |det|).                                       */
/* det = 0 (ray parallel to the plane, or a degenerate triangle) and a       */
/* non-finite det are misses.  Every product, sum and fused multiply-add is  */
/* a single correctly rounded FP32 operation in the order written.           */
/* Returns 1 on a hit and writes t, u, v.                                    */
/* ------------------------------------------------------------------------ */
static inline int mt_f32(v3 o, v3 d, float tmax, v3 p0, v3 p1, v3 p2,
                         float *t_out, float *u_out, float *v_out) {
    v3 e1 = v3_sub(p1, p0);
    v3 e2 = v3_sub(p2, p0);
    v3 P = cross_fma(d, e2);
    float det = dot_fma(e1, P);
    float adet = fabsf(det);
    if (!(adet > 0.0f && adet < INFINITY)) return 0;
    uint32_t s = f2u(det) & 0x80000000u;
    v3 S = v3_sub(o, p0);
    float U = sign_xor(dot_fma(S, P), s);
    v3 Q = cross_fma(S, e1);
    float V = sign_xor(dot_fma(d, Q), s);
    if (!(U >= 0.0f && V >= 0.0f && U + V <= adet)) return 0;
    float T = sign_xor(dot_fma(e2, Q), s);
    if (!(T > 0.0f && T <= adet * tmax)) return 0;
    float inv = 1.0f / adet;
    *t_out = T * inv;
    *u_out = U * inv;
    *v_out = V * inv;
    return 1;
}

int orc_mt_f32(const float *o, const float *d, float tmax, const float *p0,
               const float *p1, const float *p2, float *tuv) {
    float t, u, v;
    int hit = mt_f32(v3_load(o), v3_load(d), tmax, v3_load(p0), v3_load(p1),
                     v3_load(p2), &t, &u, &v);
    if (hit) { tuv[0] = t; tuv[1] = u; tuv[2] = v; }
    return hit;
}

/* Ray record: o.xyz, tmin, d.xyz, tmax (8 floats).  tmin must be 0: the MT
 * acceptance is the strict 0 < t of App. G. */
#define RAY_STRIDE 8

static inline void tri_fetch(const float *verts, const int32_t *tris, int64_t i,
                             v3 *p0, v3 *p1, v3 *p2) {
    *p0 = v3_load(verts + 3 * (int64_t)tris[3 * i + 0]);
    *p1 = v3_load(verts + 3 * (int64_t)tris[3 * i + 1]);
    *p2 = v3_load(verts + 3 * (int64_t)tris[3 * i + 2]);
}

/* (t, id) lexicographic order: lower t wins, then lower id. */
static inline int lex_less(float ta, int32_t ia, float tb, int32_t ib) {
    return ta < tb || (ta == tb && ia < ib);
}

/* ------------------------------------------------------------------------ */
/* Brute force (the plain definition).                                       */
/* out_prim[n], out_tuv[n*3]; a miss is prim -1, t +inf, u = v = 0.         */
/* ------------------------------------------------------------------------ */
void orc_brute_closest(const float *verts, const int32_t *tris, int64_t ntris,
                       const float *rays, int64_t nrays, int32_t *out_prim,
                       float *out_tuv, int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < nrays; r++) {
        const float *ray = rays + RAY_STRIDE * r;
        v3 o = v3_load(ray), d = v3_load(ray + 4);
        float tmax = ray[7];
        int32_t best = -1;
        float bt = INFINITY, bu = 0.0f, bv = 0.0f;
        for (int64_t i = 0; i < ntris; i++) {
            v3 p0, p1, p2;
            tri_fetch(verts, tris, i, &p0, &p1, &p2);
            float t, u, v;
            if (mt_f32(o, d, tmax, p0, p1, p2, &t, &u, &v) &&
                lex_less(t, (int32_t)i, bt, best < 0 ? INT32_MAX : best)) {
                best = (int32_t)i; bt = t; bu = u; bv = v;
            }
        }
        out_prim[r] = best;
        out_tuv[3 * r + 0] = bt;
        out_tuv[3 * r + 1] = bu;
        out_tuv[3 * r + 2] = bv;
    }
}

/* The ray/triangle test of every ray against one given triangle
 * (prims[r]; a negative id is a miss): out_hit[r] = 1 and out_tuv[r] = (t,
 * u, v) where mt_f32 accepts, else out_hit[r] = 0 and out_tuv[r] = (inf, 0,
 * 0).  Checks a claimed hit without a search. */
void orc_mt_fixed(const float *verts, const int32_t *tris, int64_t ntris,
                  const float *rays, int64_t nrays, const int32_t *prims,
                  float *out_tuv, int32_t *out_hit) {
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nrays; r++) {
        const float *ray = rays + RAY_STRIDE * r;
        float t = INFINITY, u = 0.0f, v = 0.0f;
        int hit = 0;
        if (prims[r] >= 0 && prims[r] < ntris) {
            v3 p0, p1, p2;
            tri_fetch(verts, tris, prims[r], &p0, &p1, &p2);
            hit = mt_f32(v3_load(ray), v3_load(ray + 4), ray[7], p0, p1, p2, &t, &u, &v);
            if (!hit) { t = INFINITY; u = 0.0f; v = 0.0f; }
        }
        out_hit[r] = hit;
        out_tuv[3 * r + 0] = t;
        out_tuv[3 * r + 1] = u;
        out_tuv[3 * r + 2] = v;
    }
}

/* Best and runner-up over distinct primitives, by brute force.
 * out[n*2] prims (second = -1 if none), out_t[n*2]. */
void orc_brute_top2(const float *verts, const int32_t *tris, int64_t ntris,
                    const float *rays, int64_t nrays, int32_t *out_prim,
                    float *out_t, int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < nrays; r++) {
        const float *ray = rays + RAY_STRIDE * r;
        v3 o = v3_load(ray), d = v3_load(ray + 4);
        float tmax = ray[7];
        int32_t i1 = -1, i2 = -1;
        float t1 = INFINITY, t2 = INFINITY;
        for (int64_t i = 0; i < ntris; i++) {
            v3 p0, p1, p2;
            tri_fetch(verts, tris, i, &p0, &p1, &p2);
            float t, u, v;
            if (!mt_f32(o, d, tmax, p0, p1, p2, &t, &u, &v)) continue;
            int32_t id = (int32_t)i;
            if (lex_less(t, id, t1, i1 < 0 ? INT32_MAX : i1)) {
                t2 = t1; i2 = i1; t1 = t; i1 = id;
            } else if (lex_less(t, id, t2, i2 < 0 ? INT32_MAX : i2)) {
                t2 = t; i2 = id;
            }
        }
        out_prim[2 * r + 0] = i1; out_prim[2 * r + 1] = i2;
        out_t[2 * r + 0] = t1;    out_t[2 * r + 1] = t2;
    }
}

/* ------------------------------------------------------------------------ */
/* Median-split BVH.                                                         */
/* ------------------------------------------------------------------------ */
#define ORC_LEAF_MAX 4
#define ORC_STACK 64

typedef struct {
    float lo[3], hi[3];
    int32_t left, right;   /* child node indices; -1 for a leaf */
    int32_t first, count;  /* leaf: range into perm[] */
} orc_node;

typedef struct {
    orc_node *nodes;
    int32_t nnodes, cap;
    int32_t *perm;         /* triangle ids in leaf order */
    int64_t ntris;
    int32_t depth;
    const float *verts;    /* borrowed */
    const int32_t *tris;   /* borrowed */
    float *centroid;       /* 3 per triangle */
} orc_bvh;

static int32_t new_node(orc_bvh *b) {
    if (b->nnodes == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 1024;
        b->nodes = (orc_node *)realloc(b->nodes, (size_t)b->cap * sizeof(orc_node));
    }
    return b->nnodes++;
}

/* Order key for the median split: centroid on the axis, then triangle id. */
static inline int key_less(const orc_bvh *b, int axis, int32_t x, int32_t y) {
    float cx = b->centroid[3 * (int64_t)x + axis], cy = b->centroid[3 * (int64_t)y + axis];
    return cx < cy || (cx == cy && x < y);
}

/* Quickselect: after the call perm[lo..k) <= perm[k] <= perm(k..hi) in key order. */
static void select_kth(orc_bvh *b, int axis, int32_t *a, int64_t lo, int64_t hi, int64_t k) {
    while (hi - lo > 1) {
        int64_t mid = lo + (hi - lo) / 2;
        /* median of three as pivot */
        int32_t x = a[lo], y = a[mid], z = a[hi - 1], piv;
        if (key_less(b, axis, x, y)) {
            if (key_less(b, axis, y, z)) piv = y;
            else if (key_less(b, axis, x, z)) piv = z;
            else piv = x;
        } else {
            if (key_less(b, axis, x, z)) piv = x;
            else if (key_less(b, axis, y, z)) piv = z;
            else piv = y;
        }
        /* three-way partition: [lo,lt) < piv, [lt,gt) == piv, [gt,hi) > piv */
        int64_t lt = lo, i = lo, gt = hi;
        while (i < gt) {
            if (key_less(b, axis, a[i], piv)) { int32_t t = a[lt]; a[lt] = a[i]; a[i] = t; lt++; i++; }
            else if (key_less(b, axis, piv, a[i])) { gt--; int32_t t = a[gt]; a[gt] = a[i]; a[i] = t; }
            else i++;
        }
        if (k < lt) hi = lt;
        else if (k >= gt) lo = gt;
        else return;
    }
}

static void node_bounds(orc_bvh *b, orc_node *n, int64_t first, int64_t count) {
    for (int a = 0; a < 3; a++) { n->lo[a] = INFINITY; n->hi[a] = -INFINITY; }
    for (int64_t i = first; i < first + count; i++) {
        int32_t t = b->perm[i];
        for (int k = 0; k < 3; k++) {
            const float *p = b->verts + 3 * (int64_t)b->tris[3 * (int64_t)t + k];
            for (int a = 0; a < 3; a++) {
                if (p[a] < n->lo[a]) n->lo[a] = p[a];
                if (p[a] > n->hi[a]) n->hi[a] = p[a];
            }
        }
    }
}

static int32_t build_rec(orc_bvh *b, int64_t first, int64_t count, int32_t depth) {
    int32_t id = new_node(b);
    if (depth > b->depth) b->depth = depth;
    orc_node *n = &b->nodes[id];
    node_bounds(b, n, first, count);
    if (count <= ORC_LEAF_MAX) {
        n->left = n->right = -1;
        n->first = (int32_t)first;
        n->count = (int32_t)count;
        return id;
    }
    /* split axis: largest extent of the centroid bounds (lowest axis on ties) */
    float clo[3] = { INFINITY, INFINITY, INFINITY }, chi[3] = { -INFINITY, -INFINITY, -INFINITY };
    for (int64_t i = first; i < first + count; i++) {
        const float *c = b->centroid + 3 * (int64_t)b->perm[i];
        for (int a = 0; a < 3; a++) {
            if (c[a] < clo[a]) clo[a] = c[a];
            if (c[a] > chi[a]) chi[a] = c[a];
        }
    }
    int axis = 0;
    for (int a = 1; a < 3; a++)
        if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
    int64_t half = count / 2;
    select_kth(b, axis, b->perm, first, first + count, first + half);
    int32_t l = build_rec(b, first, half, depth + 1);
    int32_t r = build_rec(b, first + half, count - half, depth + 1);
    n = &b->nodes[id]; /* nodes may have moved */
    n->left = l; n->right = r; n->first = (int32_t)first; n->count = (int32_t)count;
    return id;
}

void *orc_bvh_build(const float *verts, const int32_t *tris, int64_t ntris) {
    orc_bvh *b = (orc_bvh *)calloc(1, sizeof(orc_bvh));
    b->verts = verts; b->tris = tris; b->ntris = ntris;
    b->perm = (int32_t *)malloc((size_t)(ntris > 0 ? ntris : 1) * sizeof(int32_t));
    b->centroid = (float *)malloc((size_t)(ntris > 0 ? ntris : 1) * 3 * sizeof(float));
    for (int64_t i = 0; i < ntris; i++) {
        b->perm[i] = (int32_t)i;
        for (int a = 0; a < 3; a++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += verts[3 * (int64_t)tris[3 * i + k] + a];
            b->centroid[3 * i + a] = (float)(s / 3.0);
        }
    }
    if (ntris > 0) build_rec(b, 0, ntris, 1);
    return b;
}

void orc_bvh_free(void *h) {
    orc_bvh *b = (orc_bvh *)h;
    if (!b) return;
    free(b->nodes); free(b->perm); free(b->centroid); free(b);
}

int32_t orc_bvh_depth(void *h) { return ((orc_bvh *)h)->depth; }
int32_t orc_bvh_nnodes(void *h) { return ((orc_bvh *)h)->nnodes; }

/* Copies node records out for structural tests: per node 6 floats (lo, hi) and
 * 4 ints (left, right, first, count); perm (leaf order) as well. */
void orc_bvh_export(void *h, float *boxes, int32_t *links, int32_t *perm) {
    orc_bvh *b = (orc_bvh *)h;
    for (int32_t i = 0; i < b->nnodes; i++) {
        for (int a = 0; a < 3; a++) { boxes[6 * i + a] = b->nodes[i].lo[a]; boxes[6 * i + 3 + a] = b->nodes[i].hi[a]; }
        links[4 * i + 0] = b->nodes[i].left;  links[4 * i + 1] = b->nodes[i].right;
        links[4 * i + 2] = b->nodes[i].first; links[4 * i + 3] = b->nodes[i].count;
    }
    memcpy(perm, b->perm, (size_t)b->ntris * sizeof(int32_t));
}

/* Conservative slab-test widening: the far distance is scaled by 1 + 2^-21,
 * which exceeds 1 + 2*gamma_3 (gamma_3 = 3u/(1-3u), u = 2^-24), the bound on
 * the relative rounding error of the three-operation slab distance (Ize 2013,
 * "Robust BVH Ray Traversal").  Hence a box that the exact ray meets before
 * the current best distance is never culled. */
#define ORC_FAR_SCALE 1.000000476837158203125f

/* Ray/box test on a node's box with the node cull folded in (the slab     */
/* method of Kay and Kajiya 1986; planes ordered by the sign of d as in      */
/* Williams et al. 2005).  Along axis a the ray lies between the box's two   */
/* planes for t between its distance to the plane it crosses first and the   */
/* plane it crosses last, (plane - o) * (1/d); which plane comes first        */
/* follows the sign bit of d, so d = -0 (1/d = -inf) pairs with the upper     */
/* plane.  The box is visited when the largest entry distance, at least 0,   */
/* does not exceed the smallest exit distance, at most tcur, widened by      */
/* ORC_FAR_SCALE.  fmaxf/fminf ignore the NaN of 0 * inf (a ray lying in a   */
/* slab plane), so such an axis culls nothing.                               */
static inline int slab(v3 o, v3 rd, const int neg[3], const orc_node *n, float tcur) {
    const float *ov = &o.x, *rv = &rd.x;
    float enter = 0.0f, leave = tcur;
    for (int a = 0; a < 3; a++) {
        float first = neg[a] ? n->hi[a] : n->lo[a];
        float last = neg[a] ? n->lo[a] : n->hi[a];
        enter = fmaxf(enter, (first - ov[a]) * rv[a]);
        leave = fminf(leave, (last - ov[a]) * rv[a]);
    }
    return enter <= leave * ORC_FAR_SCALE;
}

enum { ORC_CLOSEST = 0, ORC_TOP2 = 1, ORC_ANY = 2 };

/* Traces one ray.  Closest: (i1, t1, u1, v1).  Top-2 additionally (i2, t2),
 * culling with the runner-up distance.  Any: the first accepted hit. */
static void trace_one(const orc_bvh *b, const float *ray, int mode, int32_t *i1o,
                      float *tuv1, int32_t *i2o, float *t2o) {
    v3 o = v3_load(ray), d = v3_load(ray + 4);
    float tmax = ray[7];
    v3 rd = { 1.0f / d.x, 1.0f / d.y, 1.0f / d.z };
    int neg[3] = { signbit(d.x) != 0, signbit(d.y) != 0, signbit(d.z) != 0 };
    int32_t i1 = -1, i2 = -1;
    float t1 = INFINITY, u1 = 0.0f, v1 = 0.0f, t2 = INFINITY;
    int32_t stack[ORC_STACK];
    int sp = 0;
    if (b->nnodes > 0) stack[sp++] = 0;
    while (sp > 0) {
        const orc_node *n = &b->nodes[stack[--sp]];
        float tcur = (mode == ORC_TOP2) ? t2 : (mode == ORC_CLOSEST ? t1 : tmax);
        if (mode == ORC_CLOSEST && tmax < tcur) tcur = tmax;
        if (mode == ORC_TOP2 && tmax < tcur) tcur = tmax;
        if (!slab(o, rd, neg, n, tcur)) continue;
        if (n->left < 0) {
            for (int32_t k = n->first; k < n->first + n->count; k++) {
                int32_t id = b->perm[k];
                v3 p0, p1, p2;
                tri_fetch(b->verts, b->tris, id, &p0, &p1, &p2);
                float t, u, v;
                if (!mt_f32(o, d, tmax, p0, p1, p2, &t, &u, &v)) continue;
                if (mode == ORC_ANY) {
                    *i1o = id; tuv1[0] = t; tuv1[1] = u; tuv1[2] = v;
                    return;
                }
                if (lex_less(t, id, t1, i1 < 0 ? INT32_MAX : i1)) {
                    t2 = t1; i2 = i1;
                    t1 = t; u1 = u; v1 = v; i1 = id;
                } else if (lex_less(t, id, t2, i2 < 0 ? INT32_MAX : i2)) {
                    t2 = t; i2 = id;
                }
            }
        } else {
            /* both children pushed; the order cannot change the result */
            stack[sp++] = n->right;
            stack[sp++] = n->left;
        }
    }
    *i1o = i1; tuv1[0] = t1; tuv1[1] = u1; tuv1[2] = v1;
    if (i2o) { *i2o = i2; *t2o = t2; }
}

/* mode: 0 closest, 1 top-2, 2 any-hit.  out_prim2/out_t2 only for top-2 (may
 * be NULL otherwise).  nthreads <= 0 keeps the OpenMP default. */
void orc_bvh_trace(void *h, const float *rays, int64_t nrays, int mode,
                   int32_t *out_prim, float *out_tuv, int32_t *out_prim2,
                   float *out_t2, int nthreads) {
    const orc_bvh *b = (const orc_bvh *)h;
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < nrays; r++) {
        int32_t i2 = -1;
        float t2 = INFINITY;
        trace_one(b, rays + RAY_STRIDE * r, mode, &out_prim[r], &out_tuv[3 * r],
                  &i2, &t2);
        if (mode == ORC_TOP2) { out_prim2[r] = i2; out_t2[r] = t2; }
    }
}

int orc_max_threads(void) { return omp_get_max_threads(); }

/* ------------------------------------------------------------------------ */
/* FP64 hit parameters and gradient at a fixed primitive.                    */
/* The hit point satisfies F = o + t d - p0 - u (p1 - p0) - v (p2 - p0) = 0. */
/* dF/d(t,u,v) = J = [d | p0-p1 | p0-p2] (columns).  For L with gradient     */
/* g = dL/d(t,u,v), solve J^T lam = g; then dL/dx = -lam^T dF/dx:            */
/*   dL/do = -lam, dL/dd = -t lam, dL/dp0 = (1-u-v) lam,                     */
/*   dL/dp1 = u lam, dL/dp2 = v lam.                                         */
/* ------------------------------------------------------------------------ */
typedef struct { double x, y, z; } d3;
static inline d3 d3_load(const float *p) { d3 r = { p[0], p[1], p[2] }; return r; }
static inline d3 d3_sub(d3 a, d3 b) { d3 r = { a.x - b.x, a.y - b.y, a.z - b.z }; return r; }
static inline d3 d3_cross(d3 a, d3 b) {
    d3 r = { a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x };
    return r;
}
static inline double d3_dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }

/* Solves J (t,u,v) = p0 - o by Cramer's rule with J = [d | p0-p1 | p0-p2].
 * Returns 0 when the system is singular (ray parallel to the plane). */
static int tuv_f64(d3 o, d3 d, d3 p0, d3 p1, d3 p2, double *t, double *u, double *v) {
    d3 a = d, b = d3_sub(p0, p1), c = d3_sub(p0, p2), rhs = d3_sub(p0, o);
    double det = d3_dot(a, d3_cross(b, c));
    if (det == 0.0) return 0;
    *t = d3_dot(rhs, d3_cross(b, c)) / det;
    *u = d3_dot(a, d3_cross(rhs, c)) / det;
    *v = d3_dot(a, d3_cross(b, rhs)) / det;
    return 1;
}

/* (t,u,v) in FP64 for rays[i] against prims[i] (prims[i] < 0 gives NaNs). */
void orc_tuv_f64(const double *verts, const int32_t *tris, const double *rays,
                 const int32_t *prims, int64_t n, double *out) {
    for (int64_t i = 0; i < n; i++) {
        out[3 * i] = out[3 * i + 1] = out[3 * i + 2] = NAN;
        if (prims[i] < 0) continue;
        const int32_t *tr = tris + 3 * (int64_t)prims[i];
        d3 p0 = { verts[3 * (int64_t)tr[0]], verts[3 * (int64_t)tr[0] + 1], verts[3 * (int64_t)tr[0] + 2] };
        d3 p1 = { verts[3 * (int64_t)tr[1]], verts[3 * (int64_t)tr[1] + 1], verts[3 * (int64_t)tr[1] + 2] };
        d3 p2 = { verts[3 * (int64_t)tr[2]], verts[3 * (int64_t)tr[2] + 1], verts[3 * (int64_t)tr[2] + 2] };
        const double *ry = rays + 8 * i;
        d3 o = { ry[0], ry[1], ry[2] }, d = { ry[4], ry[5], ry[6] };
        tuv_f64(o, d, p0, p1, p2, &out[3 * i], &out[3 * i + 1], &out[3 * i + 2]);
    }
}

/* Gradient of L = sum_i g_i . (t_i, u_i, v_i) at fixed prims.
 * grad_verts (nverts*3) is accumulated (+=), grad_rays (n*6: dL/do, dL/dd) is
 * overwritten, tuv (n*3) receives the hit parameters used.  lam depends only
 * on d and the triangle; the hit parameters enter through the weights
 * (1-u-v, u, v) and dL/dd = -t lam.  With tuv_at == NULL they are solved in
 * FP64; otherwise they are taken from tuv_at (n*3, e.g. the FP32 forward's
 * own hit), so the gradient is evaluated at that forward result. */
void orc_grad_f64(const float *verts, const int32_t *tris, const float *rays,
                  const int32_t *prims, const float *grad_hits, int64_t n,
                  double *grad_verts, double *grad_rays, double *tuv,
                  const float *tuv_at) {
    for (int64_t i = 0; i < n; i++) {
        double *gr = grad_rays + 6 * i;
        for (int k = 0; k < 6; k++) gr[k] = 0.0;
        tuv[3 * i] = tuv[3 * i + 1] = tuv[3 * i + 2] = NAN;
        if (prims[i] < 0) continue;
        const int32_t *tr = tris + 3 * (int64_t)prims[i];
        d3 p0 = d3_load(verts + 3 * (int64_t)tr[0]);
        d3 p1 = d3_load(verts + 3 * (int64_t)tr[1]);
        d3 p2 = d3_load(verts + 3 * (int64_t)tr[2]);
        const float *ry = rays + RAY_STRIDE * i;
        d3 o = d3_load(ry), d = d3_load(ry + 4);
        double t, u, v;
        if (!tuv_f64(o, d, p0, p1, p2, &t, &u, &v)) continue;
        if (tuv_at) { t = tuv_at[3 * i]; u = tuv_at[3 * i + 1]; v = tuv_at[3 * i + 2]; }
        tuv[3 * i] = t; tuv[3 * i + 1] = u; tuv[3 * i + 2] = v;
        /* J^T lam = g: rows of J^T are a = d, b = p0-p1, c = p0-p2.
         * lam = (g_t (b x c) + g_u (c x a) + g_v (a x b)) / (a . (b x c)). */
        d3 a = d, b = d3_sub(p0, p1), c = d3_sub(p0, p2);
        d3 bc = d3_cross(b, c), ca = d3_cross(c, a), ab = d3_cross(a, b);
        double det = d3_dot(a, bc);
        double gt = grad_hits[3 * i], gu = grad_hits[3 * i + 1], gv = grad_hits[3 * i + 2];
        d3 lam = { (gt * bc.x + gu * ca.x + gv * ab.x) / det,
                   (gt * bc.y + gu * ca.y + gv * ab.y) / det,
                   (gt * bc.z + gu * ca.z + gv * ab.z) / det };
        gr[0] = -lam.x; gr[1] = -lam.y; gr[2] = -lam.z;
        gr[3] = -t * lam.x; gr[4] = -t * lam.y; gr[5] = -t * lam.z;
        double w[3] = { 1.0 - u - v, u, v };
        for (int k = 0; k < 3; k++) {
            double *gv3 = grad_verts + 3 * (int64_t)tr[k];
            gv3[0] += w[k] * lam.x; gv3[1] += w[k] * lam.y; gv3[2] += w[k] * lam.z;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Closest-point query (App. G "Closest Point Query"; Sec. 9.3.2 evaluates  */
/* it on the same layouts as ray traversal).                                 */
/*                                                                           */
/* The plain definition: for a query point q with squared search radius r2,  */
/* the triangle at the smallest squared Euclidean distance from q (each      */
/* triangle a closed set, edges and vertices included), ties to the lowest   */
/* id, among the triangles with distance^2 <= r2; with the squared distance  */
/* and the barycentrics (u weights p1, v weights p2, as for hits) of the     */
/* nearest point of that triangle.                                           */
/*                                                                           */
/* Distances are computed in FP64 from the f32 inputs by a method of its own */
/* rather than the Voronoi-region case analysis the paper's listing uses    */
/* (Ericson, Real-Time Collision Detection, 5.1.5): the squared distance    */
/* from q to p0 + u e1 + v e2 is a convex quadratic in (u, v), so over the   */
/* triangle it is minimal either at its stationary point (the solution of   */
/* the 2x2 normal equations, when that lies inside) or on the boundary,     */
/* where each edge is a segment with a clamped projection.  The minimum over */
/* these at most four candidates, each an actual point of the triangle, is  */
/* the distance.  Degenerate triangles (a singular 2x2 system) reduce to    */
/* their edges.                                                              */
/* ------------------------------------------------------------------------ */
#define QUERY_STRIDE 4 /* x, y, z, r2 */

static inline void cp_consider(d3 q, d3 p0, d3 e1, d3 e2, double u, double v,
                               double *bd2, double *bu, double *bv) {
    d3 c = { p0.x + u * e1.x + v * e2.x, p0.y + u * e1.y + v * e2.y,
             p0.z + u * e1.z + v * e2.z };
    d3 w = d3_sub(q, c);
    double d2 = d3_dot(w, w);
    if (d2 < *bd2) { *bd2 = d2; *bu = u; *bv = v; }
}

/* Parameter s in [0, 1] of the point of segment a + s (b - a) nearest to q. */
static inline double seg_param(d3 q, d3 a, d3 b) {
    d3 ab = d3_sub(b, a);
    double len2 = d3_dot(ab, ab);
    if (len2 == 0.0) return 0.0;
    double s = d3_dot(d3_sub(q, a), ab) / len2;
    return s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
}

static void cp_tri_f64(d3 q, d3 p0, d3 p1, d3 p2, double *d2, double *u, double *v) {
    d3 e1 = d3_sub(p1, p0), e2 = d3_sub(p2, p0), w = d3_sub(q, p0);
    double bd2 = INFINITY, bu = 0.0, bv = 0.0;
    /* stationary point: [e1.e1 e1.e2; e1.e2 e2.e2] (u, v) = (e1.w, e2.w) */
    double a = d3_dot(e1, e1), b = d3_dot(e1, e2), c = d3_dot(e2, e2);
    double r1 = d3_dot(e1, w), r2 = d3_dot(e2, w);
    double det = a * c - b * b;
    if (det > 0.0) {
        double s = (c * r1 - b * r2) / det, t = (a * r2 - b * r1) / det;
        if (s >= 0.0 && t >= 0.0 && s + t <= 1.0) cp_consider(q, p0, e1, e2, s, t, &bd2, &bu, &bv);
    }
    /* edges: p0p1 (v = 0), p0p2 (u = 0), p1p2 (u + v = 1) */
    double s01 = seg_param(q, p0, p1), s02 = seg_param(q, p0, p2), s12 = seg_param(q, p1, p2);
    cp_consider(q, p0, e1, e2, s01, 0.0, &bd2, &bu, &bv);
    cp_consider(q, p0, e1, e2, 0.0, s02, &bd2, &bu, &bv);
    cp_consider(q, p0, e1, e2, 1.0 - s12, s12, &bd2, &bu, &bv);
    *d2 = bd2; *u = bu; *v = bv;
}

static inline void tri_fetch_f64(const float *verts, const int32_t *tris, int64_t i,
                                 d3 *p0, d3 *p1, d3 *p2) {
    const int32_t *t = tris + 3 * i;
    *p0 = d3_load(verts + 3 * (int64_t)t[0]);
    *p1 = d3_load(verts + 3 * (int64_t)t[1]);
    *p2 = d3_load(verts + 3 * (int64_t)t[2]);
}

static inline int lex_less_d(double da, int32_t ia, double db, int32_t ib) {
    return da < db || (da == db && ia < ib);
}

/* (d2, u, v) of queries[i] against prims[i]; prims[i] < 0 gives (inf, 0, 0). */
void orc_point_tri_f64(const float *verts, const int32_t *tris, const float *queries,
                       const int32_t *prims, int64_t n, double *out) {
    for (int64_t i = 0; i < n; i++) {
        out[3 * i] = INFINITY; out[3 * i + 1] = out[3 * i + 2] = 0.0;
        if (prims[i] < 0) continue;
        d3 p0, p1, p2, q = d3_load(queries + QUERY_STRIDE * i);
        tri_fetch_f64(verts, tris, prims[i], &p0, &p1, &p2);
        cp_tri_f64(q, p0, p1, p2, &out[3 * i], &out[3 * i + 1], &out[3 * i + 2]);
    }
}

/* Top-2 bookkeeping over distinct primitives, (d2, id) lexicographic. */
typedef struct { int32_t i1, i2; double d1, u1, v1, d2; } cp_top2;

static inline void cp_top2_add(cp_top2 *b, int32_t id, double d2, double u, double v) {
    if (lex_less_d(d2, id, b->d1, b->i1 < 0 ? INT32_MAX : b->i1)) {
        b->i2 = b->i1; b->d2 = b->d1;
        b->i1 = id; b->d1 = d2; b->u1 = u; b->v1 = v;
    } else if (lex_less_d(d2, id, b->d2, b->i2 < 0 ? INT32_MAX : b->i2)) {
        b->i2 = id; b->d2 = d2;
    }
}

/* Writes the query's result: the nearest triangle if within r2 (else -1,
 * inf, 0, 0), and the unrestricted nearest and runner-up (for grading). */
static inline void cp_store(const cp_top2 *b, float r2, int64_t i, int32_t *out_prim,
                            double *out_duv, int32_t *out_top2, double *out_d2top2) {
    int in = b->i1 >= 0 && b->d1 <= (double)r2;
    out_prim[i] = in ? b->i1 : -1;
    out_duv[3 * i] = in ? b->d1 : INFINITY;
    out_duv[3 * i + 1] = in ? b->u1 : 0.0;
    out_duv[3 * i + 2] = in ? b->v1 : 0.0;
    if (out_top2) {
        out_top2[2 * i] = b->i1; out_top2[2 * i + 1] = b->i2;
        out_d2top2[2 * i] = b->d1; out_d2top2[2 * i + 1] = b->d2;
    }
}

/* Exhaustive search: queries n x (x, y, z, r2); out_prim[n], out_duv[n*3]
 * (d2, u, v); out_top2[n*2] / out_d2top2[n*2] (may be NULL) the nearest and
 * runner-up over all triangles regardless of r2 (-1 / inf when absent). */
void orc_brute_closest_point(const float *verts, const int32_t *tris, int64_t ntris,
                             const float *queries, int64_t n, int32_t *out_prim,
                             double *out_duv, int32_t *out_top2, double *out_d2top2,
                             int nthreads) {
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        const float *qp = queries + QUERY_STRIDE * i;
        d3 q = d3_load(qp);
        cp_top2 b = { -1, -1, INFINITY, 0.0, 0.0, INFINITY };
        for (int64_t k = 0; k < ntris; k++) {
            d3 p0, p1, p2;
            tri_fetch_f64(verts, tris, k, &p0, &p1, &p2);
            double d2, u, v;
            cp_tri_f64(q, p0, p1, p2, &d2, &u, &v);
            cp_top2_add(&b, (int32_t)k, d2, u, v);
        }
        cp_store(&b, qp[3], i, out_prim, out_duv, out_top2, out_d2top2);
    }
}

/* Squared distance from q to a node box in FP64. */
static inline double box_d2(d3 q, const orc_node *nd) {
    const double qq[3] = { q.x, q.y, q.z };
    double s = 0.0;
    for (int a = 0; a < 3; a++) {
        double g = 0.0;
        if (qq[a] < nd->lo[a]) g = nd->lo[a] - qq[a];
        else if (qq[a] > nd->hi[a]) g = qq[a] - nd->hi[a];
        s += g * g;
    }
    return s;
}

/* The same result through the median-split BVH.  A node is skipped only when
 * its box distance exceeds the runner-up distance by a margin that covers
 * the FP64 rounding of both distances (2^-30 relative plus 2^-50 S^2, S the
 * largest coordinate magnitude of the scene and the query), so the search
 * returns what the exhaustive one does. */
void orc_bvh_closest_point(void *h, const float *queries, int64_t n, int32_t *out_prim,
                           double *out_duv, int32_t *out_top2, double *out_d2top2,
                           int nthreads) {
    const orc_bvh *bv = (const orc_bvh *)h;
    double smax = 0.0; /* the root box bounds every vertex */
    if (bv->nnodes > 0)
        for (int a = 0; a < 3; a++) {
            if (fabs(bv->nodes[0].lo[a]) > smax) smax = fabs(bv->nodes[0].lo[a]);
            if (fabs(bv->nodes[0].hi[a]) > smax) smax = fabs(bv->nodes[0].hi[a]);
        }
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
        const float *qp = queries + QUERY_STRIDE * i;
        d3 q = d3_load(qp);
        double s = smax;
        if (fabs(q.x) > s) s = fabs(q.x);
        if (fabs(q.y) > s) s = fabs(q.y);
        if (fabs(q.z) > s) s = fabs(q.z);
        const double abs_margin = ldexp(s * s, -50);
        cp_top2 b = { -1, -1, INFINITY, 0.0, 0.0, INFINITY };
        int32_t stack[ORC_STACK];
        int sp = 0;
        if (bv->nnodes > 0) stack[sp++] = 0;
        while (sp > 0) {
            const orc_node *nd = &bv->nodes[stack[--sp]];
            double bound = b.d2 + ldexp(b.d2, -30) + abs_margin;
            if (box_d2(q, nd) > bound) continue;
            if (nd->left < 0) {
                for (int32_t k = nd->first; k < nd->first + nd->count; k++) {
                    int32_t id = bv->perm[k];
                    d3 p0, p1, p2;
                    tri_fetch_f64(bv->verts, bv->tris, id, &p0, &p1, &p2);
                    double d2, u, v;
                    cp_tri_f64(q, p0, p1, p2, &d2, &u, &v);
                    cp_top2_add(&b, id, d2, u, v);
                }
            } else {
                /* nearer child on top; the order cannot change the result */
                double dl = box_d2(q, &bv->nodes[nd->left]), dr = box_d2(q, &bv->nodes[nd->right]);
                if (dl <= dr) { stack[sp++] = nd->right; stack[sp++] = nd->left; }
                else { stack[sp++] = nd->left; stack[sp++] = nd->right; }
            }
        }
        cp_store(&b, qp[3], i, out_prim, out_duv, out_top2, out_d2top2);
    }
}

/* ------------------------------------------------------------------------ */
/* Binned SAH topology (Sec. 9.2.1: trees built by top-down recursive        */
/* partitioning into two, each split chosen by the surface area heuristic    */
/* over 32 bins, after Wald 2007; the same construction as the closest-point */
/* comparison of Sec. 9.3.2, which bins along each axis and sweeps for the  */
/* cheapest partition).  Readings where the paper gives no detail:          */
/*   - a primitive's box is the exact f32 box of its vertices and its       */
/*     centroid c = 0.5 lo + 0.5 hi (f32);                                   */
/*   - a node bins along each axis over the exact bounds [cl, ch] of its    */
/*     primitives' centroids: an axis with ch - cl not positive and finite  */
/*     is skipped; otherwise s = 32 / (ch - cl) and the bin of c is          */
/*     min(31, trunc((c - cl) * s)), all in f32;                             */
/*   - the split after bin k (k = 0..30) costs A(L) N(L) + A(R) N(R) in f32, */
/*     A = dx dy + dy dz + dz dx of the union box of a side (half the        */
/*     surface area; the constant factors of the heuristic do not move the  */
/*     minimum), valid when both sides are non-empty; the cheapest valid     */
/*     split wins, ties to the lower axis, then the lower k;                 */
/*   - with no valid split (all centroids coincide) the first floor(N/2)     */
/*     primitives in the current order go left (axis recorded as 0);         */
/*   - partitions are stable (each side keeps the parent's order) and the    */
/*     initial order is by primitive id;                                     */
/*   - splitting continues down to single primitives: the layouts' leaves    */
/*     are then the subtrees of at most leaf_size primitives.                */
/* ------------------------------------------------------------------------ */
#define SAH_BINS 32

typedef struct { float lo[3], hi[3]; } fbox;

static inline void fbox_empty(fbox *b) {
    for (int a = 0; a < 3; a++) { b->lo[a] = INFINITY; b->hi[a] = -INFINITY; }
}
static inline void fbox_grow(fbox *b, const fbox *x) {
    for (int a = 0; a < 3; a++) {
        if (x->lo[a] < b->lo[a]) b->lo[a] = x->lo[a];
        if (x->hi[a] > b->hi[a]) b->hi[a] = x->hi[a];
    }
}
static inline float half_area(const fbox *b) {
    float dx = b->hi[0] - b->lo[0], dy = b->hi[1] - b->lo[1], dz = b->hi[2] - b->lo[2];
    return (dx * dy + dy * dz) + dz * dx;
}

typedef struct { int64_t first, count; int32_t node; } sah_task;

/* Builds the full binary tree.  perm[n]: primitive ids in leaf order.
 * nodes[4*i..]: (first, count, axis, left count) of node i in preorder
 * (left subtree first); a single primitive has count 1, axis -1, left 0.
 * boxes[6*i..]: node box (lo, hi).  Returns the node count 2n - 1. */
int64_t orc_sah_build(const float *verts, const int32_t *tris, int64_t n, int32_t *perm,
                      int64_t *nodes, float *boxes) {
    if (n <= 0) return 0;
    fbox *pb = (fbox *)malloc((size_t)n * sizeof(fbox));
    float *cen = (float *)malloc((size_t)n * 3 * sizeof(float));
    int32_t *tmp = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    unsigned char *side = (unsigned char *)malloc((size_t)n);
    for (int64_t i = 0; i < n; i++) {
        fbox_empty(&pb[i]);
        for (int k = 0; k < 3; k++) {
            const float *p = verts + 3 * (int64_t)tris[3 * i + k];
            for (int a = 0; a < 3; a++) {
                if (p[a] < pb[i].lo[a]) pb[i].lo[a] = p[a];
                if (p[a] > pb[i].hi[a]) pb[i].hi[a] = p[a];
            }
        }
        for (int a = 0; a < 3; a++) cen[3 * i + a] = 0.5f * pb[i].lo[a] + 0.5f * pb[i].hi[a];
        perm[i] = (int32_t)i;
    }
    sah_task *stack = (sah_task *)malloc((size_t)(n + 1) * sizeof(sah_task));
    int64_t sp = 0;
    stack[sp++] = (sah_task){ 0, n, 0 };
    while (sp > 0) {
        sah_task t = stack[--sp];
        int64_t *nd = nodes + 4 * (int64_t)t.node;
        fbox box;
        fbox_empty(&box);
        for (int64_t i = t.first; i < t.first + t.count; i++) fbox_grow(&box, &pb[perm[i]]);
        for (int a = 0; a < 3; a++) {
            boxes[6 * (int64_t)t.node + a] = box.lo[a];
            boxes[6 * (int64_t)t.node + 3 + a] = box.hi[a];
        }
        nd[0] = t.first; nd[1] = t.count;
        if (t.count == 1) { nd[2] = -1; nd[3] = 0; continue; }
        float cl[3] = { INFINITY, INFINITY, INFINITY }, ch[3] = { -INFINITY, -INFINITY, -INFINITY };
        for (int64_t i = t.first; i < t.first + t.count; i++)
            for (int a = 0; a < 3; a++) {
                float c = cen[3 * (int64_t)perm[i] + a];
                if (c < cl[a]) cl[a] = c;
                if (c > ch[a]) ch[a] = c;
            }
        int best_axis = -1, best_k = -1;
        float best_cost = INFINITY;
        for (int a = 0; a < 3; a++) {
            float ext = ch[a] - cl[a];
            if (!(ext > 0.0f) || isinf(ext)) continue;
            float scale = (float)SAH_BINS / ext;
            int64_t cnt[SAH_BINS] = { 0 };
            fbox bb[SAH_BINS];
            for (int k = 0; k < SAH_BINS; k++) fbox_empty(&bb[k]);
            for (int64_t i = t.first; i < t.first + t.count; i++) {
                int32_t p = perm[i];
                int b = (int)((cen[3 * (int64_t)p + a] - cl[a]) * scale);
                if (b > SAH_BINS - 1) b = SAH_BINS - 1;
                cnt[b]++;
                fbox_grow(&bb[b], &pb[p]);
            }
            /* suffix unions: right side of split k = bins k+1 .. 31 */
            fbox rs[SAH_BINS];
            int64_t rn[SAH_BINS];
            fbox_empty(&rs[SAH_BINS - 1]);
            fbox_grow(&rs[SAH_BINS - 1], &bb[SAH_BINS - 1]);
            rn[SAH_BINS - 1] = cnt[SAH_BINS - 1];
            for (int j = SAH_BINS - 2; j >= 0; j--) {
                rs[j] = rs[j + 1];
                fbox_grow(&rs[j], &bb[j]);
                rn[j] = rn[j + 1] + cnt[j];
            }
            fbox l;
            int64_t nl = 0;
            fbox_empty(&l);
            for (int k = 0; k < SAH_BINS - 1; k++) {
                fbox_grow(&l, &bb[k]);
                nl += cnt[k];
                int64_t nr = rn[k + 1];
                if (nl == 0 || nr == 0) continue;
                float cost = half_area(&l) * (float)nl + half_area(&rs[k + 1]) * (float)nr;
                if (cost < best_cost) { best_cost = cost; best_axis = a; best_k = k; }
            }
        }
        int64_t nl = 0;
        if (best_axis >= 0) {
            float ext = ch[best_axis] - cl[best_axis];
            float scale = (float)SAH_BINS / ext;
            for (int64_t i = t.first; i < t.first + t.count; i++) {
                int b = (int)((cen[3 * (int64_t)perm[i] + best_axis] - cl[best_axis]) * scale);
                if (b > SAH_BINS - 1) b = SAH_BINS - 1;
                side[i] = b <= best_k;
                nl += side[i];
            }
        } else {
            nl = t.count / 2;
            for (int64_t i = t.first; i < t.first + t.count; i++) side[i] = (i - t.first) < nl;
            best_axis = 0;
        }
        /* stable partition */
        int64_t w = t.first;
        for (int64_t i = t.first; i < t.first + t.count; i++) if (side[i]) tmp[w++] = perm[i];
        for (int64_t i = t.first; i < t.first + t.count; i++) if (!side[i]) tmp[w++] = perm[i];
        memcpy(perm + t.first, tmp + t.first, (size_t)t.count * sizeof(int32_t));
        nd[2] = best_axis; nd[3] = nl;
        /* preorder: the left child is the next node, the right child follows
         * the left subtree (2 nl - 1 nodes) */
        int32_t left = t.node + 1, right = t.node + (int32_t)(2 * nl);
        stack[sp++] = (sah_task){ t.first + nl, t.count - nl, right };
        stack[sp++] = (sah_task){ t.first, nl, left };
    }
    free(stack); free(side); free(tmp); free(cen); free(pb);
    return 2 * n - 1;
}
