/*
 * bvh.h - C ABI of the MI355X (gfx950) closest-hit BVH library.
 *
 * The library builds a bounding volume hierarchy over an indexed triangle
 * mesh on the GPU and traces rays through it.  The node layout is chosen at
 * build time and is independent of the traversal code: one traversal routine
 * is instantiated per layout, the separation of logical tree and physical
 * layout argued in Sec. 3-4 of "Decoupling Data Layouts from Bounding Volume
 * Hierarchies" (PLDI 2026).
 *
 * Conventions shared by every call
 *   - Pointers named "device" are device (HBM) addresses on the current HIP
 *     device; pointers named "host" are ordinary host memory.
 *   - `stream` is a hipStream_t passed as void*; NULL is the default stream.
 *     Calls that take a stream are stream-ordered and asynchronous: they
 *     enqueue work and return; buffers must stay valid until the stream has
 *     reached that point.  bvh_build is the exception: it synchronises
 *     `stream` before it returns.
 *   - Every call returns BVH_OK (0) or a negative error code and never
 *     aborts.  bvh_last_error() gives a message for the calling thread's
 *     most recent failure.  Arguments are validated before any work is
 *     enqueued; a call that fails validation enqueues nothing.
 *   - The caller owns every buffer it passes in.  A handle owns only what it
 *     allocated itself (nodes, leaf triangles) and frees it in bvh_destroy.
 *   - All records are little-endian and naturally aligned.
 */
#ifndef BVH_H
#define BVH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes -------------------------------------------------------- */
#define BVH_OK 0
#define BVH_EINVAL (-1)       /* bad argument (null pointer, size, enum, index) */
#define BVH_ENOMEM (-2)       /* a device allocation failed */
#define BVH_EHIP (-3)         /* a HIP runtime call failed */
#define BVH_ENODEV (-4)       /* no HIP device */
#define BVH_EUNSUPPORTED (-5) /* valid input beyond a documented limit */

/* ---- enums -------------------------------------------------------------- */
/* Node layouts (record formats below). */
#define BVH_LAYOUT_AABB2 0    /* binary, node stores its own f32 box, 32 B */
#define BVH_LAYOUT_BVH4 1     /* 4-wide, f32 child boxes in SoA, 128 B */
#define BVH_LAYOUT_BVH8_Q8 2  /* 8-wide, u8 child boxes in the parent frame, 128 B */
#define BVH_LAYOUT_BVH8_Q16 3 /* 8-wide, u16 child boxes in the parent frame, 160 B */
#define BVH_LAYOUT_PBRT_Q16 4 /* binary, own u16 box in the scene frame, 16 B */
#define BVH_LAYOUT_SG_EQ 5    /* binary, own 10-bit box in the scene frame, 12 B */
#define BVH_LAYOUT_PBRT_SOAOS 6     /* AABB2 as a box array and a topology array, 24 + 8 B */
#define BVH_LAYOUT_PBRT_Q16_SOAOS 7 /* PBRT_Q16 as a box array and a topology array, 12 + 4 B */
#define BVH_LAYOUT_SG_EQ_A16 8      /* SG_EQ records padded to 16 B */
#define BVH_LAYOUT_SHARED_SLAB 9    /* binary, one slab per node refining the inherited box, 16 B */
#define BVH_NUM_LAYOUTS 10

/* Leaf storage. */
#define BVH_LEAF_COMPACT 0 /* triangles copied into leaf order (bvh_tri records) */
#define BVH_LEAF_INDEXED 1 /* leaf order holds primitive ids; vertices gathered */

/* Trace modes. */
#define BVH_TRACE_CLOSEST 0 /* nearest hit, ties to the lowest primitive id */
#define BVH_TRACE_ANY 1     /* any hit with t <= tmax (occlusion) */

/* Topology builders (bvh_build_opts.builder).  LBVH: Morton codes of the
 * primitive-box centres, radix sort, Karras hierarchy (fast).  SAH: top-down
 * binary splits chosen by the surface area heuristic over 32 bins per axis
 * (Sec. 9.2.1; slower to build, fewer nodes visited per query).  SAH rules:
 * a node bins its primitives' centres c = 0.5 lo + 0.5 hi along each axis
 * over their exact bounds [cl, ch] (axes with ch - cl not positive and finite
 * are skipped; bin = min(31, trunc((c - cl) * (32 / (ch - cl)))), f32); the
 * split after bin k costs A(L) N(L) + A(R) N(R), A = dx dy + dy dz + dz dx of
 * a side's box, both sides non-empty; the cheapest wins, ties to the lower
 * axis and then the lower k; partitions are stable (initial order: primitive
 * id); coincident centres split at the index median floor(N/2).  Splitting
 * continues to single primitives; leaves are the subtrees of at most
 * leaf_size primitives (as with LBVH).  A tree deeper than the traversal
 * stack bound fails with EUNSUPPORTED. */
#define BVH_BUILDER_LBVH 0
#define BVH_BUILDER_SAH 1

/* Buffers readable with bvh_read_buffer. */
#define BVH_BUF_NODES 0
#define BVH_BUF_LEAF 1 /* COMPACT: bvh_tri[n_tris]; INDEXED: int32 prim id[n_tris] */

/* ---- records ------------------------------------------------------------ */
/* A ray: o + t d for tmin < t <= tmax.  tmin must be 0 (the intersection
 * test accepts 0 < t, App. G).  tmax = +inf means unbounded.  d need not be
 * unit length; t is measured in units of |d|. */
typedef struct bvh_ray {
    float o[3];
    float tmin;
    float d[3];
    float tmax;
} bvh_ray; /* 32 B */

/* A hit: the hit point is (1-u-v) p0 + u p1 + v p2 = o + t d (App. G's
 * barycentrics b0 = 1-u-v, b1 = u, b2 = v).  A miss is {-1, +inf, 0, 0}. */
typedef struct bvh_hit {
    int32_t prim_id;
    float t, u, v;
} bvh_hit; /* 16 B */

/* Build options; a zero field selects the default. */
typedef struct bvh_build_opts {
    int32_t leaf_size;   /* max triangles per leaf, 1..16 (1..15 for the PBRT_Q16 and SG_EQ
                            layouts and their variants; default 4) */
    int32_t leaf_mode;   /* BVH_LEAF_COMPACT (default) or BVH_LEAF_INDEXED */
    int32_t stack_lds;   /* traversal stack entries kept in LDS per ray: 8, 16 or 32 (default:
                            32 for AABB2, 16 for the wide layouts).  A ray that needs more is
                            re-traced by a fallback pass with a deep stack in global memory.
                            Results do not depend on it. */
    int32_t builder;     /* BVH_BUILDER_LBVH (default) or BVH_BUILDER_SAH */
    int32_t reserved[4]; /* must be zero */
} bvh_build_opts;

typedef struct bvh_stats {
    int32_t layout, leaf_mode, arity, leaf_size;
    int64_t n_tris;            /* triangles in the scene */
    int64_t n_nodes;           /* node records */
    int64_t n_leaves;          /* leaves (each 1..leaf_size triangles) */
    int64_t node_bytes;        /* size of one node record */
    int64_t nodes_buffer_bytes;
    int64_t leaf_buffer_bytes; /* bvh_tri array or prim-id array */
    int64_t extra_bytes;       /* INDEXED: the handle's copies of verts and tris */
    int32_t depth;             /* nodes on the longest root-to-leaf path */
    int32_t max_stack;         /* worst-case traversal stack entries */
    float scene_lo[3], scene_hi[3];
    int32_t stack_lds;         /* LDS stack entries per ray of the trace kernels */
    int32_t builder;           /* BVH_BUILDER_LBVH or BVH_BUILDER_SAH */
    /* PBRT_Q16 and SG_EQ: the scene frame of the quantised boxes (a lower
     * plane value is fmaf((float)q, frame_scale[a], frame_origin[a]); an
     * SG_EQ upper plane is fmaf(-(float)q, frame_scale[a], frame_top[a]));
     * zero otherwise. */
    float frame_origin[3], frame_scale[3], frame_top[3];
    int32_t pad2;
} bvh_stats;

/* Compacted leaf triangle (BVH_LEAF_COMPACT), 48 B, in leaf order: the
 * first vertex and the two edges of the ray/triangle test,
 * e1 = p1 - p0 and e2 = p2 - p0, each component the f32 difference the test
 * uses (so p1 and p2 are not stored). */
typedef struct bvh_tri {
    float p0[3], e1[3], e2[3];
    int32_t prim_id; /* index of the triangle in the caller's `tris` */
    int32_t pad[2];
} bvh_tri;

/*
 * Node records.  Node 0 is the root.
 *
 * BVH_LAYOUT_AABB2 (after the PBRTv4 LinearBVH node of Fig. 5): nodes in
 * preorder; the left child of interior node I is I+1 and the right child is
 * I + offset.  meta bits 0..15 = number of triangles (0 for an interior
 * node), bits 16..17 = split axis of an interior node (x, y, z = 0, 1, 2: the
 * left subtree lies on the low side).  A leaf's triangles are leaf-order
 * entries offset .. offset+n-1.
 */
typedef struct bvh_node_aabb2 {
    float lo[3], hi[3];
    uint32_t offset;
    uint32_t meta;
} bvh_node_aabb2; /* 32 B */

/*
 * Wide layouts (BVH4, BVH8_Q8, BVH8_Q16) store the boxes of the children in
 * the parent, structure-of-arrays across the children (App. D.2 uses the same
 * child-box-in-parent form for bvh8-q8-ci).  Child slots 0..nchild-1 are
 * valid; the rest hold an empty box and ref 0xFFFFFFFF.
 *
 * Child reference (u32, tagged as in App. D.2's compressed index):
 *   bit 0 = 1: interior child, node index = ref >> 1.
 *   bit 0 = 0: leaf, nprims - 1 = bits 1..4 (1..16 triangles),
 *              first leaf-order triangle = bits 5..31 (so at most 2^27 - 1
 *              triangles per scene).
 *
 * Quantised boxes (after App. D.2, but with a rounding rule that makes the
 * dequantised box always contain the exact child box): the dequantised
 * plane value is fmaf((float)q, scale[a], origin[a]) (one correctly rounded
 * fused multiply-add), where origin is the exact lower corner of the node's
 * box and q lies in 0..255 (Q8) or 0..65535 (Q16).  The builder picks the
 * largest lower and smallest upper q whose dequantised planes still
 * enclose the child.  An axis of zero extent has scale 0.
 */
typedef struct bvh_node_bvh4 {
    float lo_x[4], lo_y[4], lo_z[4];
    float hi_x[4], hi_y[4], hi_z[4];
    uint32_t child[4];
    uint32_t nchild;
    uint32_t pad[3];
} bvh_node_bvh4; /* 128 B */

typedef struct bvh_node_bvh8_q8 {
    float origin[3];
    float scale[3];
    uint8_t qlo_x[8], qlo_y[8], qlo_z[8];
    uint8_t qhi_x[8], qhi_y[8], qhi_z[8];
    uint32_t child[8];
    uint32_t nchild;
    uint32_t pad[5];
} bvh_node_bvh8_q8; /* 128 B */

typedef struct bvh_node_bvh8_q16 {
    float origin[3];
    float scale[3];
    uint16_t qlo_x[8], qlo_y[8], qlo_z[8];
    uint16_t qhi_x[8], qhi_y[8], qhi_z[8];
    uint32_t child[8];
    uint32_t nchild;
    uint32_t pad;
} bvh_node_bvh8_q16; /* 160 B */

/*
 * BVH_LAYOUT_PBRT_Q16 (the pbrt-q16 layout of Sec. 9.2.5 and App. D.3): the
 * AABB2 tree in the same preorder, each node 16 B.  Its box is quantised to
 * u16 in one frame for the whole scene (the root box split into 65535 steps
 * per axis; bvh_stats.frame_*), conservatively as for the quantised wide
 * layouts.  meta bits 0..3 = number of triangles (0 for an interior node),
 * bits 4..31 = right-child offset (interior: right child = I + offset) or
 * first leaf-order triangle (leaf).  The lowest bits of an interior node's
 * lo[0] and lo[1] carry its split axis (axis = (lo[0] & 1) | (lo[1] & 1) << 1,
 * 3 = unknown): the quantised lower plane is lowered by one step where needed
 * to hold the bit, which keeps the box conservative; the traversal uses the
 * axis only to pick the near child first.
 */
typedef struct bvh_node_pbrt_q16 {
    uint16_t lo[3], hi[3];
    uint32_t meta;
} bvh_node_pbrt_q16; /* 16 B */

/*
 * BVH_LAYOUT_SG_EQ (the snapped-grid extent quantisation of App. D.1): the
 * AABB2 tree in the same preorder, each node 12 B.  The scene box is split
 * into 1023 steps of frame_scale per axis; a lower plane counts steps up from
 * frame_origin, an upper plane counts steps down from frame_top:
 *   lo[a] = fmaf((float)qlo_a, frame_scale[a], frame_origin[a])
 *   hi[a] = fmaf(-(float)qhi_a, frame_scale[a], frame_top[a])
 * with the tightest q whose plane still encloses the node's box (the builder
 * checks this with the same fused multiply-add, so no directed rounding is
 * needed at traversal time).  Packing:
 *   qlo  = qlo_x << 20 | qlo_y << 10 | qlo_z | (nprims & 3) << 30
 *   qhi  = qhi_x << 20 | qhi_y << 10 | qhi_z | (nprims >> 2) << 30
 *   off  = bits 0..29: right-child offset (interior: right = I + off) or
 *          first leaf-order triangle (leaf); bits 30..31: split axis of an
 *          interior node (x, y, z = 0, 1, 2), used only for near-first order.
 * nprims = 0 marks an interior node (1..15 triangles in a leaf).
 */
typedef struct bvh_node_sg_eq {
    uint32_t qlo, qhi, off;
} bvh_node_sg_eq; /* 12 B */

/*
 * The "-soaos" and "-align16" variants of Table 1 (Sec. 9.1: a global
 * memory transformation for locality, and 16-byte alignment), over the same
 * preorder tree and the same field encodings:
 *
 * BVH_LAYOUT_PBRT_SOAOS: the AABB2 records split into two arrays of
 *   n_nodes entries each, one after the other in the node buffer: first the
 *   boxes (bvh_node_box_f32, 24 B), then the topology words
 *   (bvh_node_topo, 8 B: AABB2's offset and meta).  The traversal fetches a
 *   node's topology only when the ray meets its box.
 * BVH_LAYOUT_PBRT_Q16_SOAOS: the PBRT_Q16 records split the same way: first
 *   the u16 boxes (bvh_node_box_q16, 12 B, with the split axis in the lowest
 *   bits of lo[0] and lo[1] as in PBRT_Q16), then the meta words (uint32_t:
 *   count | offset << 4).
 * BVH_LAYOUT_SG_EQ_A16: SG_EQ records followed by a zero word
 *   (bvh_node_sg_eq_a16, 16 B), one aligned 16-byte fetch per node.
 */
typedef struct bvh_node_box_f32 {
    float lo[3], hi[3];
} bvh_node_box_f32; /* 24 B */

typedef struct bvh_node_topo {
    uint32_t offset, meta;
} bvh_node_topo; /* 8 B */

typedef struct bvh_node_box_q16 {
    uint16_t lo[3], hi[3];
} bvh_node_box_q16; /* 12 B */

typedef struct bvh_node_sg_eq_a16 {
    uint32_t qlo, qhi, off, pad;
} bvh_node_sg_eq_a16; /* 16 B */

/*
 * BVH_LAYOUT_SHARED_SLAB (the tree-carried shared slab of Sec. 8.3): the
 * AABB2 tree in the same preorder, each node storing one slab [slo, shi]
 * along one axis instead of a box.  A node's box is the box carried down
 * from its parent with that axis replaced by the slab (the root's carried
 * box is the scene box, bvh_stats.scene_lo/hi); the node's children inherit
 * the result.  The slab axis is the one along which the node's exact box is
 * narrowest relative to its parent's exact box (the lowest axis on ties),
 * and the slab is the exact extent there, so every node's box encloses its
 * triangles.  meta: bits 0..15 triangle count (0: interior), bits 16..17
 * slab axis, bits 18..19 split axis (near-first order); offset as AABB2.
 * The traversal carries a box per stack entry (per-lane stacks in a global
 * work area); bvh_batch_create rejects this layout with EUNSUPPORTED.
 */
typedef struct bvh_node_slab {
    float slo, shi;
    uint32_t offset, meta;
} bvh_node_slab; /* 16 B */

typedef struct bvh_handle_s *bvh_handle_t;

/* ---- calls -------------------------------------------------------------- */

/* Message for the calling thread's most recent failed call ("" if none).
 * The string stays valid until the thread's next failing call. */
const char *bvh_last_error(void);

/* Library ABI version (this header: 1). */
int32_t bvh_version(void);

/*
 * Builds a BVH over n_tris triangles (Sec. 5's two phases: a logical binary
 * tree first, then its packing into the chosen layout).  With the LBVH
 * builder the logical tree is a linear BVH: Morton codes of the triangle box
 * centres with b = ceil(log2(n_tris) / 3) + 4 bits per axis (at most 21,
 * one fewer where that saves an 8-bit sort pass), a stable radix sort over
 * the 3b key bits, the hierarchy of the sorted codes (equal codes ordered by
 * position), node boxes as unions of the leaf boxes of each node's sorted
 * range (a sparse table of range unions, no bottom-up refit), then collapse
 * of every subtree of at most leaf_size triangles into one leaf.  The Morton
 * bit count shapes only the topology; hits do not depend on it.
 *   verts   device, n_verts x 3 float (x, y, z)
 *   tris    device, n_tris x 3 int32 vertex indices, each in [0, n_verts)
 *   layout  BVH_LAYOUT_*
 *   opts    host, may be NULL for defaults
 *   out     host; receives the handle on success, NULL on failure
 * Errors: EINVAL for null pointers with a nonzero count, negative counts,
 * an unknown layout or leaf mode, leaf_size outside 1..16 (1..15 for
 * PBRT_Q16 and SG_EQ), nonzero reserved
 * fields, or (detected on the device, reported before returning) a vertex
 * index outside [0, n_verts); EUNSUPPORTED for n_tris >= 2^27, a tree whose
 * traversal stack would exceed the kernel's limit, or a wide layout whose
 * node buffer would reach 4 GiB; ENOMEM; EHIP; ENODEV.
 * n_tris = 0 gives a valid empty handle whose traces all miss.
 * Synchronises `stream` before returning.  verts and tris are not retained.
 */
int32_t bvh_build(const float *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                  int32_t layout, const bvh_build_opts *opts, void *stream, bvh_handle_t *out);

/* Frees everything the handle owns (synchronises the device first).  NULL is
 * accepted and ignored. */
int32_t bvh_destroy(bvh_handle_t h);

/* Sizes and shape of a built BVH.  out: host. */
int32_t bvh_get_stats(bvh_handle_t h, bvh_stats *out);

/* Copies up to `capacity` bytes of a handle buffer (BVH_BUF_*) to host
 * memory (synchronous); *bytes_total receives the buffer's full size.
 * host_dst may be NULL with capacity 0 to query the size only. */
int32_t bvh_read_buffer(bvh_handle_t h, int32_t which, void *host_dst, int64_t capacity,
                        int64_t *bytes_total);

/*
 * Traces n rays (closest_hit of Fig. 4 / App. G).  CLOSEST returns the hit
 * with the smallest t, ties to the lowest primitive id; ANY returns some hit
 * with t <= tmax, or a miss.  Ray-triangle test: Moller-Trumbore (the test
 * of App. G) with App. G's intervals (edges and vertices inclusive, both
 * faces, 0 < t <= tmax), evaluated in FP32 as follows, every step one
 * correctly rounded operation (fma = fused multiply-add):
 *   e1 = p1 - p0, e2 = p2 - p0, S = o - p0;
 *   a x b = (fma(a.y, b.z, -(a.z b.y)), fma(a.z, b.x, -(a.x b.z)),
 *            fma(a.x, b.y, -(a.y b.x)));
 *   a . b = fma(a.z, b.z, fma(a.y, b.y, a.x b.x));
 *   P = d x e2, det = e1 . P, Q = S x e1;
 *   U, V, T = S . P, d . Q, e2 . Q, each with the sign bit of det xor-ed in;
 *   hit iff 0 < |det| < inf, U >= 0, V >= 0, U + V <= |det|, T > 0 and
 *   T <= |det| tmax; then t, u, v = T, U, V times (1 / |det|).
 *   rays  device, n records;  hits  device, n records (written)
 * Errors: EINVAL for a null handle, n < 0, null pointers with n > 0, an
 * unknown mode.  Rays with tmin != 0 are traced as if tmin were 0.
 * Concurrent traces on one handle are allowed (the handle is read-only).
 */
int32_t bvh_trace(bvh_handle_t h, const bvh_ray *rays, int64_t n, bvh_hit *hits, int32_t mode,
                  void *stream);

/*
 * bvh_trace for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same hits as bvh_trace, and no call here allocates or frees memory.  The
 * work area (fallback-pass header, list and deep stacks) is a fixed array of
 * 16 MiB + 2,304 B in device memory, one per GPU, held from the library's
 * first use of that GPU until the process ends; each call clears its header
 * with a small kernel before tracing.  Every call on one GPU uses that GPU's
 * array, so calls that overlap in time on one GPU (different streams or host
 * threads) race and give undefined results: serialise them.  Rays run one
 * per lane with the handle's LDS stack; rays that outgrow it are re-traced
 * with a deep stack, as in bvh_trace.
 *   rays  device, n records;  hits  device, n records (written)
 * Errors: as bvh_trace, plus EINVAL for n > BVH_NOALLOC_MAX_RAYS and
 * EUNSUPPORTED for the SHARED_SLAB layout (its carried-box stacks do not fit
 * the fixed area).
 */
#define BVH_NOALLOC_MAX_RAYS 2097152
int32_t bvh_trace_noalloc(bvh_handle_t h, const bvh_ray *rays, int64_t n, bvh_hit *hits,
                          int32_t mode, void *stream);

/*
 * bvh_trace plus per-ray work counters, for measurement: counts[2i] = node
 * records fetched, counts[2i+1] = triangles tested.  Same hits as bvh_trace.
 *   counts  device, 2n uint32 (written)
 */
int32_t bvh_trace_counts(bvh_handle_t h, const bvh_ray *rays, int64_t n, bvh_hit *hits,
                         int32_t mode, uint32_t *counts, void *stream);

/*
 * Gradient of a loss L through closest-hit results with each ray's hit
 * primitive held fixed.  For ray i with p = hits[i].prim_id >= 0 (only the
 * id is read from hits), the hit (t, u, v) on triangle p is recomputed from
 * rays[i] and verts/tris with the FP32 arithmetic of the ray/triangle test
 * of bvh_trace (so it equals the forward's hit bit for bit when the same
 * inputs were traced; the interval tests are not applied, so a fixed
 * primitive that the ray now misses still gets the gradient of its
 * extended-plane solution).  With e1 = p1 - p0, e2 = p2 - p0,
 * g = grad_hits[i] = dL/d(t,u,v) and J = [d | -e1 | -e2], the solution of
 * J^T lam = g (by Cramer's rule, FP32) gives
 *   dL/do = -lam, dL/dd = -t lam, dL/dp0 = (1-u-v) lam, dL/dp1 = u lam,
 *   dL/dp2 = v lam
 * (implicit differentiation of o + t d = (1-u-v) p0 + u p1 + v p2).  No
 * traversal state is stored or needed.
 *   verts       device, n_verts x 3 float;  tris  device, n_tris x 3 int32
 *   rays, hits  device, n records (hits from bvh_trace CLOSEST)
 *   grad_hits   device, n x 3 float (dL/dt, dL/du, dL/dv)
 *   grad_verts  device, n_verts x 3 float, ACCUMULATED (+=).  Meshes of up to
 *               2^22 vertices: the contributions are grouped by vertex range
 *               in a work area (16 B per ray contribution; grow-only, kept
 *               per stream) and each range is summed in one workgroup's
 *               LDS (up to 2^18 vertices: one accumulator per wave, no
 *               atomics; beyond: LDS float atomics); larger meshes add
 *               per-block partial sums with device float atomics.  Either
 *               way the summation order (last bits) varies between runs.
 *               Calls that share a stream share its work area: they are
 *               ordered by the stream.
 *   grad_rays   device, n x 6 float (dL/do, dL/dd), OVERWRITTEN; a miss or
 *               a skipped ray gets zeros
 * Rays whose prim_id is outside [0, n_tris), whose triangle has a vertex
 * index outside [0, n_verts), or whose system is singular (det = 0 or not
 * finite) contribute nothing.
 * Errors: EINVAL for negative sizes or null pointers with a nonzero count;
 * ENOMEM when the work area cannot be allocated.
 */
int32_t bvh_trace_backward(const float *verts, int64_t n_verts, const int32_t *tris, int64_t n_tris,
                           const bvh_ray *rays, int64_t n, const bvh_hit *hits,
                           const float *grad_hits, float *grad_verts, float *grad_rays,
                           void *stream);

/* ---- closest-point query --------------------------------------------------- */
/* A query point p with squared search radius r2 (inclusive; +inf means
 * unbounded). */
typedef struct bvh_point_query {
    float p[3];
    float r2;
} bvh_point_query; /* 16 B */

/* Nearest triangle of a query: its id, the squared distance d2 and the
 * barycentrics of its nearest point, (1-u-v) p0 + u p1 + v p2.  None within
 * r2 is {-1, +inf, 0, 0}. */
typedef struct bvh_closest {
    int32_t prim_id;
    float d2, u, v;
} bvh_closest; /* 16 B */

/*
 * Closest-point query on any layout (App. G "Closest Point Query"; the same
 * layouts serve ray tracing and this query, Sec. 9.2.3 and 9.3.2): for each
 * query the triangle at the smallest squared distance d2 <= r2 from p, ties
 * to the lowest primitive id.  Children are visited nearest box first and
 * boxes farther than the best triangle so far are skipped (box distances are
 * computed conservatively, so the skip never loses a nearer triangle).  The
 * point-triangle distance is Ericson's Voronoi-region method (Real-Time
 * Collision Detection 5.1.5) in f32, the method of the paper's listing, on
 * a = p0, ab = p1 - p0, ac = p2 - p0; d2, u, v are that computation's f32
 * results.  A degenerate triangle is measured by its edges.  The handle's
 * stack_lds applies with at most 16 entries; when the build left it at its
 * default, the wide layouts use 8.  Results do not depend on it.
 *   queries  device, n records;  out  device, n records (written)
 * A query whose point has a non-finite coordinate, or whose r2 is negative
 * or NaN, gets {-1, +inf, 0, 0}.
 * Errors: EINVAL for a null handle, n < 0, null pointers with n > 0;
 * EUNSUPPORTED for more than 2^32 - 1 queries.  Concurrent queries and
 * traces on one handle are allowed.
 */
int32_t bvh_closest_point(bvh_handle_t h, const bvh_point_query *queries, int64_t n,
                          bvh_closest *out, void *stream);

/*
 * bvh_closest_point plus per-query work counters, for measurement:
 * counts[2i] = node records fetched, counts[2i+1] = triangles measured.
 * Same results as bvh_closest_point.
 *   counts  device, 2n uint32 (written)
 */
int32_t bvh_closest_point_counts(bvh_handle_t h, const bvh_point_query *queries, int64_t n,
                                 bvh_closest *out, uint32_t *counts, void *stream);

/* ---- batched tracing ------------------------------------------------------ */
/*
 * Many scenes with uneven triangle and ray counts traced by one graph launch.
 * The paper leaves execution scheduling to future work (Sec. 1) and shows that
 * the best layout depends on scene and ray distribution (Sec. 9.2.2); here
 * each scene's layout (and with it the tree arity) and LDS stack depth are
 * chosen by timing candidates on probe rays (every layout at the first stack
 * depth, then the other depths on the winner), and all scenes' rays are
 * drained from per-variant work queues by persistent kernels captured in one
 * hipGraph (variants one after another, each on the whole GPU).
 */
typedef struct bvh_scene_desc {
    const float *verts;   /* device, n_verts x 3 float */
    int64_t n_verts;
    const int32_t *tris;  /* device, n_tris x 3 int32 */
    int64_t n_tris;
    int32_t layout;       /* BVH_LAYOUT_* to fix it, or -1 to let the tuner choose */
    int32_t stack_lds;    /* 8, 16 or 32 to fix it, or 0 to let the tuner choose */
    int32_t reserved[2];  /* must be zero */
} bvh_scene_desc;

typedef struct bvh_tune_opts {
    int32_t probe_rays;           /* probe rays per scene and candidate (0: 524288, enough
                                     to fill the GPU) */
    int32_t leaf_size;            /* 1..16 (0: 4); leaves are compacted; PBRT_Q16 and
                                     SG_EQ are tuning candidates only for leaf_size <= 15 */
    const bvh_ray *probe;         /* device, optional probe rays of all scenes, concatenated */
    const int64_t *probe_offsets; /* host, n_scenes + 1 offsets into probe; required with it */
    int32_t reserved[4];          /* must be zero */
} bvh_tune_opts;

typedef struct bvh_batch_scene_info {
    int32_t layout;           /* chosen layout */
    int32_t stack_lds;        /* chosen LDS stack entries */
    int32_t candidates;       /* candidates timed (1 when nothing was left to choose) */
    float probe_ns_per_ray;   /* chosen candidate's time per probe ray (0 if not timed) */
    int64_t n_nodes;
    int64_t bvh_bytes;        /* nodes + leaf triangles */
} bvh_batch_scene_info;

typedef struct bvh_batch_s *bvh_batch_t;

/*
 * Builds a BVH per scene and tunes it.  Probe rays: opts->probe when given,
 * otherwise generated on the device (origins uniform in the scene box,
 * directions uniform on the sphere, a fixed integer-hash sequence).
 *   scenes  host array of n_scenes descriptors (device mesh pointers, not
 *           retained).  opts may be NULL.
 * Errors: as bvh_build per scene, plus EINVAL for n_scenes < 1, a bad layout
 * or stack value, nonzero reserved fields, or probe without probe_offsets.
 * Synchronises `stream`.
 */
int32_t bvh_batch_create(const bvh_scene_desc *scenes, int32_t n_scenes, const bvh_tune_opts *opts,
                         void *stream, bvh_batch_t *out);

/* The tuner's choice for one scene.  out: host. */
int32_t bvh_batch_get_scene_info(bvh_batch_t b, int32_t scene, bvh_batch_scene_info *out);

/* The scene's BVH handle (owned by the batch; valid until bvh_batch_destroy),
 * usable with bvh_trace. */
int32_t bvh_batch_scene_handle(bvh_batch_t b, int32_t scene, bvh_handle_t *out);

/*
 * Closest hit for every scene's rays: rays[ray_offsets[s] .. ray_offsets[s+1])
 * are traced against scene s and their hits written to the same positions
 * of `hits`.  Results equal bvh_trace of each scene's handle.
 *   rays, hits   device;  ray_offsets  host, n_scenes + 1 non-decreasing
 * The first call for a given (rays, hits, ray_offsets) builds and
 * instantiates a hipGraph (one small kernel that resets the work-queue
 * counters, then per layout/stack variant one persistent kernel over the
 * whole GPU followed by its deep-stack fallback pass, the variants chained
 * one after another); later calls with the same
 * arguments replay it.  Calls
 * on one batch must not overlap in time (they share the queue counters).
 */
int32_t bvh_batch_trace(bvh_batch_t b, const bvh_ray *rays, const int64_t *ray_offsets,
                        bvh_hit *hits, void *stream);

/* Frees the batch, its graph and every scene's BVH (synchronises the device). */
int32_t bvh_batch_destroy(bvh_batch_t b);

#ifdef __cplusplus
}
#endif

#endif /* BVH_H */
