"""GPU closest-point query against the CPU oracle, through the C ABI.

The oracle computes the exact (FP64) nearest triangle; the GPU computes
Ericson's region method in f32 (the paper's listing).  Tolerance, from the
f32 arithmetic: the GPU's nearest point and distance for a triangle T lie
within tol(T) = 2^-19 * (|q - p0| + L) * (1 + kappa) of the exact ones, where
L is T's longest edge and kappa = L^2 / |e1 x e2| its shape factor: each
dot product, difference and FMA of the method rounds once (relative 2^-24),
the face barycentrics divide by |e1 x e2|^2-sized quantities whose relative
error grows with kappa, and 2^-19 = 32 * 2^-24 covers the roughly ten
operations on the longest dependency chain with a factor of three to spare.
A query is graded on prim_id when the exact runner-up is farther than the
nearest by more than the two triangles' tolerances (and, with a finite
radius, the nearest is not within its tolerance of the radius); graded
results must match the oracle's triangle and agree across layouts and leaf
modes bit for bit.  Every returned triangle must be within tolerance of the
nearest distance, and its reported d2 and barycentric point within
tolerance of the exact ones for that triangle.
"""
import math

import numpy as np
import pytest

from paper_2511_15028_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LAYOUTS = ["aabb2", "bvh4", "bvh8_q8", "bvh8_q16", "pbrt_q16", "sg_eq", "pbrt_soaos",
           "pbrt_q16_soaos", "sg_eq_a16", "shared_slab"]
TOL = 2.0 ** -19


def B():
    from paper_2511_15028_amd import bvh
    return bvh


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_build(verts, tris, layout, leaf_mode="compact", leaf_size=4, stack_lds=0):
    return B().build(dev(verts), dev(tris), layout, leaf_size, leaf_mode, stack_lds=stack_lds)


def gpu_cpq(h, queries):
    out = h.closest_point(dev(queries))
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    return o[:, 0].view(np.int32).copy(), o[:, 1:4].copy()


def tri_tol(verts, tris, queries, prims):
    """tol(T) per query for triangle prims[i] (0 where prims[i] < 0)."""
    out = np.zeros(len(prims))
    ok = prims >= 0
    p = verts[tris[prims[ok]]].astype(np.float64)
    e = [p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 2] - p[:, 1]]
    longest = np.sqrt(np.max([np.sum(x * x, axis=1) for x in e], axis=0))
    area2 = np.linalg.norm(np.cross(e[0], e[1]), axis=1)
    kappa = np.where(area2 > 0, longest ** 2 / np.maximum(area2, 1e-300), 1e30)
    reach = np.linalg.norm(queries[ok, :3].astype(np.float64) - p[:, 0], axis=1) + longest
    out[ok] = TOL * reach * (1.0 + np.minimum(kappa, 1e6))
    return out


def oracle_ref(orc, verts, tris, queries, brute=True, bvh=None):
    if brute:
        return orc.brute_closest_point(verts, tris, queries)
    bvh = bvh or orc.OracleBVH(verts, tris)
    return bvh.closest_point(queries)


def check_cpq(orc, verts, tris, queries, prim, duv, ref, min_graded=0.5):
    """Checks GPU results (prim[n], duv[n,3] f32) against the oracle's
    (prim1, duv1, top2, d2top2); returns the graded mask.  min_graded: the
    share of queries expected to have a unique nearest triangle (on a mesh,
    a nearest point on a shared edge or vertex ties its triangles)."""
    p1, duv1, top2, d2top2 = ref
    n = len(prim)
    r2 = queries[:, 3].astype(np.float64)
    t1 = tri_tol(verts, tris, queries, top2[:, 0])
    t2 = tri_tol(verts, tris, queries, top2[:, 1])
    d1 = np.sqrt(d2top2[:, 0])
    dsec = np.sqrt(d2top2[:, 1])
    with np.errstate(invalid="ignore"):
        sep = (top2[:, 1] < 0) | (dsec - d1 > t1 + t2)
        radius_clear = ~np.isfinite(r2) | (np.abs(d1 - np.sqrt(np.maximum(r2, 0))) > t1)
    graded = sep & radius_clear
    assert graded.mean() > min_graded
    bad = np.nonzero(graded & (prim != p1))[0]
    assert bad.size == 0, (f"{bad.size} graded queries differ, e.g. {bad[:5]}: gpu {prim[bad[:5]]} "
                           f"oracle {p1[bad[:5]]}")
    # misses: exactly the documented record
    miss = prim < 0
    assert np.isinf(duv[miss, 0]).all() and (duv[miss, 1:] == 0).all()
    # the returned triangle, wherever the query is graded or not
    hit = ~miss
    ex = orc.point_tri_f64(verts, tris, queries, prim)
    tg = tri_tol(verts, tris, queries, prim)
    dg = np.sqrt(ex[:, 0])
    # reported distance of that triangle
    err = np.abs(np.sqrt(duv[hit, 0].astype(np.float64)) - dg[hit])
    assert (err <= tg[hit]).all(), f"distance error {np.max(err / np.maximum(tg[hit], 1e-300))} x tol"
    # near-optimal: no farther than the nearest by more than the tolerances
    assert (dg[hit] <= d1[hit] + tg[hit] + t1[hit]).all()
    # within the radius (up to the tolerance)
    with np.errstate(invalid="ignore"):
        assert (dg[hit] <= np.sqrt(r2[hit]) + tg[hit]).all()
    # a miss only where no triangle is clearly inside the radius
    with np.errstate(invalid="ignore"):
        clearly_in = (top2[:, 0] >= 0) & (d1 + t1 < np.sqrt(np.maximum(r2, 0))) & (r2 >= 0)
    assert not (miss & clearly_in).any()
    # barycentric point against the exact nearest point of that triangle
    u, v = duv[hit, 1].astype(np.float64), duv[hit, 2].astype(np.float64)
    assert (u >= -1e-3).all() and (v >= -1e-3).all() and (u + v <= 1.001).all()
    pv = verts[tris[prim[hit]]].astype(np.float64)
    cg = (1 - u - v)[:, None] * pv[:, 0] + u[:, None] * pv[:, 1] + v[:, None] * pv[:, 2]
    ue, ve = ex[hit, 1], ex[hit, 2]
    ce = (1 - ue - ve)[:, None] * pv[:, 0] + ue[:, None] * pv[:, 1] + ve[:, None] * pv[:, 2]
    perr = np.linalg.norm(cg - ce, axis=1)
    assert (perr <= tg[hit]).all(), f"point error {np.max(perr / tg[hit])} x tol"
    return graded


def _queries(n, lo, hi, seed, finite_frac=0.0, r_hi=0.05):
    q = W.box_points(n, lo, hi, seed)
    if finite_frac > 0:
        rng = np.random.default_rng(seed + 7)
        fin = rng.uniform(size=n) < finite_frac
        q[fin, 3] = rng.uniform(0.0, r_hi, fin.sum()).astype(np.float32) ** 2
    return q


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("leaf_mode", ["compact", "indexed"])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_soup_closest_point(orc, layout, leaf_mode):
    w = W.soup_workload()
    v, t = w["verts"], w["tris"]
    q = _queries(4096, (-0.2, -0.2, -0.2), (1.2, 1.2, 1.2), 31, finite_frac=0.5)
    ref = oracle_ref(orc, v, t, q)
    prim, duv = gpu_cpq(gpu_build(v, t, layout, leaf_mode), q)
    graded = check_cpq(orc, v, t, q, prim, duv, ref)
    assert (prim < 0).sum() > 100 and (prim >= 0).sum() > 1000
    # graded results are the same bits on every layout and leaf mode
    p0, duv0 = gpu_cpq(gpu_build(v, t, "aabb2", "compact"), q)
    assert np.array_equal(prim[graded], p0[graded])
    assert np.array_equal(duv[graded].view(np.uint32), duv0[graded].view(np.uint32))


@pytest.mark.parametrize("layout", LAYOUTS)
def test_terrain_closest_point(orc, layout):
    w = W.terrain_workload(cells=96, width=8, height=8)
    v, t = w["verts"], w["tris"]
    q = _queries(4096, (0.0, 0.0, -0.1), (1.0, 1.0, 0.4), 32, finite_frac=0.3, r_hi=0.1)
    ref = oracle_ref(orc, v, t, q)
    prim, duv = gpu_cpq(gpu_build(v, t, layout), q)
    # above a bumpy heightfield the nearest point is mostly a peak vertex or
    # a ridge edge, shared by several triangles: few queries are graded
    check_cpq(orc, v, t, q, prim, duv, ref, min_graded=0.05)


def _small_spheres():
    return W.spheres_workload(n_rays=16, n_spheres=40, n_slivers=3000,
                              quota=((2, 14), (3, 12), (4, 8), (5, 4), (6, 2)))


@pytest.mark.parametrize("leaf_mode", ["compact", "indexed"])
@pytest.mark.parametrize("layout", LAYOUTS)
def test_spheres_closest_point(orc, layout, leaf_mode):
    w = _small_spheres()
    v, t = w["verts"], w["tris"]
    q = _queries(20000, (0, 0, 0), (1, 1, 1), 33, finite_frac=0.25)
    ref = oracle_ref(orc, v, t, q, brute=False)
    prim, duv = gpu_cpq(gpu_build(v, t, layout, leaf_mode), q)
    check_cpq(orc, v, t, q, prim, duv, ref)


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("leaf_size", [1, 7, 15])
def test_leaf_sizes(orc, layout, leaf_size):
    w = W.soup_workload(n_tris=3000)
    v, t = w["verts"], w["tris"]
    q = _queries(3000, (-0.1, -0.1, -0.1), (1.1, 1.1, 1.1), 34)
    ref = oracle_ref(orc, v, t, q)
    prim, duv = gpu_cpq(gpu_build(v, t, layout, leaf_size=leaf_size), q)
    check_cpq(orc, v, t, q, prim, duv, ref)


@pytest.mark.parametrize("layout", LAYOUTS)
def test_edge_cases(orc, layout):
    """Points on vertices and edges (distance exactly 0), duplicate triangles
    (lowest id wins), the radius bound at equality, zero / negative / NaN
    radii and non-finite points, an empty query batch, one triangle."""
    base = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
    v = np.concatenate([base + [0.0, 0.0, 1.0], base, base, base + [3.0, 0.0, 0.0]]).astype(np.float32)
    t = np.arange(12, dtype=np.int32).reshape(4, 3)
    inf, nan = np.float32(np.inf), np.float32(np.nan)
    q = np.array([[0, 0, 0, inf],          # on a vertex of the duplicated pair -> id 1, d2 0
                  [0.5, 0, 0, 0],          # on an edge, zero radius -> id 1, d2 0
                  [0.25, 0.25, 2, 1],      # d2 = 1 to id 0 exactly at the radius
                  [0.25, 0.25, 2, 0.99],   # just outside -> none
                  [0.25, 0.25, 0.5, -1],   # negative radius -> none
                  [0.25, 0.25, 0.5, nan],  # NaN radius -> none
                  [nan, 0, 0, inf],        # non-finite point -> none
                  [inf, 0, 0, inf],
                  [3.2, 0.2, 0.0, inf]],   # on triangle 3's face
                 np.float32)
    h = gpu_build(v, t, layout, leaf_size=1)
    prim, duv = gpu_cpq(h, q)
    assert list(prim) == [1, 1, 0, -1, -1, -1, -1, -1, 3]
    assert duv[0, 0] == 0 and duv[1, 0] == 0 and duv[2, 0] == 1.0 and duv[8, 0] <= 1e-12
    assert np.isinf(duv[3:8, 0]).all() and (duv[3:8, 1:] == 0).all()
    np.testing.assert_array_equal(duv[1, 1:], [0.5, 0.0])
    empty = h.closest_point(dev(np.zeros((0, 4), np.float32)))
    assert empty.shape == (0, 4)
    one = gpu_build(base, np.array([[0, 1, 2]], np.int32), layout)
    p1, d1 = gpu_cpq(one, np.array([[0.25, 0.25, 3, inf]], np.float32))
    assert p1[0] == 0 and d1[0, 0] == 9.0


@pytest.mark.parametrize("layout", LAYOUTS)
def test_stack_depths_agree_and_fallback_is_exact(orc, layout):
    """Leaf size 1 makes deep trees; with an 8-entry LDS ring many queries
    spill and some reach the deep-stack fallback pass.  Results must be
    identical for 8, 16 and 32 entries and the default (0: 8 for the wide
    layouts' query, 16 for the binary ones) and match the oracle."""
    w = _small_spheres()
    v, t = w["verts"], w["tris"]
    q = _queries(20000, (-0.5, -0.5, -0.5), (1.5, 1.5, 1.5), 35)
    res = []
    for sl in (8, 16, 32, 0):
        res.append(gpu_cpq(gpu_build(v, t, layout, leaf_size=1, stack_lds=sl), q))
    for p, d in res[1:]:
        assert np.array_equal(p, res[0][0]) and np.array_equal(d.view(np.uint32), res[0][1].view(np.uint32))
    ref = oracle_ref(orc, v, t, q, brute=False)
    check_cpq(orc, v, t, q, res[0][0], res[0][1], ref)


@pytest.mark.parametrize("layout", ["aabb2", "bvh8_q8"])
def test_counts_variant(orc, layout):
    w = _small_spheres()
    v, t = w["verts"], w["tris"]
    q = _queries(5000, (0, 0, 0), (1, 1, 1), 36)
    h = gpu_build(v, t, layout)
    out = h.closest_point(dev(q))
    out2, counts = h.closest_point_counts(dev(q))
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint32), out2.cpu().numpy().view(np.uint32))
    c = counts.cpu().numpy()
    assert (c[:, 0] >= 1).all() and (c[:, 1] >= 1).all()
    assert c[:, 1].sum() < 0.05 * len(q) * t.shape[0]   # the tree prunes


def _sample(n, k, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=min(k, n), replace=False))


@pytest.fixture(scope="module")
def terrain_full(orc):
    w = W.terrain_workload(width=8, height=8)
    return w, orc.OracleBVH(w["verts"], w["tris"])


@pytest.mark.parametrize("layout", LAYOUTS)
def test_terrain_full_size_sampled(orc, terrain_full, layout):
    """Full 2.1 M-triangle terrain and 2^20 queries in the scene's box (the
    benchmark's launch); a 4,096-query sample is checked against the oracle."""
    w, bvh = terrain_full
    v, t = w["verts"], w["tris"]
    lo, hi = v.min(axis=0), v.max(axis=0)
    q = W.box_points(1 << 20, lo, hi, 1001)
    prim, duv = gpu_cpq(gpu_build(v, t, layout), q)
    assert (prim >= 0).all()
    s = _sample(len(q), 4096, 3)
    check_cpq(orc, v, t, q[s], prim[s], duv[s], bvh.closest_point(q[s]), min_graded=0.05)


@pytest.fixture(scope="module")
def spheres_full(orc):
    w = W.spheres_workload(n_rays=16)
    return w, orc.OracleBVH(w["verts"], w["tris"])


@pytest.mark.parametrize("layout", LAYOUTS)
def test_spheres_full_size_sampled(orc, spheres_full, layout):
    """Full 4.05 M-triangle scene and 2^20 queries in its box; a 4,096-query
    sample is checked against the oracle."""
    w, bvh = spheres_full
    v, t = w["verts"], w["tris"]
    q = W.box_points(1 << 20, v.min(axis=0), v.max(axis=0), 1002)
    prim, duv = gpu_cpq(gpu_build(v, t, layout), q)
    s = _sample(len(q), 4096, 4)
    check_cpq(orc, v, t, q[s], prim[s], duv[s], bvh.closest_point(q[s]))
