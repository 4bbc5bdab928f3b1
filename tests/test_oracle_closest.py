"""Pins for the oracle's closest-hit, top-2 and any-hit searches.

Brute force is the plain definition of closest_hit (Fig. 4, App. G): the
minimum t over every triangle the MT test accepts, ties to the lowest id.  It
is pinned by hand-built scenes with known answers, by permutation
equivariance and by an FP64 check that no triangle is hit clearly earlier.
The median-split BVH traversal is pinned against brute force (exact equality:
conservative culling cannot change the answer) and by structural invariants.
"""
import math

import numpy as np
import pytest

from paper_2511_15028_amd import workloads as W


def _stack_scene(k=8, reverse=True):
    """k copies of one triangle at heights z = 1..k (ids in reverse order)."""
    base = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
    verts = []
    zs = list(range(k, 0, -1)) if reverse else list(range(1, k + 1))
    for z in zs:
        v = base.copy()
        v[:, 2] = z
        verts.append(v)
    verts = np.concatenate(verts)
    tris = np.arange(3 * k, dtype=np.int32).reshape(k, 3)
    return verts, tris, zs


def test_brute_force_picks_nearest_of_stacked_triangles(orc):
    verts, tris, zs = _stack_scene(8)
    rays = W.make_rays(np.array([[0.2, 0.3, 0.0], [0.2, 0.3, 10.0], [0.2, 0.3, 4.5], [2.0, 2.0, 0.0]]),
                       np.array([[0, 0, 1.0], [0, 0, -1.0], [0, 0, 1.0], [0, 0, 1.0]]))
    prim, tuv = orc.brute_closest(verts, tris, rays)
    assert prim[0] == zs.index(1) and tuv[0, 0] == 1.0
    assert prim[1] == zs.index(8) and tuv[1, 0] == 2.0
    assert prim[2] == zs.index(5) and tuv[2, 0] == 0.5
    assert prim[3] == -1 and tuv[3, 0] == math.inf and tuv[3, 1] == 0 and tuv[3, 2] == 0
    np.testing.assert_array_equal(tuv[0, 1:], np.float32([0.2, 0.3]))


def test_brute_force_tie_goes_to_lowest_id(orc):
    base = np.array([[0, 0, 1], [1, 0, 1], [0, 1, 1]], np.float32)
    verts = np.concatenate([base + [5, 5, 0], base, base, base + [0, 0, 3]]).astype(np.float32)
    tris = np.arange(12, dtype=np.int32).reshape(4, 3)
    rays = W.make_rays(np.array([[0.25, 0.25, 0.0]]), np.array([[0, 0, 1.0]]))
    prim, tuv = orc.brute_closest(verts, tris, rays)
    assert prim[0] == 1
    prim2, t2 = orc.brute_top2(verts, tris, rays)
    assert tuple(prim2[0]) == (1, 2) and tuple(t2[0]) == (1.0, 1.0)
    # tmax below the first hit -> miss; top-2 runner-up distinct and ordered
    rays[0, 7] = 0.5
    prim, _ = orc.brute_closest(verts, tris, rays)
    assert prim[0] == -1


def test_brute_force_permutation_equivariance(orc):
    w = W.soup_workload(n_tris=512, res=32)
    prim, tuv = orc.brute_closest(w["verts"], w["tris"], w["rays"])
    perm = np.random.default_rng(3).permutation(512)
    prim_p, tuv_p = orc.brute_closest(w["verts"], w["tris"][perm], w["rays"])
    hit = prim >= 0
    assert (prim_p >= 0).tolist() == hit.tolist()
    # the same triangle is found, under its new index (soup: no exact ties)
    np.testing.assert_array_equal(perm[prim_p[hit]], prim[hit])
    np.testing.assert_array_equal(tuv_p, tuv)


def test_brute_force_has_no_clearly_earlier_hit_in_fp64(orc):
    w = W.soup_workload(n_tris=256, res=16)
    verts, tris, rays = w["verts"].astype(np.float64), w["tris"], w["rays"]
    prim, tuv = orc.brute_closest(w["verts"], tris, rays)
    p = verts[tris]                                  # [N,3,3]
    for r in range(rays.shape[0]):
        o = rays[r, 0:3].astype(np.float64)
        d = rays[r, 4:7].astype(np.float64)
        A = np.stack([np.broadcast_to(d, (len(tris), 3)), p[:, 0] - p[:, 1], p[:, 0] - p[:, 2]], axis=2)
        ok = np.abs(np.linalg.det(A)) > 1e-9
        sol = np.full((len(tris), 3), np.nan)
        sol[ok] = np.linalg.solve(A[ok], (p[ok, 0] - o)[..., None])[..., 0]
        t, u, v = sol[:, 0], sol[:, 1], sol[:, 2]
        m = 1e-4
        clear = ok & (u > m) & (v > m) & (u + v < 1 - m) & (t > m)
        if prim[r] < 0:
            assert not clear.any()
        else:
            assert not (clear & (t < tuv[r, 0] * (1 - 1e-4))).any()
            # the reported t is the FP64 t of the reported triangle within rounding
            assert abs(t[prim[r]] - tuv[r, 0]) <= 1e-5 * t[prim[r]]


@pytest.mark.parametrize("scene", ["soup", "terrain", "spheres"])
def test_bvh_equals_brute_force(orc, scene):
    if scene == "soup":
        w = W.soup_workload()
        rays = w["rays"]
    elif scene == "terrain":
        w = W.terrain_workload(cells=48, width=96, height=54)
        rays = w["rays"]
    else:
        w = W.spheres_workload(n_rays=3000, n_spheres=12, n_slivers=400,
                               quota=((2, 6), (3, 4), (4, 2)))
        rays = np.concatenate([w["rays"], w["shadow"]])
    verts, tris = w["verts"], w["tris"]
    bp, btuv = orc.brute_closest(verts, tris, rays)
    bvh = orc.OracleBVH(verts, tris)
    p, tuv = bvh.trace(rays, orc.CLOSEST)
    np.testing.assert_array_equal(p, bp)
    np.testing.assert_array_equal(tuv, btuv)
    # top-2 agrees with brute force top-2
    b2p, b2t = orc.brute_top2(verts, tris, rays)
    p1, _, p2, t2 = bvh.trace(rays, orc.TOP2)
    np.testing.assert_array_equal(p1, b2p[:, 0])
    np.testing.assert_array_equal(p2, b2p[:, 1])
    np.testing.assert_array_equal(t2, b2t[:, 1])
    # any-hit: occluded iff the closest hit exists
    pa, tuva = bvh.trace(rays, orc.ANY)
    np.testing.assert_array_equal(pa >= 0, bp >= 0)
    hit = pa >= 0
    assert (tuva[hit, 0] <= rays[hit, 7]).all()
    # the any-hit occluder is a genuine hit: its t is at least the closest t
    assert (tuva[hit, 0] >= btuv[hit, 0]).all()
    assert (bp >= 0).sum() > 0.05 * len(rays)


def test_bvh_structure(orc):
    w = W.spheres_workload(n_rays=16, n_spheres=8, n_slivers=300, quota=((2, 4), (3, 3), (4, 1)))
    verts, tris = w["verts"], w["tris"]
    bvh = orc.OracleBVH(verts, tris)
    boxes, links, perm = bvh.export()
    assert sorted(perm.tolist()) == list(range(len(tris)))
    n_leaves = 0
    covered = np.zeros(len(tris), np.int64)
    for i in range(len(boxes)):
        l, r, first, count = links[i]
        if l < 0:
            n_leaves += 1
            assert 1 <= count <= 4
            ids = perm[first:first + count]
            covered[ids] += 1
            pts = verts[tris[ids]].reshape(-1, 3)
            np.testing.assert_array_equal(boxes[i, 0:3], pts.min(0))
            np.testing.assert_array_equal(boxes[i, 3:6], pts.max(0))
        else:
            # a parent box is exactly the union of its children's boxes
            np.testing.assert_array_equal(boxes[i, 0:3], np.minimum(boxes[l, 0:3], boxes[r, 0:3]))
            np.testing.assert_array_equal(boxes[i, 3:6], np.maximum(boxes[l, 3:6], boxes[r, 3:6]))
            assert links[l][3] + links[r][3] == count
    assert (covered == 1).all()
    assert len(boxes) == 2 * n_leaves - 1
    assert bvh.depth < 64


def test_ambiguity_mask(orc):
    t1 = np.array([np.inf, 1.0, 1.0, 1.0, 2.0])
    p2 = np.array([-1, -1, 3, 3, 4])
    t2 = np.array([np.inf, np.inf, 1.0 + 5e-6, 1.0 + 2e-5, 2.0])
    np.testing.assert_array_equal(orc.ambiguity_mask(t1, p2, t2), [True, True, False, True, False])


def test_empty_inputs(orc):
    w = W.soup_workload(n_tris=8, res=4)
    bvh = orc.OracleBVH(w["verts"], w["tris"][:0])
    p, tuv = bvh.trace(w["rays"])
    assert (p == -1).all() and np.isinf(tuv[:, 0]).all()
    p, tuv = orc.brute_closest(w["verts"], w["tris"], w["rays"][:0])
    assert p.shape == (0,)
