"""Pins for the oracle's closest-point query (App. G "Closest Point Query").

The plain definition: the triangle nearest to a query point (ties to the
lowest id) among those within the squared radius r2, its squared distance and
the barycentrics of its nearest point.  The FP64 point-triangle distance is
pinned by closed forms, by the projection inequality (c is the nearest point
of a convex set S to q iff c lies in S and (q - c).(x - c) <= 0 for every x
in S; for a triangle it suffices to check the three vertices), and by dense
sampling of the triangle; the search by hand-built scenes (ties, the radius
bound at equality, top-2), permutation equivariance, and the BVH search
against exhaustive search (exact equality).
"""
import math

import numpy as np
import pytest

from paper_2511_15028_amd import workloads as W

INF = math.inf


def _unit_tri():
    return (np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32),
            np.array([[0, 1, 2]], np.int32))


def _q(points, r2=INF):
    p = np.asarray(points, np.float32).reshape(-1, 3)
    return np.concatenate([p, np.full((p.shape[0], 1), r2, np.float32)], axis=1)


@pytest.mark.parametrize("q, d2, u, v", [
    ((0.25, 0.25, 2.0), 4.0, 0.25, 0.25),     # above the face: distance to the plane
    ((0.25, 0.25, -3.0), 9.0, 0.25, 0.25),    # below it (two-sided)
    ((-1.0, -1.0, 0.0), 2.0, 0.0, 0.0),       # vertex region of p0
    ((2.0, -1.0, 0.0), 2.0, 1.0, 0.0),        # vertex region of p1
    ((-0.5, 3.0, 1.0), 5.25, 0.0, 1.0),       # vertex region of p2
    ((0.5, -2.0, 3.0), 13.0, 0.5, 0.0),       # edge p0p1
    ((-3.0, 0.25, 0.0), 9.0, 0.0, 0.25),      # edge p0p2
    ((1.0, 1.0, 0.0), 0.5, 0.5, 0.5),         # edge p1p2 (hypotenuse midpoint)
    ((0.0, 0.0, 0.0), 0.0, 0.0, 0.0),         # on a vertex
    ((0.5, 0.0, 0.0), 0.0, 0.5, 0.0),         # on an edge
])
def test_point_triangle_closed_forms(orc, q, d2, u, v):
    verts, tris = _unit_tri()
    prim, duv, top2, d2top2 = orc.brute_closest_point(verts, tris, _q(q))
    assert prim[0] == 0
    assert duv[0, 0] == pytest.approx(d2, abs=1e-15)
    assert duv[0, 1] == pytest.approx(u, abs=1e-15) and duv[0, 2] == pytest.approx(v, abs=1e-15)
    assert tuple(top2[0]) == (0, -1) and d2top2[0, 1] == INF
    fixed = orc.point_tri_f64(verts, tris, _q(q), np.array([0], np.int32))
    np.testing.assert_array_equal(fixed[0], duv[0])


def test_degenerate_triangles_reduce_to_segments_and_points(orc):
    verts = np.array([[0, 0, 0], [2, 0, 0], [1, 0, 0],      # collinear: segment [0,2] on x
                      [5, 5, 5], [5, 5, 5], [5, 5, 5]], np.float32)  # a single point
    tris = np.array([[0, 1, 2], [3, 4, 5]], np.int32)
    qs = _q([(1.0, 1.0, 0.0), (3.0, 0.0, 0.0), (5.0, 5.0, 7.0)])
    out = orc.point_tri_f64(verts, tris, qs, np.array([0, 0, 1], np.int32))
    assert out[0, 0] == pytest.approx(1.0, abs=1e-15)
    assert out[1, 0] == pytest.approx(1.0, abs=1e-15)
    assert out[2, 0] == pytest.approx(4.0, abs=1e-15)
    # the reported barycentrics reconstruct the nearest point
    for i, prim in enumerate((0, 0, 1)):
        p = verts[tris[prim]].astype(np.float64)
        c = (1 - out[i, 1] - out[i, 2]) * p[0] + out[i, 1] * p[1] + out[i, 2] * p[2]
        assert np.sum((qs[i, :3] - c) ** 2) == pytest.approx(out[i, 0], abs=1e-14)


def _random_tris(rng, n, kind):
    p0 = rng.uniform(-1, 1, (n, 3))
    if kind == "plain":
        p1 = p0 + rng.uniform(-1, 1, (n, 3))
        p2 = p0 + rng.uniform(-1, 1, (n, 3))
    elif kind == "sliver":
        a = rng.normal(size=(n, 3))
        a /= np.linalg.norm(a, axis=1, keepdims=True)
        b = rng.normal(size=(n, 3))
        b -= np.sum(a * b, axis=1, keepdims=True) * a
        b /= np.linalg.norm(b, axis=1, keepdims=True)
        p1 = p0 + a
        p2 = p0 + 0.5 * a + 1e-3 * b
    else:  # obtuse
        p1 = p0 + np.array([1.0, 0, 0])
        p2 = p0 + np.array([0.5, 0.05, 0.02])
    return np.stack([p0, p1, p2], axis=1).astype(np.float32)


@pytest.mark.parametrize("kind", ["plain", "sliver", "obtuse"])
def test_projection_inequality(orc, kind):
    """The reported point lies in the triangle, its squared distance is the
    reported one, and no vertex direction leads closer: this characterises
    the unique nearest point, whatever method computed it."""
    rng = np.random.default_rng(11)
    n = 4000
    tv = _random_tris(rng, n, kind)
    verts = tv.reshape(-1, 3)
    tris = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    # query points near (and in the plane of) each triangle and far from it
    centre = tv.astype(np.float64).mean(axis=1)
    scale = rng.choice([1e-3, 0.1, 1.0, 10.0], n)[:, None]
    q = (centre + scale * rng.normal(size=(n, 3))).astype(np.float32)
    out = orc.point_tri_f64(verts, tris, _q(q), np.arange(n, dtype=np.int32))
    d2, u, v = out[:, 0], out[:, 1], out[:, 2]
    assert np.all(u >= 0) and np.all(v >= 0) and np.all(u + v <= 1 + 1e-15)
    p = tv.astype(np.float64)
    c = (1 - u - v)[:, None] * p[:, 0] + u[:, None] * p[:, 1] + v[:, None] * p[:, 2]
    w = q.astype(np.float64) - c
    s2 = 1.0 + np.max(np.abs(p), axis=(1, 2)) ** 2 + np.max(np.abs(q), axis=1) ** 2
    np.testing.assert_allclose(np.sum(w * w, axis=1), d2, rtol=1e-12, atol=1e-15)
    # FP64 rounding of the 2x2 solve grows with the squared condition number
    # kappa = (longest edge)^2 / |e1 x e2| of the triangle
    e = [p[:, 1] - p[:, 0], p[:, 2] - p[:, 0], p[:, 2] - p[:, 1]]
    longest2 = np.max([np.sum(x * x, axis=1) for x in e], axis=0)
    kappa = longest2 / np.linalg.norm(np.cross(e[0], e[1]), axis=1)
    tol = 1e-14 * (1.0 + kappa ** 2) * s2
    for k in range(3):
        ineq = np.sum(w * (p[:, k] - c), axis=1)
        assert np.all(ineq <= tol), f"vertex {k}: max {np.max(ineq / tol)} of the tolerance"


def test_dense_sampling_brackets_the_distance(orc):
    """min over a barycentric grid of step h is within h * (longest edge) of
    the exact distance, and never below it."""
    rng = np.random.default_rng(12)
    n, m = 40, 200
    tv = _random_tris(rng, n, "plain")
    verts = tv.reshape(-1, 3)
    tris = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    q = rng.uniform(-2, 2, (n, 3)).astype(np.float32)
    out = orc.point_tri_f64(verts, tris, _q(q), np.arange(n, dtype=np.int32))
    i, j = np.meshgrid(np.arange(m + 1), np.arange(m + 1), indexing="ij")
    keep = i + j <= m
    a, b = (i[keep] / m), (j[keep] / m)
    for k in range(n):
        p = tv[k].astype(np.float64)
        pts = (1 - a - b)[:, None] * p[0] + a[:, None] * p[1] + b[:, None] * p[2]
        dmin = np.sqrt(np.min(np.sum((pts - q[k].astype(np.float64)) ** 2, axis=1)))
        edge = max(np.linalg.norm(p[1] - p[0]), np.linalg.norm(p[2] - p[0]), np.linalg.norm(p[2] - p[1]))
        d = math.sqrt(out[k, 0])
        assert d <= dmin + 1e-12
        assert d >= dmin - edge / m - 1e-12


def _stacked():
    """Four copies of the unit triangle at z = 3, 1, 1, 2 (ids 0..3)."""
    base, _ = _unit_tri()
    verts = np.concatenate([base + [0, 0, z] for z in (3.0, 1.0, 1.0, 2.0)]).astype(np.float32)
    return verts, np.arange(12, dtype=np.int32).reshape(4, 3)


def test_search_nearest_ties_and_radius(orc):
    verts, tris = _stacked()
    q = np.array([[0.25, 0.25, 0.0, INF],     # nearest z=1: ids 1 and 2 tie -> 1
                  [0.25, 0.25, 5.0, INF],     # nearest z=3 (id 0), runner-up z=2 (id 3)
                  [0.25, 0.25, 0.0, 1.0],     # radius exactly the distance: inclusive
                  [0.25, 0.25, 0.0, 0.99],    # radius below it: none
                  [0.25, 0.25, 1.0, 0.0]],    # on the surface, zero radius
                 np.float32)
    prim, duv, top2, d2top2 = orc.brute_closest_point(verts, tris, q)
    assert list(prim) == [1, 0, 1, -1, 1]
    assert duv[0, 0] == 1.0 and duv[1, 0] == 4.0 and duv[2, 0] == 1.0 and duv[4, 0] == 0.0
    assert tuple(duv[3]) == (INF, 0.0, 0.0)
    assert tuple(top2[0]) == (1, 2) and tuple(d2top2[0]) == (1.0, 1.0)
    assert tuple(top2[1]) == (0, 3) and tuple(d2top2[1]) == (4.0, 9.0)
    assert tuple(top2[3]) == (1, 2)          # reported regardless of the radius
    np.testing.assert_array_equal(duv[0, 1:], [0.25, 0.25])


def test_search_permutation_equivariance(orc):
    w = W.soup_workload(n_tris=300)
    rng = np.random.default_rng(13)
    q = _q(rng.uniform(-0.2, 1.2, (500, 3)))
    prim, duv, _, _ = orc.brute_closest_point(w["verts"], w["tris"], q)
    perm = rng.permutation(w["tris"].shape[0])
    prim_p, duv_p, _, _ = orc.brute_closest_point(w["verts"], w["tris"][perm], q)
    np.testing.assert_array_equal(perm[prim_p], prim)
    np.testing.assert_array_equal(duv_p[:, 0], duv[:, 0])


@pytest.mark.parametrize("scene", ["soup", "spheres"])
def test_bvh_search_equals_exhaustive(orc, scene):
    if scene == "soup":
        verts, tris = W.soup_scene(2000, seed=21)
    else:
        verts, tris = W.sphere_cluster_exact(3000, seed=22)
    rng = np.random.default_rng(14)
    n = 3000
    q = np.empty((n, 4), np.float32)
    q[:, :3] = rng.uniform(-0.3, 1.3, (n, 3))
    q[:, 3] = np.where(rng.uniform(size=n) < 0.5, INF, rng.uniform(0, 0.01, n))
    ref = orc.brute_closest_point(verts, tris, q)
    b = orc.OracleBVH(verts, tris)
    got = b.closest_point(q)
    for r, g in zip(ref, got):
        np.testing.assert_array_equal(g, r)
    assert np.any(ref[0] < 0) and np.any(ref[0] >= 0)
