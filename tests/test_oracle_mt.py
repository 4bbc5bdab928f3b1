"""Pins for the oracle's FP32 Moller-Trumbore test (App. G, intersectsp_ray_tri_mt).

The pins do not retype the oracle's formula.  They use
  * rays whose answers are exactly representable (all intermediate values of
    the hand-built triangle are small dyadic rationals), read off geometry;
  * the paper's stated acceptance intervals (u, v >= 0 and u + v <= 1
    inclusive, 0 < t exclusive, t <= tmax inclusive) at their end points;
  * an FP64 solve of o + t d = (1-u-v) p0 + u p1 + v p2 by numpy.linalg.solve
    on random inputs, which catches a wrong sign, a swapped u/v, a dropped
    term or a transposed operand.
"""
import math

import numpy as np
import pytest

from paper_2511_15028_amd import workloads as W

INF = math.inf
# Triangle in the plane z = 1 with p0 at the right angle.
P0, P1, P2 = (0.0, 0.0, 1.0), (1.0, 0.0, 1.0), (0.0, 1.0, 1.0)
UP = (0.0, 0.0, 1.0)


def test_exact_hit_reads_barycentrics_of_p1_and_p2(orc):
    # hit point (0.25, 0.25, 1) = 0.5 p0 + 0.25 p1 + 0.25 p2, one unit along d
    assert orc.mt_f32((0.25, 0.25, 0.0), UP, INF, P0, P1, P2) == (1.0, 0.25, 0.25)
    # asymmetric point pins which weight is u: (0.5, 0.125, 1) = u p1 + v p2 + ...
    assert orc.mt_f32((0.5, 0.125, 0.0), UP, INF, P0, P1, P2) == (1.0, 0.5, 0.125)


def test_distance_is_in_units_of_direction_length(orc):
    # d of length 2: the same point is reached at t = 0.5
    assert orc.mt_f32((0.25, 0.25, 0.0), (0.0, 0.0, 2.0), INF, P0, P1, P2) == (0.5, 0.25, 0.25)
    # origin 3 below the plane
    assert orc.mt_f32((0.25, 0.25, -2.0), UP, INF, P0, P1, P2) == (3.0, 0.25, 0.25)


def test_two_sided(orc):
    # ray from above going down hits the same triangle
    assert orc.mt_f32((0.25, 0.5, 2.0), (0.0, 0.0, -1.0), INF, P0, P1, P2) == (1.0, 0.25, 0.5)
    # the flipped-winding copy hits with u and v exchanged
    assert orc.mt_f32((0.25, 0.5, 0.0), UP, INF, P0, P2, P1) == (1.0, 0.5, 0.25)


def test_parallel_ray_misses(orc):
    assert orc.mt_f32((0.25, 0.25, 1.0), (1.0, 0.0, 0.0), INF, P0, P1, P2) is None
    assert orc.mt_f32((-1.0, 0.25, 1.0), (1.0, 0.0, 0.0), INF, P0, P1, P2) is None


def test_behind_and_at_origin_miss(orc):
    assert orc.mt_f32((0.25, 0.25, 2.0), UP, INF, P0, P1, P2) is None  # t = -1
    assert orc.mt_f32((0.25, 0.25, 1.0), UP, INF, P0, P1, P2) is None  # t = 0 is excluded


def test_tmax_is_inclusive(orc):
    assert orc.mt_f32((0.25, 0.25, 0.0), UP, 1.0, P0, P1, P2) == (1.0, 0.25, 0.25)
    assert orc.mt_f32((0.25, 0.25, 0.0), UP, 0.99, P0, P1, P2) is None


def test_edges_and_vertices_are_inclusive(orc):
    assert orc.mt_f32((0.5, 0.5, 0.0), UP, INF, P0, P1, P2) == (1.0, 0.5, 0.5)   # u+v = 1
    assert orc.mt_f32((0.0, 0.0, 0.0), UP, INF, P0, P1, P2) == (1.0, 0.0, 0.0)   # p0
    assert orc.mt_f32((1.0, 0.0, 0.0), UP, INF, P0, P1, P2) == (1.0, 1.0, 0.0)   # p1
    assert orc.mt_f32((0.0, 1.0, 0.0), UP, INF, P0, P1, P2) == (1.0, 0.0, 1.0)   # p2
    assert orc.mt_f32((0.25, 0.0, 0.0), UP, INF, P0, P1, P2) == (1.0, 0.25, 0.0)  # edge v = 0


def test_just_outside_misses(orc):
    assert orc.mt_f32((0.5, 0.5 + 2.0 ** -10, 0.0), UP, INF, P0, P1, P2) is None
    assert orc.mt_f32((-(2.0 ** -10), 0.25, 0.0), UP, INF, P0, P1, P2) is None
    assert orc.mt_f32((0.25, -(2.0 ** -10), 0.0), UP, INF, P0, P1, P2) is None


def _solve64(o, d, p0, p1, p2):
    """t, u, v from o + t d = p0 + u (p1 - p0) + v (p2 - p0), by LU."""
    A = np.stack([d, p0 - p1, p0 - p2], axis=1)
    return np.linalg.solve(A, p0 - o)


def test_agrees_with_fp64_linear_solve_on_random_inputs(orc):
    rng = np.random.default_rng(5)
    checked_hit = checked_miss = 0
    for _ in range(4000):
        p = rng.uniform(-1, 1, (3, 3)).astype(np.float32)
        o = rng.uniform(-2, 2, 3).astype(np.float32)
        # aim near the triangle so that roughly half the rays hit
        tgt = p.mean(0) + rng.normal(0, 0.5, 3)
        d = (tgt - o).astype(np.float32)
        p64 = p.astype(np.float64)
        A = np.stack([d, p64[0] - p64[1], p64[0] - p64[2]], axis=1).astype(np.float64)
        if abs(np.linalg.det(A)) < 1e-3:
            continue
        t, u, v = _solve64(o.astype(np.float64), d.astype(np.float64), *p64)
        res = orc.mt_f32(o, d, INF, p[0], p[1], p[2])
        margin = 1e-3
        inside = u > margin and v > margin and u + v < 1 - margin and t > margin
        outside = u < -margin or v < -margin or u + v > 1 + margin or t < -margin
        if inside:
            assert res is not None
            cond = np.linalg.cond(A)
            tol = 64 * 2.0 ** -24 * cond
            assert abs(res[0] - t) <= tol * max(1.0, abs(t))
            assert abs(res[1] - u) <= tol
            assert abs(res[2] - v) <= tol
            checked_hit += 1
        elif outside:
            assert res is None
            checked_miss += 1
    assert checked_hit > 500 and checked_miss > 500


def test_tuv_f64_matches_linear_solve(orc):
    rng = np.random.default_rng(6)
    verts = rng.uniform(-1, 1, (300, 3))
    tris = np.arange(300, dtype=np.int32).reshape(100, 3)
    rays = np.zeros((100, 8))
    rays[:, 0:3] = rng.uniform(-2, 2, (100, 3))
    rays[:, 4:7] = rng.normal(size=(100, 3))
    prims = np.arange(100, dtype=np.int32)
    prims[7] = -1
    out = orc.tuv_f64(verts, tris, rays, prims)
    for i in range(100):
        if i == 7:
            assert np.isnan(out[i]).all()
            continue
        p = verts[tris[i]]
        ref = _solve64(rays[i, 0:3], rays[i, 4:7], p[0], p[1], p[2])
        np.testing.assert_allclose(out[i], ref, rtol=1e-9, atol=1e-9)


def test_mt_fixed_reproduces_the_search_and_rejects_misses(orc):
    """The per-ray test against a given triangle returns, at the exhaustive
    search's own primitives, exactly the search's (t, u, v); a ray given a
    triangle it does not meet, or no triangle, gets a miss."""
    w = W.soup_workload()
    v, t, rays = w["verts"], w["tris"], w["rays"]
    prim, tuv = orc.brute_closest(v, t, rays)
    hit, tuv2 = orc.mt_fixed(v, t, rays, prim)
    assert np.array_equal(hit, prim >= 0)
    assert np.array_equal(tuv2.view(np.uint32), tuv.view(np.uint32))
    # a triangle far behind the camera: every camera ray misses it
    v2 = np.concatenate([v, np.array([[0, 0, -5], [1, 0, -5], [0, 1, -5]], np.float32)])
    t2 = np.concatenate([t, np.array([[len(v), len(v) + 1, len(v) + 2]], np.int32)])
    hit, tuv3 = orc.mt_fixed(v2, t2, rays, np.full(len(rays), len(t), np.int32))
    assert not hit.any() and np.isinf(tuv3[:, 0]).all() and (tuv3[:, 1:] == 0).all()
    hit, _ = orc.mt_fixed(v, t, rays, np.full(len(rays), len(t) + 3, np.int32))
    assert not hit.any()
