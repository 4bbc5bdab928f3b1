"""Checks of the seeded scene and ray generators (sizes, determinism, ranges)."""
import numpy as np
import pytest

from paper_2511_15028_amd import workloads as W


def test_soup_sizes_and_determinism():
    a = W.soup_workload()
    b = W.soup_workload()
    assert a["tris"].shape == (1024, 3) and a["verts"].shape == (3072, 3)
    assert a["rays"].shape == (4096, 8)
    np.testing.assert_array_equal(a["verts"], b["verts"])
    c = W.soup_workload(seed=7)
    assert not np.array_equal(a["verts"], c["verts"])
    np.testing.assert_array_equal(a["tris"].reshape(-1), np.arange(3072))


def test_rays_are_unit_and_well_formed():
    for r in (W.soup_camera_rays(), W.terrain_camera_rays(64, 36), W.uniform_rays(1000, 3)):
        np.testing.assert_allclose(np.linalg.norm(r[:, 4:7], axis=1), 1.0, rtol=1e-6)
        assert (r[:, 3] == 0).all()
        assert np.isinf(r[:, 7]).all()
    s = W.shadow_rays(1000, 3)
    u = W.uniform_rays(1000, 3)
    np.testing.assert_array_equal(s[:, 0:3], u[:, 0:3])  # shared origins
    assert (s[:, 7] > 0).all() and (s[:, 7] <= np.sqrt(3) + 1e-6).all()


def test_soup_camera_center_rays_point_forward():
    r = W.soup_camera_rays(64, 64)
    np.testing.assert_array_equal(r[:, 0:3], np.tile([0.5, 0.5, -1.0], (4096, 1)))
    # pixel (31.5, 31.5) is the optical axis: the four central rays are symmetric
    c = r.reshape(64, 64, 8)[31:33, 31:33, 4:7]
    np.testing.assert_allclose(np.abs(c[..., 0]), np.abs(c[0, 0, 0]), rtol=1e-6)
    assert (c[..., 2] > 0.999).all()
    # corner ray makes 30 degrees with the axis in x and in y (60 degree FOV)
    corner = r[0, 4:7].astype(np.float64)
    np.testing.assert_allclose(abs(corner[0] / corner[2]), np.tan(np.radians(30)) * 63 / 64, rtol=1e-5)


def test_terrain_full_size_counts():
    verts, tris = W.terrain_scene(1024)
    assert tris.shape == (2_097_152, 3) and verts.shape == (1_050_625, 3)
    assert verts[:, 2].min() >= 0.0 and verts[:, 2].max() < 0.2
    assert tris.min() == 0 and tris.max() == verts.shape[0] - 1
    rays = W.terrain_camera_rays()
    assert rays.shape == (2_073_600, 8)
    # image footprint at z = 0 stays inside the unit square
    t0 = -rays[:, 2] / rays[:, 6]
    xy = rays[:, 0:2] + t0[:, None] * rays[:, 4:6]
    assert xy.min() > 0.0 and xy.max() < 1.0


@pytest.mark.parametrize("level", [0, 1, 2, 3, 7])
def test_icosphere_counts_and_topology(level):
    v, f = W.icosphere(level)
    assert f.shape[0] == 20 * 4 ** level and v.shape[0] == 10 * 4 ** level + 2
    e = np.unique(np.sort(np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]]), axis=1), axis=0)
    assert v.shape[0] - e.shape[0] + f.shape[0] == 2      # Euler characteristic of a sphere
    np.testing.assert_allclose(np.linalg.norm(v, axis=1), 1.0, rtol=1e-12)


def test_sphere_cluster_full_size_counts():
    verts, tris = W.sphere_cluster_scene()
    assert tris.shape == (4_051_040, 3) and verts.shape == (2_276_544, 3)
    assert tris.max() == verts.shape[0] - 1


def test_diff_workload_sizes():
    w = W.diff_workload()
    assert w["tris"].shape == (327_680, 3) and w["verts"].shape == (163_842, 3)
    assert w["rays"].shape == (1_048_576, 8) and w["weights"].shape == (1_048_576, 3)
    r = np.linalg.norm(w["verts"], axis=1)
    assert r.min() >= 0.95 and r.max() <= 1.05


def test_bounce_rays_leave_the_surface_on_the_incoming_side(orc):
    w = W.terrain_workload(cells=32, width=40, height=30)
    prim, tuv = orc.brute_closest(w["verts"], w["tris"], w["rays"])
    # Moller-Trumbore is not watertight: a ray running exactly along the
    # shared (0,0)-(1,1) diagonal of the cells (d.x == d.y from the grid
    # vertex under the camera) can slip between both triangles.  Every other
    # primary ray hits.
    miss = prim < 0
    d = w["rays"][:, 4:7]
    assert (d[miss, 0] == d[miss, 1]).all() and miss.sum() <= 4
    b, src = W.bounce_rays(w["rays"], prim, tuv[:, 0], w["verts"], w["tris"], seed=5)
    assert b.shape == (int((~miss).sum()), 8) and (src == np.nonzero(~miss)[0]).all()
    np.testing.assert_allclose(np.linalg.norm(b[:, 4:7], axis=1), 1.0, rtol=1e-6)
    # each bounce leaves on the side the primary ray came from
    v = w["verts"].astype(np.float64)[w["tris"][prim[src]]]
    ng = np.cross(v[:, 1] - v[:, 0], v[:, 2] - v[:, 0])
    din = w["rays"][src, 4:7].astype(np.float64)
    assert (np.sum(ng * din, 1) * np.sum(ng * b[:, 4:7], 1) < 0).all()
    assert (np.sum(ng * din, 1) * np.sum(ng * (b[:, 0:3] - v[:, 0]), 1) < 0).all()
    b2, _ = W.bounce_rays(w["rays"], prim, tuv[:, 0], w["verts"], w["tris"], seed=5)
    np.testing.assert_array_equal(b, b2)
