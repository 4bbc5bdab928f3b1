"""bvh_trace_noalloc (the allocation-free trace entry point) against bvh_trace.

Both calls trace the same rays through the same handle; the closest hit is
unique under the (t, prim id) order and both paths evaluate the same FP32
ray/triangle arithmetic, so the hits must agree bit for bit.  Each case runs
two calls in a row on the fixed per-GPU work area, the second with fewer
rays, so a header left over from the first call would show.  A small LDS
stack (8 entries) on the binary layout sends deep rays through the fallback
pass that uses the fixed area's list and deep stacks."""
import ctypes

import numpy as np
import pytest

from paper_2511_15028_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def B():
    from paper_2511_15028_amd import bvh
    return bvh


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def scene():
    import oracle
    w = W.terrain_workload(cells=128, width=192, height=108)
    # bounce rays from the camera hits of the plain brute-force definition
    # (not from the code under test)
    prim, tuv = oracle.brute_closest(w["verts"], w["tris"], w["rays"])
    b, _ = W.bounce_rays(w["rays"], prim, tuv[:, 0], w["verts"], w["tris"], seed=11)
    rays = np.concatenate([w["rays"], b, W.uniform_rays(8192, seed=12)], axis=0)
    return dev(w["verts"]), dev(w["tris"]), dev(rays)


def both(h, rays, mode):
    ref = h.trace(rays, mode)
    out = torch.full_like(ref, float("nan"))
    h.trace_noalloc(rays, out, mode)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


@pytest.mark.parametrize("layout,stack_lds", [("aabb2", 8), ("aabb2", 16), ("bvh4", 8),
                                              ("bvh8_q8", 16), ("pbrt_q16", 8), ("sg_eq", 32)])
def test_noalloc_matches_trace_closest(scene, layout, stack_lds):
    verts, tris, rays = scene
    h = B().build(verts, tris, layout, stack_lds=stack_lds)
    n = rays.shape[0]
    for m in (n, n // 3 + 17):  # second call smaller, ragged
        ref, out = both(h, rays[:m], 0)
        assert np.array_equal(ref.view(np.int32), out.view(np.int32)), \
            f"{layout} sl={stack_lds} n={m}: hits differ"
    h.close()


@pytest.mark.parametrize("layout,stack_lds", [("aabb2", 8), ("bvh4", 8), ("bvh8_q8", 16)])
def test_noalloc_matches_trace_any_hit(orc, scene, layout, stack_lds):
    """Any-hit queries: whether a ray is occluded is unique and must agree;
    which occluder is reported depends on the traversal order, so each one
    is checked to be a genuine hit of that ray (the oracle's test of the ray
    against that triangle gives exactly the reported t, u, v)."""
    verts, tris, rays = scene
    h = B().build(verts, tris, layout, stack_lds=stack_lds)
    v, t = verts.cpu().numpy(), tris.cpu().numpy()
    n = rays.shape[0]
    for m in (n, n // 3 + 17):
        ref, out = both(h, rays[:m], 1)
        pr, po = ref[:, 0].view(np.int32), out[:, 0].view(np.int32)
        assert np.array_equal(pr >= 0, po >= 0)
        occ = np.nonzero(po >= 0)[0]
        ok, tuv = orc.mt_fixed(v, t, rays[:m].cpu().numpy()[occ], po[occ])
        assert ok.all() and np.array_equal(tuv.view(np.uint32), out[occ, 1:4].view(np.uint32))
        miss = po < 0
        assert np.isinf(out[miss, 1]).all() and (out[miss, 2:4] == 0).all()
    h.close()


def test_noalloc_limits(scene):
    bvh = B()
    verts, tris, rays = scene
    L = bvh.lib()
    h = bvh.build(verts, tris, "bvh4")
    hits = torch.empty((4, 4), dtype=torch.float32, device="cuda")
    big = bvh.NOALLOC_MAX_RAYS + 1
    # the count is checked before any pointer is touched
    assert L.bvh_trace_noalloc(h.handle, rays.data_ptr(), big, hits.data_ptr(), 0, None) == bvh.EINVAL
    assert b"exceed" in L.bvh_last_error()
    assert L.bvh_trace_noalloc(h.handle, rays.data_ptr(), 0, hits.data_ptr(), 0, None) == bvh.OK
    assert L.bvh_trace_noalloc(None, rays.data_ptr(), 4, hits.data_ptr(), 0, None) == bvh.EINVAL
    h.close()
    hs = bvh.build(verts, tris, "shared_slab")
    assert L.bvh_trace_noalloc(hs.handle, rays.data_ptr(), 4, hits.data_ptr(), 0,
                               None) == bvh.EUNSUPPORTED
    hs.close()


def test_noalloc_full_camera_frame():
    """The largest ray set it accepts in one call at the terrain's full size:
    1920 x 1080 camera rays (below the 2^21 limit) on the 2.1 M-triangle
    terrain, against bvh_trace."""
    w = W.terrain_workload()
    verts, tris, rays = dev(w["verts"]), dev(w["tris"]), dev(w["rays"])
    assert rays.shape[0] <= B().NOALLOC_MAX_RAYS
    h = B().build(verts, tris, "bvh4")
    ref, out = both(h, rays, 0)
    assert np.array_equal(ref.view(np.int32), out.view(np.int32))
    h.close()
