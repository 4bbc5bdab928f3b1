"""GPU binned-SAH topology against the oracle's, through the C ABI.

Both sides take every decision (bins, costs, ties, partitions) in the same
f32 arithmetic, so the trees must be identical: the AABB2 layout (preorder,
left child first) with indexed leaves gives the GPU's tree and leaf order,
compared node by node with the oracle's preorder tree collapsed at the same
leaf size (ranges, split axes, exact boxes, the primitives of every leaf; the
GPU does not split below the leaf size, so only the order inside a leaf may
differ, and with leaf size 1 the permutations are equal).  Traversal on
SAH trees must match the oracle's hits like on LBVH trees.
"""
import numpy as np
import pytest

from paper_2511_15028_amd import workloads as W
from test_gpu_parity import check_closest, gpu_trace, oracle_ref, LAYOUTS, dev, B

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

AABB2_DT = np.dtype([("lo", "<f4", 3), ("hi", "<f4", 3), ("offset", "<u4"), ("meta", "<u4")])
SMALL = np.array([[0, 0, 0], [0.1, 0, 0], [0, 0.1, 0.05]], np.float32)


def sah_build(verts, tris, layout="aabb2", leaf_size=4, leaf_mode="compact"):
    return B().build(dev(verts), dev(tris), layout, leaf_size, leaf_mode, builder="sah")


def gpu_tree(verts, tris, leaf_size):
    """(nodes, leaf order) of the GPU's SAH tree as AABB2 preorder records."""
    h = sah_build(verts, tris, "aabb2", leaf_size, "indexed")
    st = h.stats()
    assert st["builder"] == 1
    nodes = np.frombuffer(h.read_buffer(0), AABB2_DT)
    perm = np.frombuffer(h.read_buffer(1), np.int32)
    h.close()
    return nodes, perm


def check_tree(orc, verts, tris, leaf_size):
    n = tris.shape[0]
    perm, nodes, boxes = orc.sah_build(verts, tris)
    rows = orc.collapse(nodes, leaf_size)
    g, gperm = gpu_tree(verts, tris, leaf_size)
    assert len(g) == len(rows)
    first = np.array([r[0] for r in rows])
    count = np.array([r[1] for r in rows])
    axis = np.array([r[2] for r in rows])
    leaf = np.array([r[4] for r in rows], bool)
    # every leaf holds the oracle's primitives (the GPU does not split below
    # the leaf size, so the order inside a leaf may differ)
    leaf_of = np.full(n, -1, np.int64)
    for k in np.nonzero(leaf)[0]:
        leaf_of[first[k]:first[k] + count[k]] = k
    assert (leaf_of >= 0).all()
    key_g = np.lexsort((gperm, leaf_of))
    key_o = np.lexsort((perm, leaf_of))
    np.testing.assert_array_equal(gperm[key_g], perm[key_o])
    if leaf_size == 1:
        np.testing.assert_array_equal(gperm, perm)
    src = np.array([r[5] for r in rows])
    ob = boxes[src]
    np.testing.assert_array_equal(g["lo"], ob[:, :3])
    np.testing.assert_array_equal(g["hi"], ob[:, 3:])
    gcnt = g["meta"] & 0xFFFF
    np.testing.assert_array_equal(gcnt > 0, leaf)
    np.testing.assert_array_equal(g["offset"][leaf], first[leaf])
    np.testing.assert_array_equal(gcnt[leaf], count[leaf])
    np.testing.assert_array_equal((g["meta"][~leaf] >> 16) & 3, axis[~leaf])
    # the right child of an interior node follows its left subtree
    idx = np.nonzero(~leaf)[0]
    for i in idx[:2000]:
        j = i + int(g["offset"][i])
        assert first[j] == first[i + 1] + count[i + 1]
    return len(g)


@pytest.mark.parametrize("n", [2, 3, 17, 64, 65, 66, 130, 1000, 5000])
def test_tree_matches_oracle_soup(orc, n):
    v, t = W.soup_scene(n, seed=60 + n)
    for leaf_size in (1, 4):
        check_tree(orc, v, t, leaf_size)


@pytest.mark.parametrize("scene", ["spheres", "terrain", "line", "coincident", "clusters"])
def test_tree_matches_oracle_scenes(orc, scene):
    rng = np.random.default_rng(7)
    if scene == "spheres":
        v, t = W.sphere_cluster_exact(20000, seed=61)
    elif scene == "terrain":
        w = W.terrain_workload(cells=120, width=4, height=4)
        v, t = w["verts"], w["tris"]
    elif scene == "line":      # balanced, crosses the per-wave finisher size many times
        offs = np.zeros((4096, 3))
        offs[:, 0] = np.arange(4096) * 2.0
        v = np.concatenate([SMALL + o for o in offs.astype(np.float32)]).astype(np.float32)
        t = np.arange(3 * 4096, dtype=np.int32).reshape(-1, 3)
    elif scene == "coincident":  # index-median splits in the level phase and the finisher
        v = np.tile(SMALL, (300, 1)).astype(np.float32)
        t = np.arange(900, dtype=np.int32).reshape(-1, 3)
    else:
        offs = np.concatenate([rng.uniform(0, 1, (3000, 3)), rng.uniform(0, 1, (500, 3)) + [50, 0, 0],
                               rng.uniform(0, 0.001, (700, 3)) + [0, 9, 0]])[rng.permutation(4200)]
        v = np.concatenate([SMALL * 0.01 + o for o in offs.astype(np.float32)]).astype(np.float32)
        t = np.arange(3 * 4200, dtype=np.int32).reshape(-1, 3)
    check_tree(orc, v, t, 1)
    check_tree(orc, v, t, 4)


def test_single_triangle_and_deterministic(orc):
    v, t = W.soup_scene(1, seed=3)
    g, perm = gpu_tree(v, t, 4)
    assert len(g) == 1 and list(perm) == [0]
    v, t = W.soup_scene(3000, seed=4)
    a = gpu_tree(v, t, 4)
    b = gpu_tree(v, t, 4)
    assert a[0].tobytes() == b[0].tobytes() and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("layout", LAYOUTS)
def test_trace_parity_on_sah_trees(orc, layout):
    w = W.soup_workload()
    v, t, rays = w["verts"], w["tris"], w["rays"]
    h = sah_build(v, t, layout, 4)
    prim, tuv = gpu_trace(h, rays)
    check_closest(orc, v, t, rays, prim, tuv, oracle_ref(orc, v, t, rays))
    ws = W.spheres_workload(n_rays=20000, n_spheres=40, n_slivers=3000,
                            quota=((2, 14), (3, 12), (4, 8), (5, 4), (6, 2)))
    h = sah_build(ws["verts"], ws["tris"], layout, 4)
    prim, tuv = gpu_trace(h, ws["rays"])
    check_closest(orc, ws["verts"], ws["tris"], ws["rays"], prim, tuv,
                  oracle_ref(orc, ws["verts"], ws["tris"], ws["rays"], brute=False))


def test_terrain_full_size_tree_and_sampled_trace(orc):
    """Full 2.1 M-triangle terrain: the GPU's SAH tree equals the oracle's
    (leaf size 4), and a 4,096-ray camera sample matches the oracle's hits."""
    w = W.terrain_workload()
    v, t = w["verts"], w["tris"]
    check_tree(orc, v, t, 4)
    h = sah_build(v, t, "bvh4", 4)
    prim, tuv = gpu_trace(h, w["rays"])
    s = np.sort(np.random.default_rng(5).choice(len(prim), 4096, replace=False))
    ref = orc.OracleBVH(v, t).trace(w["rays"][s], orc.TOP2)
    check_closest(orc, v, t, w["rays"][s], prim[s], tuv[s], ref)


def test_builder_argument(orc):
    v, t = W.soup_scene(10, seed=5)
    with pytest.raises(B().BVHError):
        B().build(dev(v), dev(t), "aabb2", builder=2)
