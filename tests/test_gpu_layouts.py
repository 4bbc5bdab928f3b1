"""Round trip of the packed layouts: decode every node on the CPU (from the
record formats of include/bvh.h) and compare with the geometry.

  * every triangle appears in exactly one leaf, leaves hold 1..leaf_size;
  * every node is reachable exactly once from the root (a tree);
  * every box on the path to a leaf, dequantised with the exact fmaf of the
    header, contains the leaf's triangles (the paper's requirement that a
    quantised volume encloses its original);
  * f32 layouts store exact boxes: the leaf box equals the triangles' box;
  * compacted triangles are bit-copies of the input triangles.
"""
import numpy as np
import pytest

import layout_decode as LD
from paper_2511_15028_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

LAYOUTS = {"aabb2": LD.AABB2, "bvh4": LD.BVH4, "bvh8_q8": LD.BVH8_Q8, "bvh8_q16": LD.BVH8_Q16}


def _build(v, t, layout, leaf_mode="compact", leaf_size=4):
    from paper_2511_15028_amd import bvh
    return bvh.build(torch.from_numpy(v).cuda(), torch.from_numpy(t).cuda(), layout, leaf_size,
                     leaf_mode)


def _scenes():
    sp = W.spheres_workload(n_rays=1, n_spheres=30, n_slivers=2000,
                            quota=((2, 10), (3, 10), (4, 6), (5, 3), (6, 1)))
    te = W.terrain_workload(cells=40, width=2, height=2)
    so = W.soup_workload(n_tris=777, seed=8)
    return {"spheres": (sp["verts"], sp["tris"]), "terrain": (te["verts"], te["tris"]),
            "soup": (so["verts"], so["tris"])}


SCENES = _scenes()


@pytest.mark.parametrize("scene", list(SCENES))
@pytest.mark.parametrize("leaf_mode", ["compact", "indexed"])
@pytest.mark.parametrize("layout", list(LAYOUTS))
def test_round_trip(layout, leaf_mode, scene):
    from paper_2511_15028_amd import bvh
    v, t = SCENES[scene]
    leaf_size = 4
    h = _build(v, t, layout, leaf_mode, leaf_size)
    st = h.stats()
    lid = LAYOUTS[layout]
    nodes_bytes = h.read_buffer(bvh.BUF_NODES)
    assert len(nodes_bytes) == st["n_nodes"] * st["node_bytes"]
    nodes, leaves, visited = LD.walk(lid, nodes_bytes)
    assert (visited == 1).all(), "every node reachable exactly once"
    assert len(leaves) == st["n_leaves"]
    leaf_raw = h.read_buffer(bvh.BUF_LEAF)
    if leaf_mode == "compact":
        tri = np.frombuffer(leaf_raw, dtype=LD.TRI_DT)
        order = tri["prim"]
        pts = v[t[order]]
        # p0 is a bit copy; the edges are the f32 differences p0 - p1, p2 - p0
        assert np.array_equal(tri["p0"].view(np.uint32), pts[:, 0].view(np.uint32))
        assert np.array_equal(tri["e1"].view(np.uint32), (pts[:, 0] - pts[:, 1]).view(np.uint32))
        assert np.array_equal(tri["e2"].view(np.uint32), (pts[:, 2] - pts[:, 0]).view(np.uint32))
    else:
        order = np.frombuffer(leaf_raw, dtype=np.int32)
        pts = v[t[order]]
    assert sorted(order.tolist()) == list(range(len(t)))
    covered = np.zeros(len(t), np.int64)
    for first, n, path in leaves:
        assert 1 <= n <= leaf_size
        covered[order[first:first + n]] += 1
        p = pts[first:first + n].reshape(-1, 3)
        lo, hi = p.min(0), p.max(0)
        for box in path:
            assert (box[0:3] <= lo).all() and (box[3:6] >= hi).all(), (box, lo, hi)
        if lid in (LD.AABB2, LD.BVH4):
            # f32 layouts: the innermost box is exactly the leaf's box
            assert np.array_equal(path[-1][0:3], lo) and np.array_equal(path[-1][3:6], hi)
    assert (covered == 1).all()
    assert st["max_stack"] >= 1 and st["depth"] >= 2
    assert st["nodes_buffer_bytes"] == st["n_nodes"] * {0: 32, 1: 128, 2: 128, 3: 160}[lid]


@pytest.mark.parametrize("layout", list(LAYOUTS))
def test_quantised_boxes_are_tight(layout):
    """The builder picks the tightest enclosing q: moving any child plane one
    step inward would cut into the child (checked on the decoded nodes)."""
    lid = LAYOUTS[layout]
    if lid not in (LD.BVH8_Q8, LD.BVH8_Q16):
        pytest.skip("f32 layout")
    from paper_2511_15028_amd import bvh
    v, t = SCENES["spheres"]
    h = _build(v, t, layout)
    nodes, leaves, _ = LD.walk(lid, h.read_buffer(bvh.BUF_NODES))
    order = np.frombuffer(h.read_buffer(bvh.BUF_LEAF), dtype=LD.TRI_DT)
    pts = v[t[order["prim"]]]
    qmax = 255 if lid == LD.BVH8_Q8 else 65535
    # exact child boxes of leaf children: compare with the q one step tighter
    checked = 0
    for rec in nodes[:200]:
        for c in range(int(rec["nchild"])):
            r = LD.decode_ref(rec["child"][c])
            if r[0] != "leaf":
                continue
            p = pts[r[1]:r[1] + r[2]].reshape(-1, 3)
            lo, hi = p.min(0), p.max(0)
            for a, (nl, nh) in enumerate((("qlo_x", "qhi_x"), ("qlo_y", "qhi_y"), ("qlo_z", "qhi_z"))):
                s, o = rec["scale"][a], rec["origin"][a]
                if s == 0:
                    continue
                ql, qh = int(rec[nl][c]), int(rec[nh][c])
                assert LD.fma32(ql, s, o) <= lo[a] and LD.fma32(qh, s, o) >= hi[a]
                if ql < qmax:
                    assert LD.fma32(ql + 1, s, o) > lo[a]
                if qh > 0:
                    assert LD.fma32(qh - 1, s, o) < hi[a]
                checked += 1
    assert checked > 50


@pytest.mark.parametrize("layout", list(LAYOUTS))
def test_build_is_deterministic(layout):
    from paper_2511_15028_amd import bvh
    v, t = SCENES["spheres"]
    a = _build(v, t, layout).read_buffer(bvh.BUF_NODES)
    b = _build(v, t, layout).read_buffer(bvh.BUF_NODES)
    assert a == b
