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

LAYOUTS = {"aabb2": LD.AABB2, "bvh4": LD.BVH4, "bvh8_q8": LD.BVH8_Q8, "bvh8_q16": LD.BVH8_Q16,
           "pbrt_q16": LD.PBRT_Q16, "sg_eq": LD.SG_EQ, "pbrt_soaos": LD.PBRT_SOAOS,
           "pbrt_q16_soaos": LD.PBRT_Q16_SOAOS, "sg_eq_a16": LD.SG_EQ_A16,
           "shared_slab": LD.SHARED_SLAB}


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
    frame = ((st["scene_lo"], st["scene_hi"]) if lid == LD.SHARED_SLAB else
             (st["frame_origin"], st["frame_scale"], st["frame_top"]))
    nodes, leaves, visited = LD.walk(lid, nodes_bytes, frame)
    assert (visited == 1).all(), "every node reachable exactly once"
    assert len(leaves) == st["n_leaves"]
    leaf_raw = h.read_buffer(bvh.BUF_LEAF)
    if leaf_mode == "compact":
        tri = np.frombuffer(leaf_raw, dtype=LD.TRI_DT)
        order = tri["prim"]
        pts = v[t[order]]
        # p0 is a bit copy; the edges are the f32 differences p1 - p0, p2 - p0
        assert np.array_equal(tri["p0"].view(np.uint32), pts[:, 0].view(np.uint32))
        assert np.array_equal(tri["e1"].view(np.uint32), (pts[:, 1] - pts[:, 0]).view(np.uint32))
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
        if lid in (LD.AABB2, LD.BVH4, LD.PBRT_SOAOS):
            # f32 layouts: the innermost box is exactly the leaf's box
            assert np.array_equal(path[-1][0:3], lo) and np.array_equal(path[-1][3:6], hi)
    assert (covered == 1).all()
    assert st["max_stack"] >= 1 and st["depth"] >= 2
    assert st["nodes_buffer_bytes"] == st["n_nodes"] * {0: 32, 1: 128, 2: 128, 3: 160, 4: 16, 5: 12,
                                                        6: 32, 7: 16, 8: 16, 9: 16}[lid]


@pytest.mark.parametrize("layout", list(LAYOUTS))
def test_quantised_boxes_are_tight(layout):
    """The builder picks the tightest enclosing q: moving any child plane one
    step inward would cut into the child (checked on the decoded nodes)."""
    lid = LAYOUTS[layout]
    if lid not in (LD.BVH8_Q8, LD.BVH8_Q16):
        pytest.skip("f32 layout, or the scene-frame layout (its own test)")
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


@pytest.mark.parametrize("scene", list(SCENES))
def test_pbrt_q16_matches_aabb2(scene):
    """pbrt-q16 is the AABB2 tree re-encoded (App. D.3): node i has the same
    triangle count and offset, its dequantised box encloses the exact AABB2
    box with the tightest q (an interior node's lower x / y plane may sit one
    step lower to carry the split axis), and the axis bits decode to the
    AABB2 split axis wherever that lowering was possible."""
    from paper_2511_15028_amd import bvh
    v, t = SCENES[scene]
    ha = _build(v, t, "aabb2")
    hq = _build(v, t, "pbrt_q16")
    a = np.frombuffer(ha.read_buffer(bvh.BUF_NODES), dtype=LD.AABB2_DT)
    q = np.frombuffer(hq.read_buffer(bvh.BUF_NODES), dtype=LD.PQ16_DT)
    assert len(a) == len(q)
    st = hq.stats()
    o = np.asarray(st["frame_origin"], np.float32)
    s = np.asarray(st["frame_scale"], np.float32)
    assert np.array_equal(o, np.asarray(st["scene_lo"], np.float32))
    # the frame covers the scene: 65535 steps reach the upper corner
    hi_scene = np.asarray(st["scene_hi"], np.float32)
    assert (LD.fma32(65535.0, s, o) >= hi_scene).all()
    cnt_a = a["meta"] & 0xFFFF
    cnt_q = q["meta"] & 0xF
    assert np.array_equal(cnt_a, cnt_q)
    assert np.array_equal(a["offset"], q["meta"] >> 4)
    lo_d = LD.fma32(q["lo"].astype(np.float64), s, o)
    hi_d = LD.fma32(q["hi"].astype(np.float64), s, o)
    assert (lo_d <= a["lo"]).all() and (hi_d >= a["hi"]).all()
    # tightness: one step tighter would cut into the box
    interior = cnt_a == 0
    for ax in range(3):
        if s[ax] == 0:
            continue
        up = LD.fma32(q["lo"][:, ax].astype(np.float64) + 1, s[ax], o[ax])
        slack = (interior & (ax < 2)).astype(np.int64)  # axis-bit lowering
        tight_lo = (up > a["lo"][:, ax]) | (q["lo"][:, ax] == 65535)
        up2 = LD.fma32(q["lo"][:, ax].astype(np.float64) + 2, s[ax], o[ax])
        tight_lo2 = (up2 > a["lo"][:, ax]) | (q["lo"][:, ax] >= 65534)
        assert np.where(slack == 1, tight_lo2, tight_lo).all()
        dn = LD.fma32(q["hi"][:, ax].astype(np.float64) - 1, s[ax], o[ax])
        assert ((dn < a["hi"][:, ax]) | (q["hi"][:, ax] == 0)).all()
    axis_a = (a["meta"] >> 16) & 3
    axis_q = (q["lo"][:, 0] & 1) | ((q["lo"][:, 1] & 1) << 1)
    ok = axis_q == axis_a
    # the bit could not be set only where the lower plane was already at q = 0
    assert (ok | ~interior | (q["lo"][:, 0] == 0) | (q["lo"][:, 1] == 0)).all()
    assert ok[interior].mean() > 0.9


@pytest.mark.parametrize("scene", list(SCENES))
def test_sg_eq_matches_aabb2(scene):
    """sg-eq is the AABB2 tree re-encoded (App. D.1) with 10-bit planes: node
    i has the same triangle count, offset and split axis; lower planes count
    steps up from the frame origin and upper planes steps down from the frame
    top; every dequantised box encloses the exact AABB2 box with the tightest
    q (no directed rounding: the builder checks the traversal's own fmaf)."""
    from paper_2511_15028_amd import bvh
    v, t = SCENES[scene]
    a = np.frombuffer(_build(v, t, "aabb2").read_buffer(bvh.BUF_NODES), dtype=LD.AABB2_DT)
    hq = _build(v, t, "sg_eq")
    q = np.frombuffer(hq.read_buffer(bvh.BUF_NODES), dtype=LD.SGEQ_DT)
    assert len(a) == len(q)
    st = hq.stats()
    o = np.asarray(st["frame_origin"], np.float32)
    s = np.asarray(st["frame_scale"], np.float32)
    top = np.asarray(st["frame_top"], np.float32)
    assert np.array_equal(o, np.asarray(st["scene_lo"], np.float32))
    assert np.array_equal(top, np.asarray(st["scene_hi"], np.float32))
    assert (LD.fma32(1023.0, s, o) >= top).all() and (LD.fma32(-1023.0, s, top) <= o).all()
    qlo, qhi, nprim, off, axis = LD.sg_eq_fields(q)
    cnt_a = (a["meta"] & 0xFFFF).astype(np.uint64)
    assert np.array_equal(nprim, cnt_a)
    assert np.array_equal(off, a["offset"].astype(np.uint64))
    interior = cnt_a == 0
    assert np.array_equal(axis[interior], ((a["meta"] >> 16) & 3)[interior].astype(np.uint64))
    for ax in range(3):
        if s[ax] == 0:
            continue
        lo_d = LD.fma32(qlo[:, ax].astype(np.float64), s[ax], o[ax])
        hi_d = LD.fma32(-qhi[:, ax].astype(np.float64), s[ax], top[ax])
        assert (lo_d <= a["lo"][:, ax]).all() and (hi_d >= a["hi"][:, ax]).all()
        up = LD.fma32(qlo[:, ax].astype(np.float64) + 1, s[ax], o[ax])
        assert ((up > a["lo"][:, ax]) | (qlo[:, ax] == 1023)).all()
        dn = LD.fma32(-(qhi[:, ax].astype(np.float64) + 1), s[ax], top[ax])
        assert ((dn < a["hi"][:, ax]) | (qhi[:, ax] == 1023)).all()


VARIANTS = [("pbrt_soaos", "aabb2"), ("pbrt_q16_soaos", "pbrt_q16"), ("sg_eq_a16", "sg_eq")]


@pytest.mark.parametrize("scene", list(SCENES))
@pytest.mark.parametrize("variant, base", VARIANTS)
def test_soaos_and_align16_hold_the_base_records(variant, base, scene):
    """The SoAoS variants hold exactly the base layout's records, split into a
    box array followed by a topology array; sg-eq-align16 holds the sg-eq
    records each followed by a zero word; the scene frame is the base's."""
    from paper_2511_15028_amd import bvh
    v, t = SCENES[scene]
    hv, hb = _build(v, t, variant), _build(v, t, base)
    sv, sb = hv.stats(), hb.stats()
    assert sv["n_nodes"] == sb["n_nodes"] and sv["n_leaves"] == sb["n_leaves"]
    for k in ("frame_origin", "frame_scale", "frame_top"):
        assert list(sv[k]) == list(sb[k])
    base_id, rec = LD.as_base(LAYOUTS[variant], hv.read_buffer(bvh.BUF_NODES))
    assert base_id == LAYOUTS[base]
    want = np.frombuffer(hb.read_buffer(bvh.BUF_NODES), LD.DTYPES[base_id])
    assert rec.tobytes() == want.tobytes()
    assert hv.read_buffer(bvh.BUF_LEAF) == hb.read_buffer(bvh.BUF_LEAF)


@pytest.mark.parametrize("scene", list(SCENES))
def test_shared_slab_matches_aabb2(scene):
    """The shared-slab tree is the AABB2 tree: node i has AABB2 node i's count,
    offset and split axis, and its slab is AABB2 node i's exact extent along
    the axis where that box is narrowest relative to its parent's box (the
    scene box for the root; lowest axis on ties)."""
    from paper_2511_15028_amd import bvh
    v, t = SCENES[scene]
    hs, ha = _build(v, t, "shared_slab"), _build(v, t, "aabb2")
    sl = np.frombuffer(hs.read_buffer(bvh.BUF_NODES), LD.SLAB_DT)
    ab = np.frombuffer(ha.read_buffer(bvh.BUF_NODES), LD.AABB2_DT)
    assert len(sl) == len(ab)
    st = hs.stats()
    parent_lo = np.empty((len(ab), 3), np.float32)
    parent_hi = np.empty((len(ab), 3), np.float32)
    parent_lo[0], parent_hi[0] = st["scene_lo"], st["scene_hi"]
    for i in range(len(ab)):
        if ab["meta"][i] & 0xFFFF == 0:
            for c in (i + 1, i + int(ab["offset"][i])):
                parent_lo[c], parent_hi[c] = ab["lo"][i], ab["hi"][i]
    np.testing.assert_array_equal(sl["offset"], ab["offset"])
    np.testing.assert_array_equal(sl["meta"] & 0xFFFF, ab["meta"] & 0xFFFF)
    np.testing.assert_array_equal((sl["meta"] >> 18) & 3, (ab["meta"] >> 16) & 3)
    pe = (parent_hi - parent_lo).astype(np.float32)
    ce = (ab["hi"] - ab["lo"]).astype(np.float32)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(pe > 0, (ce / np.where(pe > 0, pe, 1)).astype(np.float32), np.float32(1.0))
    axis = np.argmin(ratio, axis=1)
    np.testing.assert_array_equal((sl["meta"] >> 16) & 3, axis)
    rows = np.arange(len(ab))
    np.testing.assert_array_equal(sl["slo"], ab["lo"][rows, axis])
    np.testing.assert_array_equal(sl["shi"], ab["hi"][rows, axis])


def _offset_scene(offs):
    small = np.array([[0, 0, 0], [0.01, 0, 0], [0, 0.01, 0.005]], np.float32)
    offs = np.asarray(offs, np.float32)
    v = (small[None] + offs[:, None]).reshape(-1, 3).astype(np.float32)
    return v, np.arange(len(v), dtype=np.int32).reshape(-1, 3)


@pytest.mark.parametrize("layout", ["bvh4", "bvh8_q8", "bvh8_q16"])
def test_node_block_hint_paths(layout):
    """The wide packers reuse the node count of an earlier build with the same
    (layout, leaf size, triangle count) to allocate the node block ahead.
    Two 4,096-triangle meshes: coincident triangles (a balanced tree, full
    leaves) and 512 groups of 8 where each group peels off one triangle per
    level (many small leaves, far more wide nodes).  The second mesh built
    right after the first overflows the block sized from the first one's
    count and takes the spill-and-copy path; built again it fits.  Both
    results must be byte-identical, and the first mesh rebuilt after the
    second (a larger hint) must match its first build."""
    from paper_2511_15028_amd import bvh
    a_v, a_t = _offset_scene(np.zeros((4096, 3)))
    g = np.stack(np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij"), -1)
    inner = np.array([[0, 0, 0]] * 4 + [[1, 0, 0], [2, 0, 0], [4, 0, 0], [8, 0, 0]], np.float32)
    b_v, b_t = _offset_scene((g.reshape(-1, 3)[:, None, :] * 16.0 + inner[None]).reshape(-1, 3))
    ha = _build(a_v, a_t, layout)
    na = ha.stats()["n_nodes"]
    hb1 = _build(b_v, b_t, layout)
    nb = hb1.stats()["n_nodes"]
    assert nb > na + na // 64 + 64, (na, nb)   # the first mesh's hint is too small
    hb2 = _build(b_v, b_t, layout)
    assert hb2.stats()["n_nodes"] == nb
    assert hb1.read_buffer(bvh.BUF_NODES) == hb2.read_buffer(bvh.BUF_NODES)
    ha2 = _build(a_v, a_t, layout)
    assert ha2.read_buffer(bvh.BUF_NODES) == ha.read_buffer(bvh.BUF_NODES)
    # the spilled build is a tree covering every triangle once
    st = hb1.stats()
    raw = hb1.read_buffer(bvh.BUF_NODES)
    assert len(raw) == nb * st["node_bytes"]
    frame = (st["frame_origin"], st["frame_scale"], st["frame_top"])
    _, leaves, visited = LD.walk(LAYOUTS[layout], raw, frame)
    assert (visited == 1).all() and len(leaves) == st["n_leaves"]
    tri = np.frombuffer(hb1.read_buffer(bvh.BUF_LEAF), dtype=LD.TRI_DT)
    covered = np.zeros(len(b_t), np.int64)
    for first, n, _ in leaves:
        covered[tri["prim"][first:first + n]] += 1
    assert (covered == 1).all()
