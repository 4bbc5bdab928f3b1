"""Batched tracing (bvh_batch_*): per-scene tuning, one graph launch.

* the batched hits equal bvh_trace of each scene's own (tuned) handle, bit
  for bit, and match the oracle on every scene;
* the graph is replayed several times with eager work in between, and every
  replay is checked;
* new ray offsets rebuild the graph; fixed layout / stack choices are kept.
"""
import numpy as np
import pytest

from paper_2511_15028_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _small_batch():
    w = W.batch_workload(seed=77, n_scenes=14, tri_range=(1, 6e3), ray_range=(1, 3e3))
    scenes = list(w["scenes"])
    rays = [w["rays"][w["offsets"][i]:w["offsets"][i + 1]] for i in range(14)]
    # an empty mesh, and a scene with no rays
    v0, t0 = W.soup_scene(3, seed=1)
    scenes.append((v0, t0[:0]))
    rays.append(W.uniform_rays(300, 5))
    scenes.append(W.soup_scene(50, seed=2))
    rays.append(W.uniform_rays(0, 6))
    off = np.zeros(len(scenes) + 1, np.int64)
    off[1:] = np.cumsum([len(r) for r in rays])
    return scenes, np.concatenate(rays), off


def _oracle_check(orc, scenes, rays, off, prim, tuv):
    from test_gpu_parity import check_closest
    for i, (v, t) in enumerate(scenes):
        a, b = off[i], off[i + 1]
        if b == a:
            continue
        if len(t) == 0:
            assert (prim[a:b] == -1).all()
            continue
        ref = orc.OracleBVH(v, t).trace(rays[a:b], orc.TOP2)
        check_closest(orc, v, t, rays[a:b], prim[a:b], tuv[a:b], ref)


def test_batch_matches_per_scene_and_oracle(orc):
    from paper_2511_15028_amd import bvh
    scenes, rays, off = _small_batch()
    ds = [(dev(v), dev(t)) for v, t in scenes]
    b = bvh.Batch(ds, probe_rays=2048)
    infos = [b.info(i) for i in range(len(scenes))]
    assert {i["layout"] for i in infos} <= {0, 1, 2, 3, 4, 5}
    assert all(i["stack_lds"] in (8, 16, 32) for i in infos)
    assert max(i["candidates"] for i in infos) == 8  # 6 layouts, then 2 more stack depths
    dr = dev(rays)
    hits = b.trace(dr, off)
    torch.cuda.synchronize()
    hb = hits.cpu().numpy()
    # per-scene bvh_trace with the same handles
    for i in range(len(scenes)):
        a, c = off[i], off[i + 1]
        if c == a:
            continue
        hp = b.handle(i).trace(dr[a:c]).cpu().numpy()
        assert np.array_equal(hp.view(np.uint32), hb[a:c].view(np.uint32)), i
    prim = hb[:, 0].view(np.int32)
    _oracle_check(orc, scenes, rays, off, prim, hb[:, 1:4])


def test_graph_replays_and_rebuilds(orc):
    from paper_2511_15028_amd import bvh
    scenes, rays, off = _small_batch()
    ds = [(dev(v), dev(t)) for v, t in scenes]
    b = bvh.Batch(ds, layout="bvh8_q8", stack_lds=16)
    assert all(b.info(i)["layout"] == 2 and b.info(i)["stack_lds"] == 16 for i in range(len(scenes)))
    dr = dev(rays)
    hits = torch.empty((len(rays), 4), dtype=torch.float32, device="cuda")
    first = None
    for k in range(4):
        hits.fill_(float(k + 7))          # eager work between replays
        torch.cuda.synchronize()
        b.trace(dr, off, hits=hits)
        torch.cuda.synchronize()
        cur = hits.cpu().numpy().copy()
        if first is None:
            first = cur
        assert np.array_equal(cur.view(np.uint32), first.view(np.uint32)), k
    # other offsets: the first scene loses half of its rays to the second
    off2 = off.copy()
    off2[1] = off[0] + (off[1] - off[0]) // 2
    h2 = b.trace(dr, off2)
    torch.cuda.synchronize()
    h2 = h2.cpu().numpy()
    a, c = off2[1], off2[2]
    hp = b.handle(1).trace(dr[a:c]).cpu().numpy()
    assert np.array_equal(hp.view(np.uint32), h2[a:c].view(np.uint32))
    _oracle_check(orc, scenes, rays, off2, h2[:, 0].view(np.int32), h2[:, 1:4])


def test_batch_with_user_probe_rays(orc):
    from paper_2511_15028_amd import bvh
    scenes, rays, off = _small_batch()
    ds = [(dev(v), dev(t)) for v, t in scenes]
    b = bvh.Batch(ds, layout=[None] * 8 + ["aabb2"] * (len(scenes) - 8), probe=dev(rays),
                  probe_offsets=off)
    for i in range(8, len(scenes)):
        assert b.info(i)["layout"] == 0
    hits = b.trace(dev(rays), off)
    torch.cuda.synchronize()
    hb = hits.cpu().numpy()
    _oracle_check(orc, scenes, rays, off, hb[:, 0].view(np.int32), hb[:, 1:4])


def test_batch_full_size_sampled_against_oracle(orc):
    """The benchmark's batch at full size (256 scenes, log-uniform 1 K-500 K
    triangles and 1 K-1 M incoherent rays each, tuned on device-generated
    probe rays): on every scene, 128 rays spread over its range are checked
    against the oracle's median-split BVH, and the whole batch bit for bit
    against plain per-scene traces of the same handles."""
    from paper_2511_15028_amd import bvh
    w = W.batch_workload()
    scenes, rays, off = w["scenes"], w["rays"], w["offsets"]
    ds = [(dev(v), dev(t)) for v, t in scenes]
    b = bvh.Batch(ds)
    dr = dev(rays)
    hits = b.trace(dr, off)
    plain = torch.empty_like(hits)
    for i in range(len(scenes)):
        if off[i + 1] > off[i]:
            b.handle(i).trace(dr[off[i]:off[i + 1]], hits=plain[off[i]:off[i + 1]])
    torch.cuda.synchronize()
    assert torch.equal(hits.view(torch.int32), plain.view(torch.int32))
    hb = hits.cpu().numpy()
    del dr, plain, hits
    rng = np.random.default_rng(5)
    for i, (v, t) in enumerate(scenes):
        a, c = int(off[i]), int(off[i + 1])
        k = min(128, c - a)
        idx = np.sort(rng.choice(c - a, size=k, replace=False)) + a
        ref = orc.OracleBVH(v, t).trace(rays[idx], orc.TOP2)
        from test_gpu_parity import check_closest
        check_closest(orc, v, t, rays[idx], hb[idx, 0].view(np.int32), hb[idx, 1:4], ref)
    b.close()
