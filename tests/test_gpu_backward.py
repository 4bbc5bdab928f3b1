"""Backward kernel against the FP64 oracle gradient (itself pinned by FP64
finite differences in test_oracle_grad.py).

Tolerances (no published bound): per-ray dL/do, dL/dd within 1e-4 of the
ray's FP64 gradient norm on well-conditioned hits (min barycentric > 1e-4,
|cos(d, n)| > 1e-2); grad_verts within 1e-5 relative L2 overall and, per
element, 1e-5 of the summed contribution magnitudes plus 1e-7, which allows
for FP32 atomic accumulation in any order.
"""
import numpy as np
import pytest

from paper_2511_15028_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _run(w, layout="bvh8_q8"):
    from paper_2511_15028_amd import bvh
    v, t, rays, wts = w["verts"], w["tris"], w["rays"], w["weights"]
    dv, dt, dr = dev(v), dev(t), dev(rays)
    h = bvh.build(dv, dt, layout)
    hits = h.trace(dr)
    gv, gr = bvh.trace_backward(dv, dt, dr, hits, dev(wts))
    torch.cuda.synchronize()
    hh = hits.cpu().numpy()
    return hh[:, 0].view(np.int32).copy(), hh[:, 1:4].copy(), gv.cpu().numpy(), gr.cpu().numpy()


def _compare(orc, w, prim, tuv, gv, gr):
    v, t, rays, wts = w["verts"], w["tris"], w["rays"], w["weights"]
    gv64, gr64, tuv64 = orc.grad_f64(v, t, rays, prim, wts)
    p = v[t[np.maximum(prim, 0)]].astype(np.float64)
    ng = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    d = rays[:, 4:7].astype(np.float64)
    cos = np.abs(np.sum(ng * d, 1)) / (np.linalg.norm(ng, axis=1) * np.linalg.norm(d, axis=1) + 1e-300)
    bmin = np.minimum(np.minimum(tuv[:, 1], tuv[:, 2]), 1 - tuv[:, 1] - tuv[:, 2])
    good = (prim >= 0) & (bmin > 1e-4) & (cos > 1e-2)
    assert good.mean() > 0.9
    norm = np.linalg.norm(gr64[good], axis=1)
    err = np.linalg.norm(gr[good] - gr64[good], axis=1)
    assert (err <= 1e-4 * norm).all(), err.max()
    assert (gr[prim < 0] == 0).all()
    # vertex gradients over all rays
    rel = np.linalg.norm(gv - gv64) / np.linalg.norm(gv64)
    assert rel <= 1e-5, rel
    # per element bound from the summed magnitude of the contributions
    mag = np.zeros_like(gv64)
    lam = -gr64[:, 0:3]
    wgt = np.stack([1 - tuv64[:, 1] - tuv64[:, 2], tuv64[:, 1], tuv64[:, 2]], 1)
    hit = prim >= 0
    for k in range(3):
        np.add.at(mag, t[prim[hit], k], np.abs(wgt[hit, k:k + 1] * lam[hit]))
    assert (np.abs(gv - gv64) <= 1e-5 * mag + 1e-7).all()


def test_backward_small(orc):
    w = W.diff_workload(level=4, n_cams=8, res=32)
    prim, tuv, gv, gr = _run(w)
    p1, tuv1 = orc.brute_closest(w["verts"], w["tris"], w["rays"])
    assert np.array_equal(prim, p1)
    _compare(orc, w, prim, tuv, gv, gr)


def test_backward_full_size(orc):
    """The full differentiable workload: 327,680 triangles, 1,048,576 rays."""
    w = W.diff_workload()
    prim, tuv, gv, gr = _run(w)
    assert (prim >= 0).all()
    _compare(orc, w, prim, tuv, gv, gr)


def test_backward_skips_invalid_prims(orc):
    from paper_2511_15028_amd import bvh
    w = W.diff_workload(level=2, n_cams=2, res=8)
    v, t, rays = w["verts"], w["tris"], w["rays"]
    hits = np.zeros((len(rays), 4), np.float32)
    hits[:, 0] = np.array([-1, len(t), 10 ** 6, 0] * (len(rays) // 4), np.int32).view(np.float32)
    hits[:, 1:] = [1.0, 0.2, 0.3]
    gv, gr = bvh.trace_backward(dev(v), dev(t), dev(rays), dev(hits), dev(w["weights"]))
    torch.cuda.synchronize()
    gr = gr.cpu().numpy()
    assert (gr[0::4] == 0).all() and (gr[1::4] == 0).all() and (gr[2::4] == 0).all()
    assert (np.abs(gr[3::4]).sum(1) > 0).all()


def test_autograd_function(orc):
    from paper_2511_15028_amd import bvh
    w = W.diff_workload(level=3, n_cams=4, res=16)
    v = dev(w["verts"]).requires_grad_(True)
    t = dev(w["tris"])
    o = dev(w["rays"][:, 0:3]).requires_grad_(True)
    d = dev(w["rays"][:, 4:7]).requires_grad_(True)
    h = bvh.build(v.detach(), t, "bvh4")
    prim, tuv = bvh.BVHTrace.apply(v, t, o, d, h)
    loss = (tuv * dev(w["weights"])).sum()
    loss.backward()
    gv64, gr64, _ = orc.grad_f64(w["verts"], w["tris"], w["rays"], prim.cpu().numpy(), w["weights"])
    np.testing.assert_allclose(o.grad.cpu().numpy(), gr64[:, 0:3], rtol=1e-3, atol=1e-4)
    np.testing.assert_allclose(d.grad.cpu().numpy(), gr64[:, 3:6], rtol=1e-3, atol=1e-4)
    np.testing.assert_allclose(v.grad.cpu().numpy(), gv64, rtol=1e-3, atol=1e-4)
