"""Backward kernel against the FP64 oracle gradient (itself pinned by FP64
finite differences in test_oracle_grad.py).

The kernel is given the oracle's own FP32 forward hits and compared with the
FP64 gradient evaluated at those same hit parameters (the gradient is defined
at the forward result).  Tolerances (no published bound): per-ray dL/do,
dL/dd within 1e-4 of the ray's FP64 gradient norm on well-conditioned hits
(min barycentric > 1e-4, |cos(d, n)| > 1e-2); grad_verts within 1e-5
relative L2 and, per element, the propagated per-ray FP32 error in lam plus
1e-5 of the summed contribution magnitudes plus 1e-7, which allows for FP32
atomic accumulation in any order.  Against the fully FP64 gradient (hit
parameters re-solved in FP64) the gap may add the FP32 forward's own
rounding of (t, u, v), measured on the oracle side.
"""
import numpy as np
import pytest

from paper_2511_15028_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _run(w, hits_np):
    """Backward kernel on the given (oracle) hits."""
    from paper_2511_15028_amd import bvh
    v, t, rays, wts = w["verts"], w["tris"], w["rays"], w["weights"]
    gv, gr = bvh.trace_backward(dev(v), dev(t), dev(rays), dev(hits_np), dev(wts))
    torch.cuda.synchronize()
    return gv.cpu().numpy(), gr.cpu().numpy()


def _hits_array(prim, tuv):
    h = np.zeros((len(prim), 4), np.float32)
    h[:, 0] = prim.astype(np.int32).view(np.float32)
    h[:, 1:4] = tuv
    return h


def _compare(orc, w, prim, tuv, gv, gr):
    """prim/tuv: the oracle's FP32 forward hits, which the kernel was given."""
    v, t, rays, wts = w["verts"], w["tris"], w["rays"], w["weights"]
    # the FP64 gradient evaluated at the same FP32 forward result
    gv64, gr64, _ = orc.grad_f64(v, t, rays, prim, wts, tuv_at=tuv)
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
    rel = np.linalg.norm(gv - gv64) / np.linalg.norm(gv64)
    assert rel <= 1e-5, rel
    # per element: ray i adds w_k * lam_i to a vertex; the FP32 solve for lam
    # is off by |dlam| (large only for grazing hits, where J is
    # ill-conditioned) and the float atomics add rounding, covered by 1e-5 of
    # the summed contribution magnitudes, plus 1e-7
    mag = np.zeros_like(gv64)
    prop = np.zeros_like(gv64)
    lam = -gr64[:, 0:3]
    dlam = np.abs(gr[:, 0:3] - gr64[:, 0:3])
    wgt = np.stack([1 - tuv[:, 1] - tuv[:, 2], tuv[:, 1], tuv[:, 2]], 1).astype(np.float64)
    hit = prim >= 0
    for k in range(3):
        np.add.at(mag, t[prim[hit], k], np.abs(wgt[hit, k:k + 1] * lam[hit]))
        np.add.at(prop, t[prim[hit], k], np.abs(wgt[hit, k:k + 1]) * dlam[hit])
    assert (np.abs(gv - gv64) <= prop + 1e-5 * mag + 1e-7).all()
    # against the fully FP64 gradient (hit parameters re-solved in FP64): the
    # gap is the FP32 forward's own rounding of (t, u, v), measured on the
    # oracle side alone
    gvx, grx, _ = orc.grad_f64(v, t, rays, prim, wts)
    fwd = np.linalg.norm(gv64 - gvx) / np.linalg.norm(gvx)
    assert np.linalg.norm(gv - gvx) / np.linalg.norm(gvx) <= fwd + 1e-5
    return rel, fwd


def test_backward_small(orc):
    w = W.diff_workload(level=4, n_cams=8, res=32)
    p1, tuv1 = orc.brute_closest(w["verts"], w["tris"], w["rays"])
    gv, gr = _run(w, _hits_array(p1, tuv1))
    _compare(orc, w, p1, tuv1, gv, gr)
    # the GPU forward gives the same hits, so its own hits give the same gradient
    from paper_2511_15028_amd import bvh
    h = bvh.build(dev(w["verts"]), dev(w["tris"]), "bvh8_q8")
    hits = h.trace(dev(w["rays"])).cpu().numpy()
    assert np.array_equal(hits[:, 0].view(np.int32), p1)
    assert np.array_equal(hits[:, 1:4], tuv1)


def test_backward_full_size(orc):
    """The full differentiable workload: 327,680 triangles, 1,048,576 rays."""
    w = W.diff_workload()
    p1, tuv1 = orc.OracleBVH(w["verts"], w["tris"]).trace(w["rays"])
    assert (p1 >= 0).all()
    gv, gr = _run(w, _hits_array(p1, tuv1))
    _compare(orc, w, p1, tuv1, gv, gr)


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
