"""Pins for the oracle's FP64 gradient of L = sum(w_t t + w_u u + w_v v).

Pinned by central finite differences (step 1e-6, FP64) of (t, u, v) obtained
from numpy.linalg.solve, which shares nothing with the oracle's closed form,
and by exact identities of the hit-point relation o + t d = (1-u-v) p0 +
u p1 + v p2: translation invariance, the scaling law of the direction, and
zero contribution from misses.
"""
import numpy as np
import pytest

from paper_2511_15028_amd import workloads as W

H = 1e-6


def _tuv_solve(verts64, tris, rays64, prims):
    out = np.empty((len(prims), 3))
    for i, p in enumerate(prims):
        q = verts64[tris[p]]
        A = np.stack([rays64[i, 4:7], q[0] - q[1], q[0] - q[2]], axis=1)
        out[i] = np.linalg.solve(A, q[0] - rays64[i, 0:3])
    return out


def _loss(verts64, tris, rays64, prims, w):
    return float(np.sum(_tuv_solve(verts64, tris, rays64, prims) * w))


@pytest.fixture(scope="module")
def hits(orc):
    w = W.diff_workload(level=3, n_cams=4, res=8)
    verts, tris, rays = w["verts"], w["tris"], w["rays"]
    prim, tuv = orc.brute_closest(verts, tris, rays)
    assert (prim >= 0).all()          # every camera ray meets the sphere
    return verts, tris, rays, prim, tuv, w["weights"]


def _well_conditioned(verts, tris, rays, prim, tuv):
    p = verts[tris[prim]].astype(np.float64)
    ng = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    d = rays[:, 4:7].astype(np.float64)
    cos = np.abs(np.sum(ng * d, 1)) / (np.linalg.norm(ng, axis=1) * np.linalg.norm(d, axis=1))
    u, v = tuv[:, 1], tuv[:, 2]
    return (np.minimum(np.minimum(u, v), 1 - u - v) > 1e-4) & (cos > 1e-2)


def test_gradient_matches_finite_differences(orc, hits):
    verts, tris, rays, prim, tuv, wts = hits
    keep = _well_conditioned(verts, tris, rays, prim, tuv)
    sel = np.nonzero(keep)[0][:64]
    rays, prim, wts = rays[sel], prim[sel], wts[sel]
    gv, gr, tuv64 = orc.grad_f64(verts, tris, rays, prim, wts)
    v64 = verts.astype(np.float64)
    r64 = rays.astype(np.float64)
    rng = np.random.default_rng(11)
    # ray components
    for i in rng.choice(len(sel), 24, replace=False):
        for k, col in enumerate([0, 1, 2, 4, 5, 6]):
            rp, rm = r64[i:i + 1].copy(), r64[i:i + 1].copy()
            rp[0, col] += H
            rm[0, col] -= H
            fd = (_loss(v64, tris, rp, prim[i:i + 1], wts[i:i + 1])
                  - _loss(v64, tris, rm, prim[i:i + 1], wts[i:i + 1])) / (2 * H)
            a = gr[i, k]
            assert abs(a - fd) <= 1e-6 * (abs(a) + abs(fd)) + 1e-9, (i, k, a, fd)
    # vertex coordinates touched by the selected hits
    touched = np.unique(tris[prim].reshape(-1))
    for vi in rng.choice(touched, 24, replace=False):
        for c in range(3):
            vp, vm = v64.copy(), v64.copy()
            vp[vi, c] += H
            vm[vi, c] -= H
            fd = (_loss(vp, tris, r64, prim, wts) - _loss(vm, tris, r64, prim, wts)) / (2 * H)
            a = gv[vi, c]
            assert abs(a - fd) <= 1e-6 * (abs(a) + abs(fd)) + 1e-9, (vi, c, a, fd)


def test_tuv_matches_fp32_hits(orc, hits):
    verts, tris, rays, prim, tuv, wts = hits
    _, _, tuv64 = orc.grad_f64(verts, tris, rays, prim, wts)
    np.testing.assert_allclose(tuv64, tuv, rtol=1e-4, atol=1e-5)


def test_translation_and_scaling_identities(orc, hits):
    verts, tris, rays, prim, tuv, wts = hits
    n = len(prim)
    gv, gr, tuv64 = orc.grad_f64(verts, tris, rays, prim, wts)
    # per ray: moving o and the three vertices together leaves (t,u,v) fixed
    for i in range(0, n, 7):
        one = slice(i, i + 1)
        gvi, gri, _ = orc.grad_f64(verts, tris, rays[one], prim[one], wts[one])
        total = gri[0, 0:3] + gvi.sum(0)
        scale = np.abs(gri[0, 0:3]).sum() + np.abs(gvi).sum()
        assert np.all(np.abs(total) <= 1e-12 * scale + 1e-300)
    # scaling d by a leaves u, v and divides t by a: d . dL/dd = -t dL/dt
    d = rays[:, 4:7].astype(np.float64)
    lhs = np.sum(d * gr[:, 3:6], 1)
    rhs = -tuv64[:, 0] * wts[:, 0]
    np.testing.assert_allclose(lhs, rhs, rtol=1e-10, atol=1e-12)


def test_misses_contribute_nothing(orc, hits):
    verts, tris, rays, prim, tuv, wts = hits
    miss = prim.copy()
    miss[::2] = -1
    gv, gr, tuv64 = orc.grad_f64(verts, tris, rays, miss, wts)
    assert (gr[::2] == 0).all()
    assert np.isnan(tuv64[::2]).all()
    gv_odd, _, _ = orc.grad_f64(verts, tris, rays[1::2], prim[1::2], wts[1::2])
    np.testing.assert_allclose(gv, gv_odd, rtol=1e-12, atol=1e-15)


def test_gradient_at_given_hit_parameters(orc, hits):
    verts, tris, rays, prim, tuv, wts = hits
    gv, gr, tuv64 = orc.grad_f64(verts, tris, rays, prim, wts)
    # evaluated at the FP64 parameters rounded to FP32: lam is unchanged, the
    # weights and -t lam move by at most the rounding of (t, u, v)
    gv2, gr2, tuv2 = orc.grad_f64(verts, tris, rays, prim, wts, tuv_at=tuv64.astype(np.float32))
    np.testing.assert_array_equal(tuv2, tuv64.astype(np.float32).astype(np.float64))
    np.testing.assert_array_equal(gr2[:, 0:3], gr[:, 0:3])
    np.testing.assert_allclose(gr2[:, 3:6], gr[:, 3:6], rtol=1e-6)
    # weights move by float32 rounding (< 2^-23 absolute); sums may cancel
    np.testing.assert_allclose(gv2, gv, rtol=0, atol=1e-6 * np.abs(gv).max())
    # and at the FP32 forward's own hit: the same lam, weights from that hit
    gv3, gr3, tuv3 = orc.grad_f64(verts, tris, rays, prim, wts, tuv_at=tuv)
    np.testing.assert_array_equal(tuv3, tuv.astype(np.float64))
    np.testing.assert_array_equal(gr3[:, 0:3], gr[:, 0:3])
    # dL/dd = -t lam with lam = -dL/do
    np.testing.assert_allclose(gr3[:, 3:6], tuv[:, 0:1].astype(np.float64) * gr[:, 0:3], rtol=1e-12)
