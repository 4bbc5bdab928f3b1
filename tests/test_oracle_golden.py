"""The stored golden fixture (tests/golden/soup_closest_hits.txt, written by
tests/golden/make_golden.py from the oracle's exhaustive search) still
matches the oracle bit for bit, and its hits are genuine: each recorded hit
is accepted by the FP32 test of that ray against that triangle, and an FP64
solve of the hit equation agrees to within the FP32 error bound."""
import os

import numpy as np

from paper_2511_15028_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "soup_closest_hits.txt")


def load_golden():
    rows = [l.split() for l in open(GOLDEN) if not l.startswith("#")]
    idx = np.array([int(r[0]) for r in rows])
    prim = np.array([int(r[1]) for r in rows], np.int32)
    tuv = np.array([[int(x, 16) for x in r[2:5]] for r in rows], np.uint32).view(np.float32)
    return idx, prim, tuv


def test_golden_matches_the_oracle(orc):
    idx, prim, tuv = load_golden()
    w = W.soup_workload()
    p, t = orc.brute_closest(w["verts"], w["tris"], w["rays"][idx])
    assert np.array_equal(p, prim)
    assert np.array_equal(t.view(np.uint32), tuv.view(np.uint32))
    assert 40 <= (prim >= 0).sum() <= 200


def test_golden_hits_are_genuine(orc):
    idx, prim, tuv = load_golden()
    w = W.soup_workload()
    v, tr, rays = w["verts"], w["tris"], w["rays"][idx]
    hit = prim >= 0
    ok, t2 = orc.mt_fixed(v, tr, rays[hit], prim[hit])
    assert ok.all() and np.array_equal(t2, tuv[hit])
    # FP64 solve of o + t d = (1-u-v) p0 + u p1 + v p2
    p = v[tr[prim[hit]]].astype(np.float64)
    o, d = rays[hit, 0:3].astype(np.float64), rays[hit, 4:7].astype(np.float64)
    A = np.stack([d, p[:, 0] - p[:, 1], p[:, 0] - p[:, 2]], axis=2)
    x = np.linalg.solve(A, (p[:, 0] - o)[:, :, None])[:, :, 0]
    assert np.allclose(x, tuv[hit], rtol=0, atol=1e-5)
