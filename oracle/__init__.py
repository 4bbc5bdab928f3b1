"""CPU oracle for closest-hit BVH traversal (test infrastructure only).

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
import this package.  The GPU product path never does: it must fail loudly
when its HIP library is missing rather than fall back here.

The arithmetic lives in ``oracle.c`` (plain C11 + OpenMP, built with
``-ffp-contract=off``); this module only marshals numpy arrays through ctypes.
Each entry point cites the paper passage it follows in ``oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

# Portable ISA level so the library also runs on a host CPU other than the
# one it was built on; no FMA contraction anywhere.
CFLAGS = ["-O3", "-std=c11", "-march=x86-64-v2", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(out: str = LIB_PATH) -> str:
    """Compiles oracle.c into a shared library with gcc."""
    cmd = ["gcc", *CFLAGS, SRC_PATH, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = ctypes.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32


def _declare(L):
    L.orc_mt_f32.argtypes = [_P, _P, ctypes.c_float, _P, _P, _P, _P]
    L.orc_mt_f32.restype = ctypes.c_int
    L.orc_mt_fixed.argtypes = [_P, _P, _I64, _P, _I64, _P, _P, _P]
    L.orc_mt_fixed.restype = None
    L.orc_brute_closest.argtypes = [_P, _P, _I64, _P, _I64, _P, _P, ctypes.c_int]
    L.orc_brute_closest.restype = None
    L.orc_brute_top2.argtypes = [_P, _P, _I64, _P, _I64, _P, _P, ctypes.c_int]
    L.orc_brute_top2.restype = None
    L.orc_bvh_build.argtypes = [_P, _P, _I64]
    L.orc_bvh_build.restype = _P
    L.orc_bvh_free.argtypes = [_P]
    L.orc_bvh_free.restype = None
    L.orc_bvh_depth.argtypes = [_P]
    L.orc_bvh_depth.restype = _I32
    L.orc_bvh_nnodes.argtypes = [_P]
    L.orc_bvh_nnodes.restype = _I32
    L.orc_bvh_export.argtypes = [_P, _P, _P, _P]
    L.orc_bvh_export.restype = None
    L.orc_bvh_trace.argtypes = [_P, _P, _I64, ctypes.c_int, _P, _P, _P, _P, ctypes.c_int]
    L.orc_bvh_trace.restype = None
    L.orc_max_threads.argtypes = []
    L.orc_max_threads.restype = ctypes.c_int
    L.orc_tuv_f64.argtypes = [_P, _P, _P, _P, _I64, _P]
    L.orc_tuv_f64.restype = None
    L.orc_grad_f64.argtypes = [_P, _P, _P, _P, _P, _I64, _P, _P, _P, _P]
    L.orc_grad_f64.restype = None
    L.orc_point_tri_f64.argtypes = [_P, _P, _P, _P, _I64, _P]
    L.orc_point_tri_f64.restype = None
    L.orc_brute_closest_point.argtypes = [_P, _P, _I64, _P, _I64, _P, _P, _P, _P, ctypes.c_int]
    L.orc_brute_closest_point.restype = None
    L.orc_bvh_closest_point.argtypes = [_P, _P, _I64, _P, _P, _P, _P, ctypes.c_int]
    L.orc_bvh_closest_point.restype = None
    L.orc_sah_build.argtypes = [_P, _P, _I64, _P, _P, _P]
    L.orc_sah_build.restype = _I64


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


MISS = -1


def mt_f32(o, d, tmax, p0, p1, p2):
    """FP32 Moller-Trumbore (App. G).  Returns (t, u, v) or None on a miss."""
    o, d, p0, p1, p2 = (_c(x, np.float32) for x in (o, d, p0, p1, p2))
    out = np.zeros(3, np.float32)
    hit = lib().orc_mt_f32(_ptr(o), _ptr(d), ctypes.c_float(tmax), _ptr(p0), _ptr(p1),
                           _ptr(p2), _ptr(out))
    return (float(out[0]), float(out[1]), float(out[2])) if hit else None


def mt_fixed(verts, tris, rays, prims):
    """FP32 Moller-Trumbore of each ray against its given triangle prims[i]
    (negative: none).  Returns (hit[n] bool, tuv[n,3] float32; (inf,0,0) on
    a miss)."""
    verts, tris, rays = _c(verts, np.float32), _c(tris, np.int32), _c(rays, np.float32)
    prims = _c(prims, np.int32)
    n = rays.shape[0]
    tuv = np.empty((n, 3), np.float32)
    hit = np.empty(n, np.int32)
    lib().orc_mt_fixed(_ptr(verts), _ptr(tris), tris.shape[0], _ptr(rays), n, _ptr(prims),
                       _ptr(tuv), _ptr(hit))
    return hit.astype(bool), tuv


def brute_closest(verts, tris, rays, nthreads: int = 0):
    """Exhaustive closest hit.  Returns (prim[n] int32, tuv[n,3] float32)."""
    verts, tris, rays = _c(verts, np.float32), _c(tris, np.int32), _c(rays, np.float32)
    n = rays.shape[0]
    prim = np.empty(n, np.int32)
    tuv = np.empty((n, 3), np.float32)
    lib().orc_brute_closest(_ptr(verts), _ptr(tris), tris.shape[0], _ptr(rays), n,
                            _ptr(prim), _ptr(tuv), nthreads)
    return prim, tuv


def brute_top2(verts, tris, rays, nthreads: int = 0):
    """Exhaustive best and runner-up.  Returns (prim[n,2], t[n,2])."""
    verts, tris, rays = _c(verts, np.float32), _c(tris, np.int32), _c(rays, np.float32)
    n = rays.shape[0]
    prim = np.empty((n, 2), np.int32)
    t = np.empty((n, 2), np.float32)
    lib().orc_brute_top2(_ptr(verts), _ptr(tris), tris.shape[0], _ptr(rays), n,
                         _ptr(prim), _ptr(t), nthreads)
    return prim, t


CLOSEST, TOP2, ANY = 0, 1, 2


class OracleBVH:
    """Median-split BVH with scalar stack traversal.  Keeps references to the
    vertex and triangle arrays for its lifetime."""

    def __init__(self, verts, tris):
        self.verts = _c(verts, np.float32)
        self.tris = _c(tris, np.int32)
        self._h = lib().orc_bvh_build(_ptr(self.verts), _ptr(self.tris), self.tris.shape[0])

    def close(self):
        if self._h:
            lib().orc_bvh_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def depth(self) -> int:
        return int(lib().orc_bvh_depth(self._h))

    @property
    def nnodes(self) -> int:
        return int(lib().orc_bvh_nnodes(self._h))

    def export(self):
        nn = self.nnodes
        boxes = np.empty((nn, 6), np.float32)
        links = np.empty((nn, 4), np.int32)
        perm = np.empty(self.tris.shape[0], np.int32)
        lib().orc_bvh_export(self._h, _ptr(boxes), _ptr(links), _ptr(perm))
        return boxes, links, perm

    def trace(self, rays, mode: int = CLOSEST, nthreads: int = 0):
        """Returns (prim[n], tuv[n,3]) for CLOSEST/ANY and additionally
        (prim2[n], t2[n]) for TOP2."""
        rays = _c(rays, np.float32)
        n = rays.shape[0]
        prim = np.empty(n, np.int32)
        tuv = np.empty((n, 3), np.float32)
        prim2 = np.empty(n, np.int32)
        t2 = np.empty(n, np.float32)
        lib().orc_bvh_trace(self._h, _ptr(rays), n, mode, _ptr(prim), _ptr(tuv),
                            _ptr(prim2), _ptr(t2), nthreads)
        if mode == TOP2:
            return prim, tuv, prim2, t2
        return prim, tuv

    def closest_point(self, queries, nthreads: int = 0):
        """Closest-point query through the BVH; same result as
        brute_closest_point."""
        queries = _c(queries, np.float32)
        assert queries.ndim == 2 and queries.shape[1] == 4
        n = queries.shape[0]
        prim = np.empty(n, np.int32)
        duv = np.empty((n, 3), np.float64)
        top2 = np.empty((n, 2), np.int32)
        d2top2 = np.empty((n, 2), np.float64)
        lib().orc_bvh_closest_point(self._h, _ptr(queries), n, _ptr(prim), _ptr(duv),
                                    _ptr(top2), _ptr(d2top2), nthreads)
        return prim, duv, top2, d2top2


def tuv_f64(verts, tris, rays, prims):
    """(t, u, v) in FP64 at fixed primitives; verts/rays are taken as float64."""
    verts = _c(verts, np.float64)
    tris = _c(tris, np.int32)
    rays = _c(rays, np.float64)
    prims = _c(prims, np.int32)
    n = prims.shape[0]
    out = np.empty((n, 3), np.float64)
    lib().orc_tuv_f64(_ptr(verts), _ptr(tris), _ptr(rays), _ptr(prims), n, _ptr(out))
    return out


def grad_f64(verts, tris, rays, prims, grad_hits, tuv_at=None):
    """Closed-form FP64 gradient at fixed primitives.

    tuv_at: optional [n,3] hit parameters at which to evaluate it (the
    oracle's own FP32 forward result); by default they are solved in FP64.
    Returns (grad_verts[V,3] f64, grad_rays[n,6] f64, tuv[n,3] f64)."""
    verts = _c(verts, np.float32)
    tris = _c(tris, np.int32)
    rays = _c(rays, np.float32)
    prims = _c(prims, np.int32)
    grad_hits = _c(grad_hits, np.float32)
    n = prims.shape[0]
    gv = np.zeros((verts.shape[0], 3), np.float64)
    gr = np.empty((n, 6), np.float64)
    tuv = np.empty((n, 3), np.float64)
    at = None
    if tuv_at is not None:
        at = _c(tuv_at, np.float32)
        assert at.shape == (n, 3)
    lib().orc_grad_f64(_ptr(verts), _ptr(tris), _ptr(rays), _ptr(prims), _ptr(grad_hits),
                       n, _ptr(gv), _ptr(gr), _ptr(tuv), _ptr(at) if at is not None else None)
    return gv, gr, tuv


def point_tri_f64(verts, tris, queries, prims):
    """(d2, u, v) in FP64 of queries[i] (x, y, z, r2) against triangle
    prims[i]; the nearest point is (1-u-v) p0 + u p1 + v p2.  prims < 0 give
    (inf, 0, 0)."""
    verts, tris = _c(verts, np.float32), _c(tris, np.int32)
    queries, prims = _c(queries, np.float32), _c(prims, np.int32)
    n = prims.shape[0]
    out = np.empty((n, 3), np.float64)
    lib().orc_point_tri_f64(_ptr(verts), _ptr(tris), _ptr(queries), _ptr(prims), n, _ptr(out))
    return out


def brute_closest_point(verts, tris, queries, nthreads: int = 0):
    """Exhaustive closest-point query (App. G "Closest Point Query").

    queries: [n,4] float32 (x, y, z, r2).  Returns (prim[n] int32, duv[n,3]
    float64 = (d2, u, v), top2[n,2] int32, d2top2[n,2] float64): the nearest
    triangle within r2 (else -1, inf, 0, 0) and, regardless of r2, the
    nearest and runner-up triangles and their squared distances."""
    verts, tris, queries = _c(verts, np.float32), _c(tris, np.int32), _c(queries, np.float32)
    assert queries.ndim == 2 and queries.shape[1] == 4
    n = queries.shape[0]
    prim = np.empty(n, np.int32)
    duv = np.empty((n, 3), np.float64)
    top2 = np.empty((n, 2), np.int32)
    d2top2 = np.empty((n, 2), np.float64)
    lib().orc_brute_closest_point(_ptr(verts), _ptr(tris), tris.shape[0], _ptr(queries), n,
                                  _ptr(prim), _ptr(duv), _ptr(top2), _ptr(d2top2), nthreads)
    return prim, duv, top2, d2top2


def sah_build(verts, tris):
    """Binned-SAH binary tree (32 bins; readings in oracle.c).  Returns
    (perm[n] int32, nodes[2n-1,4] int64 = (first, count, axis, left count) in
    preorder, boxes[2n-1,6] float32)."""
    verts, tris = _c(verts, np.float32), _c(tris, np.int32)
    n = tris.shape[0]
    perm = np.empty(max(n, 1), np.int32)
    nodes = np.empty((max(2 * n - 1, 1), 4), np.int64)
    boxes = np.empty((max(2 * n - 1, 1), 6), np.float32)
    m = lib().orc_sah_build(_ptr(verts), _ptr(tris), n, _ptr(perm), _ptr(nodes), _ptr(boxes))
    return perm[:n], nodes[:m], boxes[:m]


def collapse(nodes, leaf_size):
    """Preorder nodes of the tree whose subtrees of at most leaf_size
    primitives become leaves: rows (first, count, axis, left count, is_leaf)."""
    out = []
    i = 0
    stack = [0]
    while stack:
        i = stack.pop()
        first, count, axis, nl = (int(x) for x in nodes[i])
        if count <= leaf_size:
            out.append((first, count, axis, nl, 1, i))
            continue
        out.append((first, count, axis, nl, 0, i))
        stack.append(i + 2 * nl)
        stack.append(i + 1)
    return out


def max_threads() -> int:
    return int(lib().orc_max_threads())


def ambiguity_mask(t1, prim2, t2, rel: float = 1e-5):
    """Rays graded on prim_id: a miss, no runner-up, or a runner-up farther
    than rel * t1 behind the best hit."""
    t1 = np.asarray(t1, np.float64)
    t2 = np.asarray(t2, np.float64)
    miss = ~np.isfinite(t1)
    no_second = np.asarray(prim2) < 0
    with np.errstate(invalid="ignore"):
        sep = (t2 - t1) > rel * t1
    return miss | no_second | sep
