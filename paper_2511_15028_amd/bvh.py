"""Python binding of libbvh (include/bvh.h).

Argument marshalling only: every step of building and tracing runs in the
HIP library.  PyTorch supplies device memory and the stream.  If the
library has not been built, every call raises; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libbvh.so")

# enums of bvh.h
OK, EINVAL, ENOMEM, EHIP, ENODEV, EUNSUPPORTED = 0, -1, -2, -3, -4, -5
(LAYOUT_AABB2, LAYOUT_BVH4, LAYOUT_BVH8_Q8, LAYOUT_BVH8_Q16, LAYOUT_PBRT_Q16, LAYOUT_SG_EQ,
 LAYOUT_PBRT_SOAOS, LAYOUT_PBRT_Q16_SOAOS, LAYOUT_SG_EQ_A16, LAYOUT_SHARED_SLAB) = range(10)
LAYOUTS = {"aabb2": LAYOUT_AABB2, "bvh4": LAYOUT_BVH4, "bvh8_q8": LAYOUT_BVH8_Q8,
           "bvh8_q16": LAYOUT_BVH8_Q16, "pbrt_q16": LAYOUT_PBRT_Q16, "sg_eq": LAYOUT_SG_EQ,
           "pbrt_soaos": LAYOUT_PBRT_SOAOS, "pbrt_q16_soaos": LAYOUT_PBRT_Q16_SOAOS,
           "sg_eq_a16": LAYOUT_SG_EQ_A16, "shared_slab": LAYOUT_SHARED_SLAB}
LAYOUT_NAMES = {v: k for k, v in LAYOUTS.items()}
LEAF_COMPACT, LEAF_INDEXED = 0, 1
LEAF_MODES = {"compact": LEAF_COMPACT, "indexed": LEAF_INDEXED}
TRACE_CLOSEST, TRACE_ANY = 0, 1
NOALLOC_MAX_RAYS = 1 << 21  # BVH_NOALLOC_MAX_RAYS
BUF_NODES, BUF_LEAF = 0, 1
NODE_BYTES = {LAYOUT_AABB2: 32, LAYOUT_BVH4: 128, LAYOUT_BVH8_Q8: 128, LAYOUT_BVH8_Q16: 160,
              LAYOUT_PBRT_Q16: 16, LAYOUT_SG_EQ: 12, LAYOUT_PBRT_SOAOS: 32,
              LAYOUT_PBRT_Q16_SOAOS: 16, LAYOUT_SG_EQ_A16: 16, LAYOUT_SHARED_SLAB: 16}


class BVHError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"bvh error {code}: {msg}")
        self.code = code


class BuildOpts(ctypes.Structure):
    _fields_ = [("leaf_size", ctypes.c_int32), ("leaf_mode", ctypes.c_int32),
                ("stack_lds", ctypes.c_int32), ("builder", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]


class Stats(ctypes.Structure):
    _fields_ = [("layout", ctypes.c_int32), ("leaf_mode", ctypes.c_int32),
                ("arity", ctypes.c_int32), ("leaf_size", ctypes.c_int32),
                ("n_tris", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("n_leaves", ctypes.c_int64), ("node_bytes", ctypes.c_int64),
                ("nodes_buffer_bytes", ctypes.c_int64), ("leaf_buffer_bytes", ctypes.c_int64),
                ("extra_bytes", ctypes.c_int64), ("depth", ctypes.c_int32),
                ("max_stack", ctypes.c_int32), ("scene_lo", ctypes.c_float * 3),
                ("scene_hi", ctypes.c_float * 3), ("stack_lds", ctypes.c_int32),
                ("builder", ctypes.c_int32), ("frame_origin", ctypes.c_float * 3),
                ("frame_scale", ctypes.c_float * 3), ("frame_top", ctypes.c_float * 3),
                ("pad2", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        for k in ("scene_lo", "scene_hi", "frame_origin", "frame_scale", "frame_top"):
            d[k] = list(getattr(self, k))
        return d


_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_lib = None


class SceneDesc(ctypes.Structure):
    _fields_ = [("verts", _P), ("n_verts", _I64), ("tris", _P), ("n_tris", _I64),
                ("layout", _I32), ("stack_lds", _I32), ("reserved", _I32 * 2)]


class TuneOpts(ctypes.Structure):
    _fields_ = [("probe_rays", _I32), ("leaf_size", _I32), ("probe", _P),
                ("probe_offsets", ctypes.POINTER(_I64)), ("reserved", _I32 * 4)]


class SceneInfo(ctypes.Structure):
    _fields_ = [("layout", _I32), ("stack_lds", _I32), ("candidates", _I32),
                ("probe_ns_per_ray", ctypes.c_float), ("n_nodes", _I64), ("bvh_bytes", _I64)]


def lib() -> ctypes.CDLL:
    """Loads the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        L.bvh_last_error.restype = ctypes.c_char_p
        L.bvh_last_error.argtypes = []
        L.bvh_version.restype = _I32
        L.bvh_build.argtypes = [_P, _I64, _P, _I64, _I32, ctypes.POINTER(BuildOpts), _P,
                                ctypes.POINTER(_P)]
        L.bvh_build.restype = _I32
        L.bvh_destroy.argtypes = [_P]
        L.bvh_destroy.restype = _I32
        L.bvh_get_stats.argtypes = [_P, ctypes.POINTER(Stats)]
        L.bvh_get_stats.restype = _I32
        L.bvh_read_buffer.argtypes = [_P, _I32, _P, _I64, ctypes.POINTER(_I64)]
        L.bvh_read_buffer.restype = _I32
        L.bvh_trace.argtypes = [_P, _P, _I64, _P, _I32, _P]
        L.bvh_trace.restype = _I32
        L.bvh_trace_noalloc.argtypes = [_P, _P, _I64, _P, _I32, _P]
        L.bvh_trace_noalloc.restype = _I32
        L.bvh_trace_counts.argtypes = [_P, _P, _I64, _P, _I32, _P, _P]
        L.bvh_trace_counts.restype = _I32
        L.bvh_closest_point.argtypes = [_P, _P, _I64, _P, _P]
        L.bvh_closest_point.restype = _I32
        L.bvh_closest_point_counts.argtypes = [_P, _P, _I64, _P, _P, _P]
        L.bvh_closest_point_counts.restype = _I32
        L.bvh_trace_backward.argtypes = [_P, _I64, _P, _I64, _P, _I64, _P, _P, _P, _P, _P]
        L.bvh_trace_backward.restype = _I32
        L.bvh_batch_create.argtypes = [ctypes.POINTER(SceneDesc), _I32, ctypes.POINTER(TuneOpts),
                                       _P, ctypes.POINTER(_P)]
        L.bvh_batch_create.restype = _I32
        L.bvh_batch_get_scene_info.argtypes = [_P, _I32, ctypes.POINTER(SceneInfo)]
        L.bvh_batch_get_scene_info.restype = _I32
        L.bvh_batch_scene_handle.argtypes = [_P, _I32, ctypes.POINTER(_P)]
        L.bvh_batch_scene_handle.restype = _I32
        L.bvh_batch_trace.argtypes = [_P, _P, ctypes.POINTER(_I64), _P, _P]
        L.bvh_batch_trace.restype = _I32
        L.bvh_batch_destroy.argtypes = [_P]
        L.bvh_batch_destroy.restype = _I32
        _lib = L
    return _lib


def _check(rc: int):
    if rc != OK:
        raise BVHError(rc, lib().bvh_last_error().decode())


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _dev(t: torch.Tensor, dtype, cols: int, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}")
    if t.dim() != 2 or t.shape[1] != cols:
        raise ValueError(f"{name} must have shape [n, {cols}]")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _layout_id(layout) -> int:
    return LAYOUTS[layout] if isinstance(layout, str) else int(layout)


class BVH:
    """A built BVH.  Build with :func:`build`; a BVH taken from a
    :class:`Batch` is borrowed (the batch owns it)."""

    def __init__(self, handle: int, layout: int, leaf_mode: int, owned: bool = True):
        self._h = handle
        self.layout = layout
        self.leaf_mode = leaf_mode
        self._owned = owned

    def close(self):
        if self._h and self._owned:
            lib().bvh_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self) -> int:
        return self._h

    def stats(self) -> dict:
        s = Stats()
        _check(lib().bvh_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()

    def read_buffer(self, which: int) -> bytes:
        total = _I64(0)
        _check(lib().bvh_read_buffer(self._h, which, None, 0, ctypes.byref(total)))
        buf = ctypes.create_string_buffer(max(total.value, 1))
        _check(lib().bvh_read_buffer(self._h, which, buf, total.value, ctypes.byref(total)))
        return buf.raw[:total.value]

    def trace(self, rays: torch.Tensor, mode: int = TRACE_CLOSEST, hits: torch.Tensor = None,
              stream=None) -> torch.Tensor:
        """rays: [n,8] float32 device.  Returns hits [n,4] float32 whose first
        column holds the int32 primitive id bits (use :func:`prim_ids`)."""
        _dev(rays, torch.float32, 8, "rays")
        n = rays.shape[0]
        if hits is None:
            hits = torch.empty((n, 4), dtype=torch.float32, device=rays.device)
        _dev(hits, torch.float32, 4, "hits")
        _check(lib().bvh_trace(self._h, rays.data_ptr(), n, hits.data_ptr(), mode, _stream(stream)))
        return hits

    def trace_noalloc(self, rays: torch.Tensor, hits: torch.Tensor, mode: int = TRACE_CLOSEST,
                      stream=None) -> torch.Tensor:
        """bvh_trace_noalloc: like trace, into a caller-provided hits [n,4]
        tensor, with the library's fixed per-GPU work area (at most
        NOALLOC_MAX_RAYS rays; calls on one GPU must not overlap)."""
        _dev(rays, torch.float32, 8, "rays")
        _dev(hits, torch.float32, 4, "hits")
        if hits.shape[0] != rays.shape[0]:
            raise ValueError("hits must have one row per ray")
        _check(lib().bvh_trace_noalloc(self._h, rays.data_ptr(), rays.shape[0], hits.data_ptr(),
                                       mode, _stream(stream)))
        return hits

    def trace_counts(self, rays: torch.Tensor, mode: int = TRACE_CLOSEST, stream=None):
        """Like trace, plus per-ray (nodes fetched, triangles tested) int32 [n,2]."""
        _dev(rays, torch.float32, 8, "rays")
        n = rays.shape[0]
        hits = torch.empty((n, 4), dtype=torch.float32, device=rays.device)
        counts = torch.zeros((n, 2), dtype=torch.int32, device=rays.device)
        _check(lib().bvh_trace_counts(self._h, rays.data_ptr(), n, hits.data_ptr(), mode,
                                      counts.data_ptr(), _stream(stream)))
        return hits, counts

    def closest_point(self, queries: torch.Tensor, out: torch.Tensor = None,
                      stream=None) -> torch.Tensor:
        """queries: [n,4] float32 device (x, y, z, r2).  Returns [n,4] float32
        (prim id bits, d2, u, v); see :func:`prim_ids`."""
        _dev(queries, torch.float32, 4, "queries")
        n = queries.shape[0]
        if out is None:
            out = torch.empty((n, 4), dtype=torch.float32, device=queries.device)
        _dev(out, torch.float32, 4, "out")
        _check(lib().bvh_closest_point(self._h, queries.data_ptr(), n, out.data_ptr(),
                                       _stream(stream)))
        return out

    def closest_point_counts(self, queries: torch.Tensor, stream=None):
        """Like closest_point, plus per-query (nodes fetched, triangles
        measured) int32 [n,2]."""
        _dev(queries, torch.float32, 4, "queries")
        n = queries.shape[0]
        out = torch.empty((n, 4), dtype=torch.float32, device=queries.device)
        counts = torch.zeros((n, 2), dtype=torch.int32, device=queries.device)
        _check(lib().bvh_closest_point_counts(self._h, queries.data_ptr(), n, out.data_ptr(),
                                              counts.data_ptr(), _stream(stream)))
        return out, counts


BUILDERS = {"lbvh": 0, "sah": 1}


def build(verts: torch.Tensor, tris: torch.Tensor, layout="bvh8_q8", leaf_size: int = 4,
          leaf_mode="compact", stream=None, stack_lds: int = 0, builder="lbvh") -> BVH:
    """verts [V,3] float32 device, tris [N,3] int32 device; builder "lbvh"
    (Morton order, Karras hierarchy) or "sah" (binned SAH, 32 bins)."""
    _dev(verts, torch.float32, 3, "verts")
    _dev(tris, torch.int32, 3, "tris")
    lm = LEAF_MODES[leaf_mode] if isinstance(leaf_mode, str) else int(leaf_mode)
    lid = _layout_id(layout)
    bid = BUILDERS[builder] if isinstance(builder, str) else int(builder)
    opts = BuildOpts(leaf_size, lm, stack_lds, bid)
    h = _P()
    _check(lib().bvh_build(verts.data_ptr(), verts.shape[0], tris.data_ptr(), tris.shape[0], lid,
                           ctypes.byref(opts), _stream(stream), ctypes.byref(h)))
    return BVH(h.value, lid, lm)


def prim_ids(hits: torch.Tensor) -> torch.Tensor:
    return hits[:, 0].contiguous().view(torch.int32)


def trace_backward(verts, tris, rays, hits, grad_hits, grad_verts=None, stream=None):
    """Returns (grad_verts [V,3] (accumulated into if given), grad_rays [n,6])."""
    _dev(verts, torch.float32, 3, "verts")
    _dev(tris, torch.int32, 3, "tris")
    _dev(rays, torch.float32, 8, "rays")
    _dev(hits, torch.float32, 4, "hits")
    _dev(grad_hits, torch.float32, 3, "grad_hits")
    n = rays.shape[0]
    if grad_verts is None:
        grad_verts = torch.zeros_like(verts)
    _dev(grad_verts, torch.float32, 3, "grad_verts")
    grad_rays = torch.empty((n, 6), dtype=torch.float32, device=rays.device)
    _check(lib().bvh_trace_backward(verts.data_ptr(), verts.shape[0], tris.data_ptr(),
                                    tris.shape[0], rays.data_ptr(), n, hits.data_ptr(),
                                    grad_hits.data_ptr(), grad_verts.data_ptr(),
                                    grad_rays.data_ptr(), _stream(stream)))
    return grad_verts, grad_rays


class BVHTrace(torch.autograd.Function):
    """Differentiable closest hit.

    forward(verts, tris, origins [n,3], dirs [n,3], bvh, tmax=None) returns
    (prim [n] int32, tuv [n,3] float32); gradients flow to verts, origins and
    dirs through (t, u, v) with each ray's hit primitive held fixed.  The BVH
    must have been built from the same verts/tris."""

    @staticmethod
    def forward(ctx, verts, tris, origins, dirs, bvh, tmax=None):
        n = origins.shape[0]
        rays = torch.zeros((n, 8), dtype=torch.float32, device=origins.device)
        rays[:, 0:3] = origins.detach()
        rays[:, 4:7] = dirs.detach()
        rays[:, 7] = float("inf") if tmax is None else tmax
        hits = bvh.trace(rays)
        ctx.save_for_backward(verts.detach(), tris, rays, hits)
        prim = prim_ids(hits)
        ctx.mark_non_differentiable(prim)
        return prim, hits[:, 1:4].clone()

    @staticmethod
    def backward(ctx, grad_prim, grad_tuv):
        verts, tris, rays, hits = ctx.saved_tensors
        if grad_tuv is None:
            return None, None, None, None, None, None
        gv, gr = trace_backward(verts, tris, rays, hits, grad_tuv.contiguous().float())
        return gv, None, gr[:, 0:3], gr[:, 3:6], None, None


class Batch:
    """Many scenes traced by one graph launch (bvh_batch_*).

    scenes: list of (verts [V,3] f32, tris [N,3] i32) device tensors.
    layout / stack_lds: None lets the tuner choose per scene; a value (or a
    per-scene list) fixes it.  probe / probe_offsets: optional device rays and
    host offsets for the tuner."""

    def __init__(self, scenes, layout=None, stack_lds=None, probe=None, probe_offsets=None,
                 probe_rays: int = 0, leaf_size: int = 4, stream=None):
        n = len(scenes)
        descs = (SceneDesc * n)()
        lay = layout if isinstance(layout, (list, tuple)) else [layout] * n
        sls = stack_lds if isinstance(stack_lds, (list, tuple)) else [stack_lds] * n
        for i, (v, t) in enumerate(scenes):
            _dev(v, torch.float32, 3, "verts")
            _dev(t, torch.int32, 3, "tris")
            descs[i].verts = v.data_ptr()
            descs[i].n_verts = v.shape[0]
            descs[i].tris = t.data_ptr()
            descs[i].n_tris = t.shape[0]
            descs[i].layout = -1 if lay[i] is None else _layout_id(lay[i])
            descs[i].stack_lds = 0 if sls[i] is None else int(sls[i])
        opts = TuneOpts(probe_rays, leaf_size)
        self._probe_off = None
        if probe is not None:
            _dev(probe, torch.float32, 8, "probe")
            self._probe_off = (_I64 * (n + 1))(*[int(x) for x in probe_offsets])
            opts.probe = probe.data_ptr()
            opts.probe_offsets = self._probe_off
        b = _P()
        _check(lib().bvh_batch_create(descs, n, ctypes.byref(opts), _stream(stream), ctypes.byref(b)))
        self._b = b.value
        self.n_scenes = n
        self._off = None

    def close(self):
        if self._b:
            lib().bvh_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self, i: int) -> dict:
        s = SceneInfo()
        _check(lib().bvh_batch_get_scene_info(self._b, i, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in s._fields_}

    def handle(self, i: int) -> BVH:
        h = _P()
        _check(lib().bvh_batch_scene_handle(self._b, i, ctypes.byref(h)))
        inf = self.info(i)
        return BVH(h.value, inf["layout"], LEAF_COMPACT, owned=False)

    def trace(self, rays: torch.Tensor, offsets, hits: torch.Tensor = None, stream=None):
        """rays [n,8] device; offsets: n_scenes + 1 ray offsets (host ints)."""
        _dev(rays, torch.float32, 8, "rays")
        if hits is None:
            hits = torch.empty((rays.shape[0], 4), dtype=torch.float32, device=rays.device)
        _dev(hits, torch.float32, 4, "hits")
        off = [int(x) for x in offsets]
        if len(off) != self.n_scenes + 1:
            raise ValueError("offsets must have n_scenes + 1 entries")
        if off[-1] > rays.shape[0] or off[-1] > hits.shape[0]:
            raise ValueError("offsets exceed the ray or hit buffer")
        self._off = (_I64 * (self.n_scenes + 1))(*off)
        _check(lib().bvh_batch_trace(self._b, rays.data_ptr(), self._off, hits.data_ptr(),
                                     _stream(stream)))
        return hits
