"""Numpy decoder of the node records documented in include/bvh.h.

Written from the header's format description only (it shares nothing with
the HIP sources), so that a packed BVH can be decoded on the CPU and
compared with the geometry: the round trip of Sec. B (dec(enc(t)) = t),
with quantised boxes required to contain the exact ones (Sec. 9.1 footnote).
"""
from __future__ import annotations

import numpy as np

AABB2, BVH4, BVH8_Q8, BVH8_Q16, PBRT_Q16, SG_EQ = 0, 1, 2, 3, 4, 5
PBRT_SOAOS, PBRT_Q16_SOAOS, SG_EQ_A16, SHARED_SLAB = 6, 7, 8, 9

AABB2_DT = np.dtype([("lo", "<f4", 3), ("hi", "<f4", 3), ("offset", "<u4"), ("meta", "<u4")])
BVH4_DT = np.dtype([("lo_x", "<f4", 4), ("lo_y", "<f4", 4), ("lo_z", "<f4", 4),
                    ("hi_x", "<f4", 4), ("hi_y", "<f4", 4), ("hi_z", "<f4", 4),
                    ("child", "<u4", 4), ("nchild", "<u4"), ("pad", "<u4", 3)])
Q8_DT = np.dtype([("origin", "<f4", 3), ("scale", "<f4", 3),
                  ("qlo_x", "u1", 8), ("qlo_y", "u1", 8), ("qlo_z", "u1", 8),
                  ("qhi_x", "u1", 8), ("qhi_y", "u1", 8), ("qhi_z", "u1", 8),
                  ("child", "<u4", 8), ("nchild", "<u4"), ("pad", "<u4", 5)])
Q16_DT = np.dtype([("origin", "<f4", 3), ("scale", "<f4", 3),
                   ("qlo_x", "<u2", 8), ("qlo_y", "<u2", 8), ("qlo_z", "<u2", 8),
                   ("qhi_x", "<u2", 8), ("qhi_y", "<u2", 8), ("qhi_z", "<u2", 8),
                   ("child", "<u4", 8), ("nchild", "<u4"), ("pad", "<u4")])
PQ16_DT = np.dtype([("lo", "<u2", 3), ("hi", "<u2", 3), ("meta", "<u4")])
SGEQ_DT = np.dtype([("qlo", "<u4"), ("qhi", "<u4"), ("off", "<u4")])
TRI_DT = np.dtype([("p0", "<f4", 3), ("e1", "<f4", 3), ("e2", "<f4", 3), ("prim", "<i4"),
                   ("pad", "<i4", 2)])
assert AABB2_DT.itemsize == 32 and BVH4_DT.itemsize == 128
assert Q8_DT.itemsize == 128 and Q16_DT.itemsize == 160 and TRI_DT.itemsize == 48
assert PQ16_DT.itemsize == 16 and SGEQ_DT.itemsize == 12

DTYPES = {AABB2: AABB2_DT, BVH4: BVH4_DT, BVH8_Q8: Q8_DT, BVH8_Q16: Q16_DT, PBRT_Q16: PQ16_DT,
          SG_EQ: SGEQ_DT}
BOXF_DT = np.dtype([("lo", "<f4", 3), ("hi", "<f4", 3)])
TOPO_DT = np.dtype([("offset", "<u4"), ("meta", "<u4")])
BOXQ_DT = np.dtype([("lo", "<u2", 3), ("hi", "<u2", 3)])
SGEQ16_DT = np.dtype([("qlo", "<u4"), ("qhi", "<u4"), ("off", "<u4"), ("pad", "<u4")])
assert BOXF_DT.itemsize == 24 and TOPO_DT.itemsize == 8 and BOXQ_DT.itemsize == 12
assert SGEQ16_DT.itemsize == 16
VARIANT_BYTES = {PBRT_SOAOS: 32, PBRT_Q16_SOAOS: 16, SG_EQ_A16: 16}
SLAB_DT = np.dtype([("slo", "<f4"), ("shi", "<f4"), ("offset", "<u4"), ("meta", "<u4")])
assert SLAB_DT.itemsize == 16
DTYPES[SHARED_SLAB] = SLAB_DT


def as_base(layout, nodes_bytes):
    """A variant's node buffer re-assembled as the base layout's records:
    (base layout, records).  SoAoS: n box entries, then n topology entries;
    align16: sg-eq records plus a zero word."""
    if layout == PBRT_SOAOS:
        n = len(nodes_bytes) // 32
        box = np.frombuffer(nodes_bytes[:24 * n], BOXF_DT)
        topo = np.frombuffer(nodes_bytes[24 * n:], TOPO_DT)
        rec = np.zeros(n, AABB2_DT)
        rec["lo"], rec["hi"] = box["lo"], box["hi"]
        rec["offset"], rec["meta"] = topo["offset"], topo["meta"]
        return AABB2, rec
    if layout == PBRT_Q16_SOAOS:
        n = len(nodes_bytes) // 16
        box = np.frombuffer(nodes_bytes[:12 * n], BOXQ_DT)
        meta = np.frombuffer(nodes_bytes[12 * n:], "<u4")
        rec = np.zeros(n, PQ16_DT)
        rec["lo"], rec["hi"], rec["meta"] = box["lo"], box["hi"], meta
        return PBRT_Q16, rec
    if layout == SG_EQ_A16:
        r16 = np.frombuffer(nodes_bytes, SGEQ16_DT)
        assert (r16["pad"] == 0).all()
        rec = np.zeros(len(r16), SGEQ_DT)
        rec["qlo"], rec["qhi"], rec["off"] = r16["qlo"], r16["qhi"], r16["off"]
        return SG_EQ, rec
    return layout, np.frombuffer(nodes_bytes, DTYPES[layout])


def fma32(q, s, o):
    """Correctly rounded fmaf(q, s, o) for q < 2^16, vectorised.

    q*s is exact in float64 (at most 16 + 24 significant bits); adding o
    rounds once in float64 and the cast to float32 rounds again.  The two
    roundings can differ from one correct rounding only when the float64 sum
    lands exactly on a float32 midpoint; those elements are redone with
    exact rational arithmetic."""
    q = np.asarray(q, np.float64)
    s = np.asarray(s, np.float32).astype(np.float64)
    o = np.asarray(o, np.float32).astype(np.float64)
    shape = np.broadcast(q, s, o).shape
    q, s, o = (np.atleast_1d(x) for x in np.broadcast_arrays(q, s, o))
    y = q * s + o
    f = y.astype(np.float32)
    lo = np.nextafter(f, np.float32(-np.inf)).astype(np.float64)
    hi = np.nextafter(f, np.float32(np.inf)).astype(np.float64)
    f64 = f.astype(np.float64)
    amb = (y == 0.5 * (lo + f64)) | (y == 0.5 * (f64 + hi))
    if amb.any():
        from fractions import Fraction
        for idx in zip(*np.nonzero(amb)):
            exact = Fraction(float(q[idx])) * Fraction(float(s[idx])) + Fraction(float(o[idx]))
            f[idx] = _round_f32(exact)
    return f.reshape(shape)


def _round_f32(x):
    """Round a Fraction to the nearest float32 (ties to even)."""
    from fractions import Fraction
    f = np.float32(float(x))
    best = None
    for c in (np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))):
        if not np.isfinite(c):
            continue
        key = (abs(Fraction(float(c)) - x), int(np.float32(c).view(np.uint32)) & 1)
        if best is None or key < best[0]:
            best = (key, c)
    return best[1]


def decode_ref(ref):
    """Tagged child reference -> ("node", index) or ("leaf", first, n)."""
    ref = int(ref)
    if ref & 1:
        return ("node", ref >> 1)
    return ("leaf", ref >> 5, ((ref >> 1) & 0xF) + 1)


def child_boxes(layout, rec):
    """Decoded child boxes [K,6] (lo xyz, hi xyz) as float32 for one wide node."""
    if layout == BVH4:
        return np.stack([rec["lo_x"], rec["lo_y"], rec["lo_z"],
                         rec["hi_x"], rec["hi_y"], rec["hi_z"]], axis=1).astype(np.float32)
    o, s = rec["origin"], rec["scale"]
    cols = []
    for name, a in (("qlo_x", 0), ("qlo_y", 1), ("qlo_z", 2), ("qhi_x", 0), ("qhi_y", 1), ("qhi_z", 2)):
        cols.append(fma32(rec[name].astype(np.float64), s[a], o[a]))
    return np.stack(cols, axis=1)


def pbrt_q16_box(rec, frame):
    """Decoded box (lo xyz, hi xyz) of one pbrt-q16 node in the scene frame
    (frame = (origin[3], scale[3], ...))."""
    o, s = (np.asarray(x, np.float32) for x in frame[:2])
    lo = fma32(rec["lo"].astype(np.float64), s, o)
    hi = fma32(rec["hi"].astype(np.float64), s, o)
    return np.concatenate([lo, hi]).astype(np.float32)


def sg_eq_fields(rec):
    """(qlo[3], qhi[3], nprims, offset, axis) of sg-eq records (vectorised)."""
    ql = np.asarray(rec["qlo"], np.uint64)
    qh = np.asarray(rec["qhi"], np.uint64)
    w = np.asarray(rec["off"], np.uint64)
    qlo = np.stack([(ql >> 20) & 1023, (ql >> 10) & 1023, ql & 1023], axis=-1)
    qhi = np.stack([(qh >> 20) & 1023, (qh >> 10) & 1023, qh & 1023], axis=-1)
    nprim = (ql >> 30) | ((qh >> 30) << 2)
    return qlo, qhi, nprim, w & 0x3FFFFFFF, w >> 30


def sg_eq_box(rec, frame):
    """Decoded box of one sg-eq node; frame = (origin, scale, top)."""
    o, s, top = (np.asarray(x, np.float32) for x in frame)
    qlo, qhi, _, _, _ = sg_eq_fields(rec)
    lo = fma32(qlo.astype(np.float64), s, o)
    hi = fma32(-qhi.astype(np.float64), s, top)
    return np.concatenate([lo, hi]).astype(np.float32)


def walk(layout, nodes_bytes, frame=None):
    """Decodes a packed tree.  Returns a list of leaves (first, n, box or None,
    path boxes) and the count of visited nodes; raises on malformed records.
    frame: the scene frame of PBRT_Q16 (origin[3], scale[3])."""
    layout, nodes = as_base(layout, nodes_bytes)
    leaves = []
    visited = np.zeros(len(nodes), np.int64)
    if len(nodes) == 0:
        return nodes, leaves, visited
    if layout == SHARED_SLAB:
        # frame = (scene lo, scene hi): the root's inherited box
        root = np.concatenate([np.asarray(frame[0], np.float32), np.asarray(frame[1], np.float32)])
        stack = [(0, root, [])]
        while stack:
            i, carried, path = stack.pop()
            visited[i] += 1
            rec = nodes[i]
            meta = int(rec["meta"])
            a = (meta >> 16) & 3
            assert a < 3
            box = carried.copy()
            box[a], box[3 + a] = rec["slo"], rec["shi"]
            nprim = meta & 0xFFFF
            if nprim > 0:
                leaves.append((int(rec["offset"]), nprim, path + [box]))
            else:
                assert rec["offset"] >= 2
                stack.append((i + 1, box, path + [box]))
                stack.append((i + int(rec["offset"]), box, path + [box]))
        return nodes, leaves, visited
    if layout in (PBRT_Q16, SG_EQ):
        stack = [(0, [])]
        while stack:
            i, path = stack.pop()
            visited[i] += 1
            rec = nodes[i]
            if layout == PBRT_Q16:
                box = pbrt_q16_box(rec, frame)
                meta = int(rec["meta"])
                nprim, off = meta & 0xF, meta >> 4
            else:
                box = sg_eq_box(rec, frame)
                _, _, nprim, off, _ = sg_eq_fields(rec)
                nprim, off = int(nprim), int(off)
            if nprim > 0:
                leaves.append((off, nprim, path + [box]))
            else:
                assert off >= 2
                stack.append((i + 1, path + [box]))
                stack.append((i + off, path + [box]))
        return nodes, leaves, visited
    if layout == AABB2:
        stack = [(0, [])]
        while stack:
            i, path = stack.pop()
            visited[i] += 1
            rec = nodes[i]
            box = np.concatenate([rec["lo"], rec["hi"]]).astype(np.float32)
            nprim = int(rec["meta"]) & 0xFFFF
            if nprim > 0:
                leaves.append((int(rec["offset"]), nprim, path + [box]))
            else:
                assert rec["offset"] >= 2
                stack.append((i + 1, path + [box]))
                stack.append((i + int(rec["offset"]), path + [box]))
        return nodes, leaves, visited
    stack = [(0, [])]
    while stack:
        i, path = stack.pop()
        visited[i] += 1
        rec = nodes[i]
        nc = int(rec["nchild"])
        assert 1 <= nc <= len(rec["child"])
        boxes = child_boxes(layout, rec)
        for c in range(nc):
            r = decode_ref(rec["child"][c])
            if r[0] == "node":
                stack.append((r[1], path + [boxes[c]]))
            else:
                leaves.append((r[1], r[2], path + [boxes[c]]))
        for c in range(nc, len(rec["child"])):
            assert int(rec["child"][c]) == 0xFFFFFFFF
    return nodes, leaves, visited
