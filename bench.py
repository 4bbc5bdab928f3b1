"""Benchmark: closest-hit BVH traversal on one MI355X.

Workload: the procedural terrain (1024 x 1024 cells = 2,097,152 triangles,
heights from 6-octave value noise, amplitude 0.2), 1920 x 1080 coherent
camera rays plus one cosine-distributed diffuse bounce ray per hit
(incoherent).  Inputs are generated on the host, uploaded once and stay
resident in HBM; the bounce rays are made from the GPU's own camera hits
before timing starts.

One step = one pass of the hot path over that input: build the BVH on the
GPU (bounds, Morton codes, radix sort, hierarchy, refit, collapse, packing
into the node layout) and trace the camera rays and the bounce rays.
`value` = rays traced per step / step time, in Mrays/s.

Also reported: per-layout trace-only throughput and algorithmic bytes per
ray (from the counting kernel), the roofline of the traversal kernel
(timed with HIP events on the launch stream), closest-point query
throughput per layout on the terrain and sphere scenes, the differentiable
workload's forward and forward+backward throughput, batched tracing, and
the CPU oracle timed on the host cores.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--layout L]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak, GB/s
# VALU peak in lane operations per second: 256 CUs x 4 SIMDs x 16 lanes, one
# FP32/integer operation per lane per clock (fused multiply-add counted as
# one operation; packed FP32 is not used), at 2.4 GHz.
ALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12  # 39.32 T lane-ops/s

# Algorithmic VALU operations per unit of traversal work (the arithmetic the
# method needs, address arithmetic, loads, loop control and stack traffic
# excluded):
#   one ray/box slab test: 6 plane distances (one FMA each), 3 max for the
#     entry distance (with 0), 3 min for the exit distance (with the current
#     best), the exit widening (1 mul), the compare and the select: 15;
#   dequantising one quantised box: 6 planes x (field extract, int->float
#     convert, one FMA): 18;
#   one ray/triangle test: the numerators and |det| (31: 3 cross products of
#     2 ops per component less the shared ones, 3 dot products of 3 ops, 3
#     subtractions for o - p0, 3 sign xors, one abs) and the interval tests
#     (7 compares, one add, one multiply): 40; indexed leaves also form the
#     two edges from the three gathered vertices (6 subtractions): 46.
# A node record fetched costs the box tests of every child slot it holds
# (binary layouts: the node's own box).
ALU_OPS_BOX, ALU_OPS_DEQUANT = 15, 18
ALU_OPS_TRI = {"compact": 40, "indexed": 46}
ALU_OPS_NODE = {
    "aabb2": ALU_OPS_BOX, "pbrt_soaos": ALU_OPS_BOX, "shared_slab": ALU_OPS_BOX,
    "pbrt_q16": ALU_OPS_BOX + ALU_OPS_DEQUANT, "sg_eq": ALU_OPS_BOX + ALU_OPS_DEQUANT,
    "pbrt_q16_soaos": ALU_OPS_BOX + ALU_OPS_DEQUANT, "sg_eq_a16": ALU_OPS_BOX + ALU_OPS_DEQUANT,
    "bvh4": 4 * ALU_OPS_BOX,
    "bvh8_q8": 8 * (ALU_OPS_BOX + ALU_OPS_DEQUANT), "bvh8_q16": 8 * (ALU_OPS_BOX + ALU_OPS_DEQUANT),
}
# Closest-point queries, the same model: one point/box distance (per axis two
# subtractions and two maxima, then one multiply and two FMAs for the squared
# distance, the conservative scale and the compare with the best): 17; one
# point/triangle test (Ericson's regions, written branch-free: the three
# offsets p - a, p - b, p - c (9), six dot products (18), the three
# sub-determinants (6), the region flags (26), the chosen region's division
# as a reciprocal and a multiply with its operand selects (14), the
# barycentrics and their selects (16), the face check (12), the point, its
# offset and squared distance (12), the best update (5)): 118.
ALU_OPS_CP_BOX, ALU_OPS_CP_TRI = 17, 118
ALU_OPS_CP_NODE = {  # per node record fetched: the distance to every box it holds
    "aabb2": ALU_OPS_CP_BOX, "pbrt_soaos": ALU_OPS_CP_BOX, "shared_slab": ALU_OPS_CP_BOX,
    "pbrt_q16": ALU_OPS_CP_BOX + ALU_OPS_DEQUANT, "sg_eq": ALU_OPS_CP_BOX + ALU_OPS_DEQUANT,
    "pbrt_q16_soaos": ALU_OPS_CP_BOX + ALU_OPS_DEQUANT, "sg_eq_a16": ALU_OPS_CP_BOX + ALU_OPS_DEQUANT,
    "bvh4": 4 * ALU_OPS_CP_BOX,
    "bvh8_q8": 8 * (ALU_OPS_CP_BOX + ALU_OPS_DEQUANT), "bvh8_q16": 8 * (ALU_OPS_CP_BOX + ALU_OPS_DEQUANT),
}
RAY_BYTES, HIT_BYTES = 32, 16
# Backward, algorithmic bytes per ray: the ray (32), its hit record (16), the
# loss gradient g (12), the triangle's indices (12) and three vertices (36) in;
# the ray gradient (24) out, and three vertex-gradient rows read and written
# (2 x 36).
BWD_BYTES_PER_RAY = 32 + 16 + 12 + 12 + 36 + 24 + 2 * 36
QUERY_BYTES, CLOSEST_BYTES = 16, 16  # bvh_point_query, bvh_closest
LAYOUTS = ("aabb2", "bvh4", "bvh8_q8", "bvh8_q16", "pbrt_q16", "sg_eq", "pbrt_soaos",
           "pbrt_q16_soaos", "sg_eq_a16", "shared_slab")
LEAF_TRI_BYTES = {"compact": 48, "indexed": 4 + 12 + 36}  # record, or id + index + 3 verts


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--layout", default="bvh4")
    ap.add_argument("--leaf-mode", default="compact")
    ap.add_argument("--leaf-size", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip per-layout table and fwd+bwd")
    ap.add_argument("--layouts", default=",".join(LAYOUTS),
                    help="layouts of the per_layout and spheres sections (comma-separated)")
    ap.add_argument("--no-sah-rows", action="store_true",
                    help="skip the SAH-tree rows of the spheres section")
    ap.add_argument("--sections", default="per_layout,sah,closest_point,fwd_bwd,spheres,batched",
                    help="comma-separated extra sections to run (default: all)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run an elementwise kernel over this many MiB (counter calibration)")
    return ap.parse_args()


def algorithmic_bytes(counts, layout_bytes, leaf_mode):
    """Per-ray bytes the method must move: ray + hit + node records fetched +
    triangles tested (from the counting kernel)."""
    nodes = counts[:, 0].astype(np.float64)
    tris = counts[:, 1].astype(np.float64)
    return RAY_BYTES + HIT_BYTES + nodes * layout_bytes + tris * LEAF_TRI_BYTES[leaf_mode]


def algorithmic_ops(counts, layout, leaf_mode):
    """Per-ray algorithmic VALU lane operations: node records fetched x the
    layout's box-test cost + triangles tested x the triangle-test cost."""
    nodes = counts[:, 0].astype(np.float64)
    tris = counts[:, 1].astype(np.float64)
    return nodes * ALU_OPS_NODE[layout] + tris * ALU_OPS_TRI[leaf_mode]


def trimmed_mean(times):
    """The paper's protocol (Sec. 9.1): of nine timed runs after a warm-up,
    drop the two lowest and the two highest and average the middle five."""
    t = sorted(times)
    assert len(t) == 9, len(t)
    return float(np.mean(t[2:7]))


COUNTERS_FILE = os.path.join(ROOT, "profiles", "trace_kernel_counters.txt")
TRAVERSAL_SOURCES = [os.path.join(ROOT, "paper_2511_15028_amd", "csrc", f)
                     for f in ("traverse.h", "trace.hip")]


def traversal_source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in TRAVERSAL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(args):
    """HBM bytes per traversal launch pair (camera + bounce) from the committed
    rocprofv3 counter summary, scaled by its calibration factors; None when the
    summary is missing, was taken for another configuration, or the traversal
    sources changed since."""
    try:
        kv = {}
        with open(COUNTERS_FILE) as fh:
            for line in fh:
                if "=" in line and not line.startswith("#"):
                    k, v = line.split("=", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_digest") != traversal_source_digest():
            return None
        if kv.get("layout") != args.layout or kv.get("leaf_mode") != args.leaf_mode:
            return None
        return int(float(kv["hbm_bytes_per_step_launches"]))
    except (OSError, KeyError, ValueError):
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); rays shard across GPUs "
              "without communication, so the one-GPU number is the per-GPU share.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2511_15028_amd import bvh, workloads as W

    bvh.lib()  # fails loudly if the HIP library is missing
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    t0 = time.time()
    w = W.terrain_workload()
    verts = torch.from_numpy(w["verts"]).to(dev)
    tris = torch.from_numpy(w["tris"]).to(dev)
    prim_rays = torch.from_numpy(w["rays"]).to(dev)
    log(f"generated terrain: {w['tris'].shape[0]} tris, {w['rays'].shape[0]} camera rays "
        f"({time.time() - t0:.1f}s)")

    # bounce rays from the GPU's own camera hits (untimed setup)
    h0 = bvh.build(verts, tris, args.layout, args.leaf_size, args.leaf_mode)
    hits0 = h0.trace(prim_rays)
    torch.cuda.synchronize()
    hh = hits0.cpu().numpy()
    prim0 = hh[:, 0].view(np.int32)
    bounce_np, _ = W.bounce_rays(w["rays"], prim0, hh[:, 1], w["verts"], w["tris"], seed=1001)
    bounce_rays = torch.from_numpy(bounce_np).to(dev)
    h0.close()
    n_rays = prim_rays.shape[0] + bounce_rays.shape[0]
    log(f"bounce rays: {bounce_rays.shape[0]}")

    hits_p = torch.empty((prim_rays.shape[0], 4), dtype=torch.float32, device=dev)
    hits_b = torch.empty((bounce_rays.shape[0], 4), dtype=torch.float32, device=dev)

    def step(ev=None):
        h = bvh.build(verts, tris, args.layout, args.leaf_size, args.leaf_mode)
        if ev is not None:
            ev[0].record(stream)
        h.trace(prim_rays, hits=hits_p)
        if ev is not None:
            ev[1].record(stream)
            ev[2].record(stream)
        h.trace(bounce_rays, hits=hits_b)
        if ev is not None:
            ev[3].record(stream)
        return h

    for _ in range(args.warmup):
        step().close()
    torch.cuda.synchronize()
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    handles = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        handles.append(step(events[k]))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    for h in handles:
        h.close()
    ms_step = 1000.0 * t_total / args.steps
    dur_p = np.array([e[0].elapsed_time(e[1]) for e in events])
    dur_b = np.array([e[2].elapsed_time(e[3]) for e in events])
    value = n_rays / (t_total / args.steps) / 1e6

    # measurement-only passes (outside the timed region)
    h = bvh.build(verts, tris, args.layout, args.leaf_size, args.leaf_mode)
    st = h.stats()
    _, cnt_p = h.trace_counts(prim_rays)
    _, cnt_b = h.trace_counts(bounce_rays)
    torch.cuda.synchronize()
    cnt_p, cnt_b = cnt_p.cpu().numpy(), cnt_b.cpu().numpy()
    bytes_p = algorithmic_bytes(cnt_p, st["node_bytes"], args.leaf_mode)
    bytes_b = algorithmic_bytes(cnt_b, st["node_bytes"], args.leaf_mode)
    ops_p = algorithmic_ops(cnt_p, args.layout, args.leaf_mode)
    ops_b = algorithmic_ops(cnt_b, args.layout, args.leaf_mode)
    # dominant kernel: the traversal kernel; two launches per step (camera, bounce)
    launch_bytes = bytes_p.sum() + bytes_b.sum()
    launch_s = (dur_p.mean() + dur_b.mean()) / 1000.0
    achieved_gbs = launch_bytes / launch_s / 1e9
    achieved_tops = (ops_p.sum() + ops_b.sum()) / launch_s / 1e12
    traffic = measured_traffic(args)
    trace_mrays = n_rays / launch_s / 1e6
    build_ms = ms_step - (dur_p.mean() + dur_b.mean())
    h.close()

    out = {
        "metric": "Mrays/s closest-hit per layout, % HBM roofline; batched & fwd+bwd vs plain",
        "value": round(value, 3),
        "unit": "Mrays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "terrain 1024x1024 cells (2,097,152 tris), 1920x1080 camera rays + 1 "
                        "diffuse bounce per hit; step = GPU BVH build + trace of both ray sets",
            "layout": args.layout, "leaf_mode": args.leaf_mode, "leaf_size": args.leaf_size,
            "rays_per_step": int(n_rays), "camera_rays": int(prim_rays.shape[0]),
            "bounce_rays": int(bounce_rays.shape[0]),
        },
        "trace_mrays_s": round(trace_mrays, 2),
        "trace_ms": {"camera": round(float(dur_p.mean()), 4), "bounce": round(float(dur_b.mean()), 4)},
        "build_ms": round(build_ms, 3),
        "bytes_per_ray": {"camera": round(float(bytes_p.mean()), 1),
                          "bounce": round(float(bytes_b.mean()), 1)},
        "bvh": {"nodes": st["n_nodes"], "node_bytes": st["node_bytes"],
                "nodes_mb": round(st["nodes_buffer_bytes"] / 1e6, 2),
                "leaf_mb": round(st["leaf_buffer_bytes"] / 1e6, 2), "depth": st["depth"]},
        # The traversal kernel issues VALU work most of the time (counter
        # VALUBusy) while its node and triangle data stay largely in the
        # caches (counter HBM bytes well below the algorithmic bytes), so the
        # bound reported is the VALU lane-operation peak; `achieved` counts the
        # algorithmic operations of the node and triangle tests per launch.
        "roofline": {"bound": "alu", "achieved": round(achieved_tops, 3), "peak": round(ALU_PEAK_TOPS, 2),
                     "unit": "Tops/s", "frac": round(achieved_tops / ALU_PEAK_TOPS, 4),
                     "traffic": traffic,
                     "kernel": f"trace ({args.layout}, {args.leaf_mode}), camera + bounce launches",
                     "ops_per_ray": {"camera": round(float(ops_p.mean()), 1),
                                     "bounce": round(float(ops_b.mean()), 1)},
                     "hbm": {"peak_gbs": HBM_PEAK_GBS,
                             "algorithmic_gbs": round(achieved_gbs, 1),
                             "algorithmic_frac": round(achieved_gbs / HBM_PEAK_GBS, 4),
                             "counter_gbs": (round(traffic / launch_s / 1e9, 1) if traffic else None),
                             "counter_frac": (round(traffic / launch_s / 1e9 / HBM_PEAK_GBS, 4)
                                              if traffic else None),
                             "note": "algorithmic bytes count every node and triangle fetch, "
                                     "most of which the caches serve; counter bytes are HBM "
                                     "reads and writes (rocprofv3 FETCH_SIZE, WRITE_SIZE)"}},
    }

    if not args.no_extras:
        sec = set(args.sections.split(","))
        if "per_layout" in sec:
            out["per_layout"] = per_layout(torch, bvh, verts, tris, prim_rays, bounce_rays, args)
        if "sah" in sec:
            out["sah"] = sah_rows(torch, bvh, verts, tris, prim_rays, bounce_rays, args)
        cpq = None
        if "closest_point" in sec:
            cpq = out["closest_point"] = {"terrain": closest_point_rows(
                torch, bvh, W, w["verts"], verts, w["tris"], tris, args, 1001)}
        if "fwd_bwd" in sec:
            out["fwd_bwd"] = fwd_bwd(torch, bvh, W)
        del verts, tris, prim_rays, bounce_rays, hits_p, hits_b
        if "spheres" in sec:
            out["spheres"] = spheres(torch, bvh, W, args, cpq)
        if "batched" in sec:
            out["batched"] = batched(torch, bvh, W)

    if args.copy_calib_mib > 0:
        n = args.copy_calib_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 2.0, out=b)  # one elementwise kernel: reads n*4 B, writes n*4 B
        torch.cuda.synchronize()
        out["copy_calib_bytes"] = {"read": n * 4, "write": n * 4}

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, W)

    print(json.dumps(out), flush=True)


def timed_events(torch, fn):
    """Event time (ms) of fn() on the current stream under the paper's
    protocol: one warm-up run, nine timed runs, trimmed mean of the middle
    five."""
    stream = torch.cuda.current_stream()
    times = []
    for _ in range(10):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        e[0].record(stream)
        fn()
        e[1].record(stream)
        torch.cuda.synchronize()
        times.append(e[0].elapsed_time(e[1]))
    return trimmed_mean(times[1:])


def time_trace(torch, h, rays, mode=0):
    hits = torch.empty((rays.shape[0], 4), dtype=torch.float32, device=rays.device)
    return timed_events(torch, lambda: h.trace(rays, mode=mode, hits=hits))


def layout_row(torch, h, layout, leaf_mode, ray_sets):
    """Per ray set: Mrays/s (trimmed mean of nine launches), algorithmic
    bytes per ray and their rate against the HBM peak, and algorithmic VALU
    operations per ray and their rate against the VALU peak."""
    st = h.stats()
    row = {"bvh_mb": round((st["nodes_buffer_bytes"] + st["leaf_buffer_bytes"]
                            + st["extra_bytes"]) / 1e6, 1)}
    for name, rays, mode in ray_sets:
        t_ms = time_trace(torch, h, rays, mode)
        _, c = h.trace_counts(rays, mode=mode)
        torch.cuda.synchronize()
        c = c.cpu().numpy()
        by = algorithmic_bytes(c, st["node_bytes"], leaf_mode)
        ops = algorithmic_ops(c, layout, leaf_mode)
        gbs = by.sum() / (t_ms / 1000.0) / 1e9
        tops = ops.sum() / (t_ms / 1000.0) / 1e12
        row[name] = {"mrays_s": round(rays.shape[0] / (t_ms / 1000.0) / 1e6, 1),
                     "ms": round(t_ms, 4), "nodes_per_ray": round(float(c[:, 0].mean()), 2),
                     "tris_per_ray": round(float(c[:, 1].mean()), 2),
                     "bytes_per_ray": round(float(by.mean()), 1),
                     "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "ops_per_ray": round(float(ops.mean()), 1), "alu_tops": round(tops, 3),
                     "alu_frac": round(tops / ALU_PEAK_TOPS, 4)}
    return row


def per_layout(torch, bvh, verts, tris, prim_rays, bounce_rays, args):
    """Terrain: trace-only Mrays/s, algorithmic bytes per ray and roofline
    fraction for every layout and leaf mode, camera (coherent) and bounce
    (incoherent) rays separately (median of 5 launches, events on the stream)."""
    res = {}
    for layout in args.layouts.split(","):
        for leaf_mode in ("compact", "indexed"):
            h = bvh.build(verts, tris, layout, args.leaf_size, leaf_mode)
            res[f"{layout}/{leaf_mode}"] = layout_row(
                torch, h, layout, leaf_mode, [("camera", prim_rays, bvh.TRACE_CLOSEST),
                                      ("bounce", bounce_rays, bvh.TRACE_CLOSEST)])
            h.close()
            log(f"terrain {layout}/{leaf_mode}: {res[f'{layout}/{leaf_mode}']}")
    return res


def time_closest(torch, h, q):
    out = torch.empty((q.shape[0], 4), dtype=torch.float32, device=q.device)
    return timed_events(torch, lambda: h.closest_point(q, out=out))


def closest_point_rows(torch, bvh, W, verts_np, verts, tris_np, tris, args, seed):
    """Closest-point queries: 2^20 points uniform in the scene's bounding box
    (unbounded radius), per layout with compacted leaves: Mqueries/s,
    node records and triangles per query (counting kernel), algorithmic
    bytes per query (query + result + nodes x node size + triangles x 48 B)
    and the fraction of the HBM peak; plus the CPU oracle on a sample."""
    import oracle
    lo, hi = verts_np.min(axis=0), verts_np.max(axis=0)
    q_np = W.box_points(1 << 20, lo, hi, seed)
    q = torch.from_numpy(q_np).to(verts.device)
    res = {"queries": int(q.shape[0])}
    for layout, builder in [(x, "lbvh") for x in LAYOUTS] + [("aabb2", "sah"), ("bvh4", "sah")]:
        key = layout if builder == "lbvh" else f"{layout}/sah"
        h = bvh.build(verts, tris, layout, args.leaf_size, "compact", builder=builder)
        st = h.stats()
        t_ms = time_closest(torch, h, q)
        _, c = h.closest_point_counts(q)
        torch.cuda.synchronize()
        c = c.cpu().numpy().astype(np.float64)
        by = QUERY_BYTES + CLOSEST_BYTES + c[:, 0] * st["node_bytes"] + c[:, 1] * LEAF_TRI_BYTES["compact"]
        gbs = by.sum() / (t_ms / 1000.0) / 1e9
        ops = c[:, 0] * ALU_OPS_CP_NODE[layout] + c[:, 1] * ALU_OPS_CP_TRI
        tops = ops.sum() / (t_ms / 1000.0) / 1e12
        res[key] = {"mqueries_s": round(q.shape[0] / (t_ms / 1000.0) / 1e6, 1),
                       "ms": round(t_ms, 4), "nodes_per_query": round(float(c[:, 0].mean()), 1),
                       "tris_per_query": round(float(c[:, 1].mean()), 1),
                       "bytes_per_query": round(float(by.mean()), 1),
                       "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                       "ops_per_query": round(float(ops.mean()), 1), "alu_tops": round(tops, 3),
                       "alu_frac": round(tops / ALU_PEAK_TOPS, 4)}
        h.close()
        log(f"closest point {key}: {res[key]}")
    if not args.no_cpu_baseline:
        b = oracle.OracleBVH(verts_np, tris_np)
        sample = q_np[: 1 << 17]
        t0 = time.perf_counter()
        b.closest_point(sample)
        secs = time.perf_counter() - t0
        res["cpu_oracle"] = {"mqueries_s": round(len(sample) / secs / 1e6, 3),
                             "cores": oracle.max_threads(),
                             "sample": f"first {len(sample)} queries, FP64 median-split BVH search "
                                       f"({secs:.2f} s wall)"}
    return res


def timed_build(torch, bvh, verts, tris, layout, leaf_size, builder, reps=3):
    """Median wall time (ms) of bvh_build, the stream drained before and after."""
    ms = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = bvh.build(verts, tris, layout, leaf_size, "compact", builder=builder)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1000.0)
        h.close()
    return float(np.median(ms))


def sah_rows(torch, bvh, verts, tris, prim_rays, bounce_rays, args):
    """Terrain: binned-SAH topology (32 bins) against LBVH per layout: build
    time (median of 3 builds, wall clock) and the trace rows (camera and
    bounce Mrays/s, algorithmic bytes per ray, roofline fraction)."""
    res = {}
    for layout in ("aabb2", "bvh4", "bvh8_q8", "pbrt_q16"):
        row = {}
        for builder in ("lbvh", "sah"):
            build_ms = timed_build(torch, bvh, verts, tris, layout, args.leaf_size, builder)
            h = bvh.build(verts, tris, layout, args.leaf_size, "compact", builder=builder)
            r = layout_row(torch, h, layout, "compact", [("camera", prim_rays, bvh.TRACE_CLOSEST),
                                                 ("bounce", bounce_rays, bvh.TRACE_CLOSEST)])
            r["build_ms"] = round(build_ms, 3)
            r["depth"] = h.stats()["depth"]
            h.close()
            row[builder] = r
        res[layout] = row
        log(f"terrain sah vs lbvh {layout}: {row}")
    return res


def spheres(torch, bvh, W, args, cpq=None):
    """Non-uniform density scene: 512 icospheres (levels 2-6 by radius rank)
    plus 100,000 slivers, 4,051,040 tris; 2^23 incoherent closest-hit rays
    and 2^23 any-hit shadow rays, per layout (compacted leaves).  With `cpq`
    (a dict), the closest-point rows of this scene are added to it."""
    t0 = time.time()
    w = W.spheres_workload()
    dev = torch.device("cuda:0")
    verts = torch.from_numpy(w["verts"]).to(dev)
    tris = torch.from_numpy(w["tris"]).to(dev)
    rays = torch.from_numpy(w["rays"]).to(dev)
    shadow = torch.from_numpy(w["shadow"]).to(dev)
    log(f"spheres workload: {w['tris'].shape[0]} tris ({time.time() - t0:.1f}s)")
    res = {"workload": f"{len(w['tris'])} tris (512 spheres + 100K slivers), {rays.shape[0]} "
                       "uniform closest-hit rays + as many shadow rays (any hit)"}
    for layout in args.layouts.split(","):
        h = bvh.build(verts, tris, layout, args.leaf_size, "compact")
        res[layout] = layout_row(torch, h, layout, "compact", [("closest", rays, bvh.TRACE_CLOSEST),
                                                       ("shadow_any", shadow, bvh.TRACE_ANY)])
        h.close()
        log(f"spheres {layout}: {res[layout]}")
    for layout in () if args.no_sah_rows else ("aabb2", "bvh4"):
        build_ms = timed_build(torch, bvh, verts, tris, layout, args.leaf_size, "sah")
        h = bvh.build(verts, tris, layout, args.leaf_size, "compact", builder="sah")
        r = layout_row(torch, h, layout, "compact", [("closest", rays, bvh.TRACE_CLOSEST),
                                                     ("shadow_any", shadow, bvh.TRACE_ANY)])
        r["build_ms"] = round(build_ms, 3)
        h.close()
        res[f"{layout}/sah"] = r
        log(f"spheres {layout}/sah: {r}")
    if cpq is not None:
        del rays, shadow
        cpq["spheres"] = closest_point_rows(torch, bvh, W, w["verts"], verts, w["tris"], tris,
                                            args, 1002)
    return res


def fwd_bwd(torch, bvh, W):
    """Differentiable workload: icosphere level 7 (327,680 tris), 1,048,576
    rays; forward-only vs forward + backward throughput (BVH prebuilt)."""
    w = W.diff_workload()
    dev = torch.device("cuda:0")
    v = torch.from_numpy(w["verts"]).to(dev)
    t = torch.from_numpy(w["tris"]).to(dev)
    r = torch.from_numpy(w["rays"]).to(dev)
    g = torch.from_numpy(w["weights"]).to(dev)
    h = bvh.build(v, t, "bvh8_q8")
    hits = torch.empty((r.shape[0], 4), dtype=torch.float32, device=dev)
    gv = torch.zeros_like(v)
    gr = torch.empty((r.shape[0], 6), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    def run(bwd):
        """(forward [+ backward] ms, backward alone ms); grad_verts is zeroed
        between the two events, outside the backward's own interval."""
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(stream)
        h.trace(r, hits=hits)
        if bwd:
            gv.zero_()
        e[1].record(stream)
        if bwd:
            bvh.lib().bvh_trace_backward(v.data_ptr(), v.shape[0], t.data_ptr(), t.shape[0],
                                         r.data_ptr(), r.shape[0], hits.data_ptr(), g.data_ptr(),
                                         gv.data_ptr(), gr.data_ptr(), stream.cuda_stream)
        e[2].record(stream)
        torch.cuda.synchronize()
        return e[0].elapsed_time(e[2]), e[1].elapsed_time(e[2])

    for _ in range(2):
        run(False), run(True)
    f = trimmed_mean([run(False)[0] for _ in range(9)])
    both = [run(True) for _ in range(9)]
    fb = trimmed_mean([x[0] for x in both])
    b = trimmed_mean([x[1] for x in both])
    h.close()
    n = r.shape[0]
    gbs = BWD_BYTES_PER_RAY * n / (b / 1000) / 1e9
    return {"workload": "icosphere level 7 (327,680 tris), 1,048,576 rays from 64 cameras",
            "fwd_mrays_s": round(n / (f / 1000) / 1e6, 1),
            "fwd_bwd_mrays_s": round(n / (fb / 1000) / 1e6, 1),
            "fwd_ms": round(f, 4), "fwd_bwd_ms": round(fb, 4), "bwd_us": round(b * 1000, 1),
            "bwd_roofline": {"bound": "hbm", "bytes_per_ray": BWD_BYTES_PER_RAY,
                             "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": round(gbs / HBM_PEAK_GBS, 4)}}


def batched(torch, bvh, W):
    """256 scenes of uneven size (1 K-500 K triangles, 1 K-1 M rays each):
    one graph launch of the per-variant persistent kernels vs 256 plain
    bvh_trace launches on one stream (same tuned BVHs), and vs plain launches
    with one fixed layout (the tuner's own gain).  The tuner probes with rays
    generated on the device, not with the timed rays.  BVH builds and tuning
    are excluded."""
    t0 = time.time()
    w = W.batch_workload()
    log(f"batch workload: {len(w['scenes'])} scenes, {int(w['n_tris'].sum())} tris, "
        f"{w['rays'].shape[0]} rays ({time.time() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    scenes = [(torch.from_numpy(v).to(dev), torch.from_numpy(t).to(dev)) for v, t in w["scenes"]]
    rays = torch.from_numpy(w["rays"]).to(dev)
    off = w["offsets"]
    n = rays.shape[0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # tuned on probe rays the library generates on the device (uniform in each
    # scene's box), not on the rays timed below
    b = bvh.Batch(scenes)
    create_s = time.perf_counter() - t0
    infos = [b.info(i) for i in range(len(scenes))]
    handles = [b.handle(i) for i in range(len(scenes))]

    def timed(fn):
        return timed_events(torch, fn)

    hits_b = torch.empty((n, 4), dtype=torch.float32, device=dev)
    hits_p = torch.empty((n, 4), dtype=torch.float32, device=dev)
    t_batch = timed(lambda: b.trace(rays, off, hits=hits_b))

    def plain(hs, out):
        for i, h in enumerate(hs):
            if off[i + 1] > off[i]:
                h.trace(rays[off[i]:off[i + 1]], hits=out[off[i]:off[i + 1]])

    t_plain = timed(lambda: plain(handles, hits_p))
    same = bool(torch.equal(hits_b.view(torch.int32), hits_p.view(torch.int32)))
    fixed = [bvh.build(v, t, "bvh8_q8") for v, t in scenes]
    t_fixed = timed(lambda: plain(fixed, hits_p))
    for h in fixed:
        h.close()
    layouts = {}
    for inf in infos:
        k = f"{bvh.LAYOUT_NAMES[inf['layout']]}/lds{inf['stack_lds']}"
        layouts[k] = layouts.get(k, 0) + 1
    b.close()
    return {"workload": f"{len(scenes)} scenes, {int(w['n_tris'].sum())} tris, {n} rays "
                        "(log-uniform 1K-500K tris, 1K-1M incoherent rays per scene)",
            "batched_mrays_s": round(n / (t_batch / 1000) / 1e6, 1),
            "plain_tuned_mrays_s": round(n / (t_plain / 1000) / 1e6, 1),
            "plain_bvh8_q8_mrays_s": round(n / (t_fixed / 1000) / 1e6, 1),
            "speedup_vs_plain_tuned": round(t_plain / t_batch, 3),
            "speedup_vs_plain_fixed": round(t_fixed / t_batch, 3),
            "tuner_gain_plain": round(t_fixed / t_plain, 3),
            "batched_ms": round(t_batch, 3), "plain_tuned_ms": round(t_plain, 3),
            "plain_fixed_ms": round(t_fixed, 3), "hits_equal_plain": same,
            "create_and_tune_s": round(create_s, 2), "chosen": layouts}


def cpu_baseline(w, W):
    """The CPU oracle (median-split BVH, scalar stack traversal, OpenMP
    dynamic,64 over rays) on the same terrain: all camera rays, then the
    bounce rays made from the oracle's own hits.  Build time excluded."""
    import oracle
    b = oracle.OracleBVH(w["verts"], w["tris"])
    cores = oracle.max_threads()
    rays = w["rays"]
    t0 = time.perf_counter()
    p, tuv = b.trace(rays, nthreads=cores)
    t1 = time.perf_counter()
    bounce, _ = W.bounce_rays(rays, p, tuv[:, 0], w["verts"], w["tris"], seed=1001)
    t2 = time.perf_counter()
    b.trace(bounce, nthreads=cores)
    t3 = time.perf_counter()
    secs = (t1 - t0) + (t3 - t2)
    n = rays.shape[0] + bounce.shape[0]
    # one thread on a bounded sample: the first 2^18 camera and 2^18 bounce rays
    k = 1 << 18
    t4 = time.perf_counter()
    b.trace(rays[:k], nthreads=1)
    b.trace(bounce[:k], nthreads=1)
    secs1 = time.perf_counter() - t4
    return {"value": round(n / secs / 1e6, 3), "unit": "Mrays/s", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"all {rays.shape[0]} camera rays + {bounce.shape[0]} bounce rays of the "
                      f"terrain workload, traversal only ({secs:.2f} s wall on {cores} threads, "
                      "OpenMP dynamic,64 over rays; one run)",
            "one_thread": {"value": round(2 * k / secs1 / 1e6, 3), "unit": "Mrays/s",
                           "sample": f"first {k} camera + first {k} bounce rays ({secs1:.2f} s)"}}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
