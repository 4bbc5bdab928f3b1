"""Seeded synthetic scenes and rays.

This module is shared by the GPU path's tests and benchmark and by the CPU
oracle's tests.  It holds scene and ray *generation* only (meshes, cameras,
noise, sampling); none of the traversal, intersection or gradient arithmetic
of the method lives here.

Conventions
-----------
* Meshes are indexed: ``verts`` float32 [V,3], ``tris`` int32 [N,3].
* Rays are float32 [n,8]: ``o.xyz, tmin, d.xyz, tmax`` with tmin = 0 and
  tmax = +inf unless stated.  Directions are unit length.
* Every generator takes a seed and draws from ``numpy.random.default_rng``
  (PCG64), so the same seed gives the same arrays on every machine.

The paper's own scenes (scanned and architectural meshes of 36 K to 28 M
triangles) are not available; these procedural scenes stand in for them at
the same scale and with the same two ray classes, coherent camera rays and
incoherent secondary rays (Sec. 9.2.1).
"""
from __future__ import annotations

import math

import numpy as np

INF = np.float32(np.inf)


def _rng(seed, tag=0):
    return np.random.default_rng([int(seed), int(tag)])


def _normalize(v):
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def make_rays(o, d, tmax=None):
    """Packs origins/directions (float64 or float32) into the [n,8] record."""
    n = o.shape[0]
    r = np.zeros((n, 8), np.float32)
    r[:, 0:3] = o
    r[:, 4:7] = d
    r[:, 7] = np.inf if tmax is None else tmax
    return r


# ---------------------------------------------------------------------------
# Value noise and fBm
# ---------------------------------------------------------------------------
def _smooth(f):
    return f * f * (3.0 - 2.0 * f)


def value_noise_2d(table, x, y):
    """Smoothstep-interpolated lattice noise over a wrapped square table."""
    m = table.shape[0]
    xi = np.floor(x)
    yi = np.floor(y)
    fx = _smooth(x - xi)
    fy = _smooth(y - yi)
    xi = xi.astype(np.int64) % m
    yi = yi.astype(np.int64) % m
    x1 = (xi + 1) % m
    y1 = (yi + 1) % m
    a = table[xi, yi]
    b = table[x1, yi]
    c = table[xi, y1]
    d = table[x1, y1]
    return (a * (1 - fx) + b * fx) * (1 - fy) + (c * (1 - fx) + d * fx) * fy


def value_noise_3d(table, p):
    m = table.shape[0]
    pi = np.floor(p)
    f = _smooth(p - pi)
    i = pi.astype(np.int64) % m
    j = (i + 1) % m
    out = 0.0
    for cx in (0, 1):
        wx = f[:, 0] if cx else 1 - f[:, 0]
        ix = j[:, 0] if cx else i[:, 0]
        for cy in (0, 1):
            wy = f[:, 1] if cy else 1 - f[:, 1]
            iy = j[:, 1] if cy else i[:, 1]
            for cz in (0, 1):
                wz = f[:, 2] if cz else 1 - f[:, 2]
                iz = j[:, 2] if cz else i[:, 2]
                out = out + wx * wy * wz * table[ix, iy, iz]
    return out


def fbm_2d(table, x, y, octaves, base=4.0, lacunarity=2.0, gain=0.5):
    """fBm normalised by the weight sum, so values stay in [0, 1)."""
    total = 0.0
    wsum = 0.0
    f = base
    w = 1.0
    for _ in range(octaves):
        total = total + w * value_noise_2d(table, x * f, y * f)
        wsum += w
        f *= lacunarity
        w *= gain
    return total / wsum


def fbm_3d(table, p, octaves, base=4.0, lacunarity=2.0, gain=0.5):
    total = 0.0
    wsum = 0.0
    f = base
    w = 1.0
    for _ in range(octaves):
        total = total + w * value_noise_3d(table, p * f)
        wsum += w
        f *= lacunarity
        w *= gain
    return total / wsum


# ---------------------------------------------------------------------------
# Cameras
# ---------------------------------------------------------------------------
def pinhole_rays(eye, target, up, width, height, hfov_deg):
    """Pixel-centre rays of a pinhole camera; row 0 is the top of the image.

    The horizontal field of view is ``hfov_deg``; the vertical one follows
    from the aspect ratio.  Rays are ordered row-major."""
    eye = np.asarray(eye, np.float64)
    f = _normalize(np.asarray(target, np.float64) - eye)
    r = _normalize(np.cross(f, np.asarray(up, np.float64)))
    u = np.cross(r, f)
    s = math.tan(math.radians(hfov_deg) / 2.0)
    i = (np.arange(width) + 0.5) / width * 2.0 - 1.0
    j = 1.0 - (np.arange(height) + 0.5) / height * 2.0
    sx = np.tile(i * s, height)
    sy = np.repeat(j * s * height / width, width)
    d = _normalize(f[None, :] + sx[:, None] * r[None, :] + sy[:, None] * u[None, :])
    o = np.broadcast_to(eye, d.shape)
    return make_rays(o, d)


def soup_camera_rays(width=64, height=64):
    """Camera at (0.5,0.5,-1) looking +z, up +y, 60 degree field of view."""
    return pinhole_rays((0.5, 0.5, -1.0), (0.5, 0.5, 0.0), (0.0, 1.0, 0.0), width, height, 60.0)


def terrain_camera_rays(width=1920, height=1080):
    """Camera at (0.5,0.5,1.2) looking down at (0.5,0.5,0), up +y, 45 degree
    horizontal field of view.  Every ray meets the unit-square terrain."""
    return pinhole_rays((0.5, 0.5, 1.2), (0.5, 0.5, 0.0), (0.0, 1.0, 0.0), width, height, 45.0)


# ---------------------------------------------------------------------------
# Scenes
# ---------------------------------------------------------------------------
def soup_scene(n_tris=1024, seed=1000, spread=0.05):
    """Triangle soup: centroids U[0,1]^3, each vertex = centroid + U[-s,s]^3.
    Vertices are not shared: tris[i] = (3i, 3i+1, 3i+2)."""
    rng = _rng(seed, 0)
    c = rng.uniform(0.0, 1.0, (n_tris, 3))
    off = rng.uniform(-spread, spread, (n_tris, 3, 3))
    verts = (c[:, None, :] + off).reshape(-1, 3).astype(np.float32)
    tris = np.arange(3 * n_tris, dtype=np.int32).reshape(n_tris, 3)
    return verts, tris


def terrain_scene(cells=1024, seed=1001, amplitude=0.2, octaves=6):
    """Heightfield over the unit square: (cells+1)^2 vertices, 2*cells^2
    triangles, each cell split along its (0,0)-(1,1) diagonal; height =
    amplitude * fBm(x, y) from a wrapped 256^2 value-noise table."""
    rng = _rng(seed, 0)
    table = rng.uniform(0.0, 1.0, (256, 256))
    g = np.arange(cells + 1, dtype=np.float64) / cells
    x = np.tile(g, cells + 1)          # vertex index = j*(cells+1) + i
    y = np.repeat(g, cells + 1)
    z = amplitude * fbm_2d(table, x, y, octaves)
    verts = np.stack([x, y, z], axis=1).astype(np.float32)
    i = np.tile(np.arange(cells), cells)
    j = np.repeat(np.arange(cells), cells)
    a = j * (cells + 1) + i
    b = a + 1
    c = a + (cells + 1)
    d = c + 1
    t0 = np.stack([a, b, d], axis=1)
    t1 = np.stack([a, d, c], axis=1)
    tris = np.stack([t0, t1], axis=1).reshape(-1, 3).astype(np.int32)
    return verts, tris


def _icosahedron():
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            v.append((s1, s2 * p, 0.0))
            v.append((0.0, s1, s2 * p))
            v.append((s2 * p, 0.0, s1))
    v = np.array(v, np.float64)
    # faces: the 20 vertex triples that are mutually one edge (length 2) apart
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=-1)
    adj = np.abs(d - 2.0) < 1e-9
    faces = []
    for a in range(12):
        for b in range(a + 1, 12):
            if not adj[a, b]:
                continue
            for c in range(b + 1, 12):
                if adj[a, c] and adj[b, c]:
                    n = np.cross(v[b] - v[a], v[c] - v[a])
                    faces.append((a, b, c) if n @ (v[a] + v[b] + v[c]) > 0 else (a, c, b))
    faces = np.array(faces, np.int64)
    assert faces.shape == (20, 3)
    return _normalize(v), faces


_ICO_CACHE: dict = {}


def icosphere(level):
    """Unit icosphere: 20*4^level faces, 10*4^level + 2 vertices (float64)."""
    if level in _ICO_CACHE:
        return _ICO_CACHE[level]
    v, f = _icosahedron()
    for _ in range(level):
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]], axis=0)
        e = np.sort(e, axis=1)
        uniq, inv = np.unique(e, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        mids = _normalize(v[uniq[:, 0]] + v[uniq[:, 1]])
        nf = f.shape[0]
        ab = inv[0:nf] + v.shape[0]
        bc = inv[nf:2 * nf] + v.shape[0]
        ca = inv[2 * nf:3 * nf] + v.shape[0]
        a, b, c = f[:, 0], f[:, 1], f[:, 2]
        f = np.stack([np.stack([a, ab, ca], 1), np.stack([b, bc, ab], 1),
                      np.stack([c, ca, bc], 1), np.stack([ab, bc, ca], 1)], 1).reshape(-1, 3)
        v = np.concatenate([v, mids], axis=0)
    _ICO_CACHE[level] = (v, f)
    return v, f


# Subdivision levels assigned by radius rank (smallest first) for 512 spheres.
SPHERE_LEVEL_QUOTA = ((2, 179), (3, 154), (4, 102), (5, 51), (6, 26))


def _sphere_levels(radii, quota):
    order = np.argsort(radii, kind="stable")
    levels = np.empty(len(radii), np.int64)
    k = 0
    for lvl, cnt in quota:
        levels[order[k:k + cnt]] = lvl
        k += cnt
    assert k == len(radii)
    return levels


def _slivers(rng, n):
    """Long thin triangles: long edge l ~ logU[0.01,0.2] along a random unit
    a, apex at height l/200 along a random unit b orthogonal to a."""
    c = rng.uniform(0.0, 1.0, (n, 3))
    ell = np.exp(rng.uniform(math.log(0.01), math.log(0.2), n))
    a = _normalize(rng.normal(size=(n, 3)))
    w = rng.normal(size=(n, 3))
    b = _normalize(w - np.sum(w * a, axis=1, keepdims=True) * a)
    p0 = c - 0.5 * ell[:, None] * a
    p1 = c + 0.5 * ell[:, None] * a
    p2 = c + (ell / 200.0)[:, None] * b
    return np.stack([p0, p1, p2], axis=1).reshape(-1, 3)


def sphere_cluster_scene(n_spheres=512, n_slivers=100_000, seed=1002, quota=SPHERE_LEVEL_QUOTA):
    """Icospheres with centres U[0,1]^3 and radii log-uniform in [0.005,0.2],
    subdivision level by radius rank, plus long thin slivers."""
    rng = _rng(seed, 0)
    centers = rng.uniform(0.0, 1.0, (n_spheres, 3))
    radii = np.exp(rng.uniform(math.log(0.005), math.log(0.2), n_spheres))
    levels = _sphere_levels(radii, quota)
    vs, fs = [], []
    base = 0
    for s in range(n_spheres):
        v, f = icosphere(int(levels[s]))
        vs.append(centers[s] + radii[s] * v)
        fs.append(f + base)
        base += v.shape[0]
    sl = _slivers(rng, n_slivers)
    vs.append(sl)
    fs.append(base + np.arange(sl.shape[0], dtype=np.int64).reshape(-1, 3))
    verts = np.concatenate(vs, axis=0).astype(np.float32)
    tris = np.concatenate(fs, axis=0).astype(np.int32)
    return verts, tris


def uniform_rays(n, seed, tag=1):
    """Origins U[0,1]^3, directions uniform on the sphere, tmax = +inf."""
    rng = _rng(seed, tag)
    o = rng.uniform(0.0, 1.0, (n, 3))
    z = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    d = np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)
    return make_rays(o, d)


def box_points(n, lo, hi, seed, tag=5, r2=math.inf):
    """Closest-point queries: points uniform in the box [lo, hi] (queries
    sampled inside the scene's bounding volume, Sec. 9.3.2), packed as [n,4]
    float32 records (x, y, z, r2) with squared search radius r2."""
    rng = _rng(seed, tag)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    p = lo + (hi - lo) * rng.uniform(0.0, 1.0, (n, 3))
    out = np.empty((n, 4), np.float32)
    out[:, :3] = p
    out[:, 3] = np.float32(r2)
    return out


def shadow_rays(n, seed, tag=1):
    """Same origins as uniform_rays(n, seed, tag); each aims at a target
    U[0,1]^3 with tmax = distance to the target (occlusion queries)."""
    rng = _rng(seed, tag)
    o = rng.uniform(0.0, 1.0, (n, 3))
    rng2 = _rng(seed, tag + 100)
    tgt = rng2.uniform(0.0, 1.0, (n, 3))
    v = tgt - o
    dist = np.linalg.norm(v, axis=1)
    dist = np.where(dist > 0.0, dist, 1.0)
    return make_rays(o, v / dist[:, None], tmax=dist.astype(np.float32))


def _onb(n):
    """Orthonormal tangent frame about unit normals n (branchless form of
    Duff et al. 2017)."""
    sign = np.where(n[:, 2] >= 0.0, 1.0, -1.0)
    a = -1.0 / (sign + n[:, 2])
    b = n[:, 0] * n[:, 1] * a
    t = np.stack([1.0 + sign * n[:, 0] * n[:, 0] * a, sign * b, -sign * n[:, 0]], axis=1)
    bt = np.stack([b, sign + n[:, 1] * n[:, 1] * a, -n[:, 1]], axis=1)
    return t, bt


def bounce_rays(rays, prim, t, verts, tris, seed, eps=1e-4):
    """One cosine-weighted diffuse bounce per hit (prim >= 0).

    The origin is the hit point o + t d moved eps along the geometric normal
    turned toward the incoming side; the direction is drawn by Malley's method
    (uniform disk lifted to the hemisphere).  Returns (bounce_rays[m,8],
    source_index[m])."""
    prim = np.asarray(prim)
    idx = np.nonzero(prim >= 0)[0]
    r = np.asarray(rays, np.float64)[idx]
    o = r[:, 0:3]
    d = r[:, 4:7]
    p = o + np.asarray(t, np.float64)[idx, None] * d
    tri = np.asarray(tris)[prim[idx]]
    v = np.asarray(verts, np.float64)
    ng = _normalize(np.cross(v[tri[:, 1]] - v[tri[:, 0]], v[tri[:, 2]] - v[tri[:, 0]]))
    flip = np.sum(ng * d, axis=1) > 0.0
    ng[flip] = -ng[flip]
    rng = _rng(seed, 7)
    u1 = rng.uniform(0.0, 1.0, idx.shape[0])
    u2 = rng.uniform(0.0, 1.0, idx.shape[0])
    rad = np.sqrt(u1)
    phi = 2.0 * math.pi * u2
    x = rad * np.cos(phi)
    y = rad * np.sin(phi)
    z = np.sqrt(np.maximum(0.0, 1.0 - u1))
    tt, bb = _onb(ng)
    nd = _normalize(x[:, None] * tt + y[:, None] * bb + z[:, None] * ng)
    return make_rays(p + eps * ng, nd), idx


def perturbed_icosphere(level=7, seed=1004, amplitude=0.05, octaves=3):
    """Unit icosphere with each vertex v scaled by 1 + amp*(2*fBm(2v+2) - 1),
    fBm over a wrapped 64^3 value-noise table."""
    rng = _rng(seed, 0)
    table = rng.uniform(0.0, 1.0, (64, 64, 64))
    v, f = icosphere(level)
    s = 1.0 + amplitude * (2.0 * fbm_3d(table, 2.0 * v + 2.0, octaves) - 1.0)
    return (v * s[:, None]).astype(np.float32), f.astype(np.int32)


def sphere_cameras_rays(n_cams=64, res=128, radius=3.0, fov_deg=25.0):
    """Cameras on a Fibonacci sphere of the given radius, each looking at the
    origin with a square image of res^2 pixels."""
    out = []
    golden = math.pi * (3.0 - math.sqrt(5.0))
    for k in range(n_cams):
        z = 1.0 - (2.0 * k + 1.0) / n_cams
        r = math.sqrt(max(0.0, 1.0 - z * z))
        eye = radius * np.array([r * math.cos(k * golden), r * math.sin(k * golden), z])
        fwd = -eye / np.linalg.norm(eye)
        up = (0.0, 1.0, 0.0) if abs(fwd[1]) < 0.9 else (1.0, 0.0, 0.0)
        out.append(pinhole_rays(eye, (0.0, 0.0, 0.0), up, res, res, fov_deg))
    return np.concatenate(out, axis=0)


# ---------------------------------------------------------------------------
# The five workloads (full sizes) and their scaled-down test variants
# ---------------------------------------------------------------------------
def soup_workload(seed=1000, n_tris=1024, res=64):
    verts, tris = soup_scene(n_tris, seed)
    return dict(name=f"soup-{n_tris}", verts=verts, tris=tris, rays=soup_camera_rays(res, res))


def terrain_workload(seed=1001, cells=1024, width=1920, height=1080):
    verts, tris = terrain_scene(cells, seed)
    return dict(name=f"terrain-{cells}", verts=verts, tris=tris,
                rays=terrain_camera_rays(width, height))


def spheres_workload(seed=1002, n_rays=1 << 23, n_spheres=512, n_slivers=100_000,
                     quota=SPHERE_LEVEL_QUOTA):
    verts, tris = sphere_cluster_scene(n_spheres, n_slivers, seed, quota)
    return dict(name=f"spheres-{tris.shape[0]}", verts=verts, tris=tris,
                rays=uniform_rays(n_rays, seed), shadow=shadow_rays(n_rays, seed))


def diff_workload(seed=1004, level=7, n_cams=64, res=128):
    verts, tris = perturbed_icosphere(level, seed)
    rays = sphere_cameras_rays(n_cams, res)
    w = _rng(seed, 9).uniform(-1.0, 1.0, (rays.shape[0], 3)).astype(np.float32)
    return dict(name=f"ico{level}", verts=verts, tris=tris, rays=rays, weights=w)


def sphere_cluster_exact(n_tris, seed, quota=SPHERE_LEVEL_QUOTA, tris_per_sphere=7717):
    """A sphere cluster of exactly n_tris triangles: ceil(n_tris / 7717)
    icospheres (7717 = the mean triangles per sphere of the 512-sphere scene),
    levels by radius rank with the same proportions as that scene's quota,
    the largest spheres' levels lowered until the count fits, slivers for the
    remainder."""
    rng = _rng(seed, 0)
    k = max(1, int(math.ceil(n_tris / tris_per_sphere)))
    centers = rng.uniform(0.0, 1.0, (k, 3))
    radii = np.exp(rng.uniform(math.log(0.005), math.log(0.2), k))
    total_q = sum(c for _, c in quota)
    bounds = np.cumsum([c for _, c in quota])
    order = np.argsort(radii, kind="stable")
    levels = np.empty(k, np.int64)
    for r, s in enumerate(order):
        pos = (r + 0.5) / k * total_q
        levels[s] = quota[int(np.searchsorted(bounds, pos))][0]
    count = lambda: int(sum(20 * 4 ** int(l) for l in levels))
    for s in order[::-1]:                 # largest first
        while count() > n_tris and levels[s] > 0:
            levels[s] -= 1
    vs, fs, base = [], [], 0
    if count() <= n_tris:
        for s in range(k):
            v, f = icosphere(int(levels[s]))
            vs.append(centers[s] + radii[s] * v)
            fs.append(f + base)
            base += v.shape[0]
        n_sl = n_tris - count()
    else:                                 # fewer than 20 triangles: slivers only
        n_sl = n_tris
    if n_sl > 0:
        sl = _slivers(rng, n_sl)
        vs.append(sl)
        fs.append(base + np.arange(sl.shape[0], dtype=np.int64).reshape(-1, 3))
    verts = np.concatenate(vs, axis=0).astype(np.float32)
    tris = np.concatenate(fs, axis=0).astype(np.int32)
    assert tris.shape[0] == n_tris
    return verts, tris


def batch_workload(seed=1003, n_scenes=256, tri_range=(1e3, 5e5), ray_range=(1e3, 1e6)):
    """Scenes of uneven size for batched tracing: triangle counts log-uniform
    in tri_range (even scenes: soups as in the soup workload; odd scenes:
    sphere clusters with slivers), each with a log-uniform number of
    incoherent rays (origins U[0,1]^3, uniform directions).  Returns a dict
    with per-scene (verts, tris), the concatenated rays and the ray offsets."""
    rng = _rng(seed, 0)
    lt = np.log(np.asarray(tri_range, np.float64))
    lr = np.log(np.asarray(ray_range, np.float64))
    n_tris = np.round(np.exp(rng.uniform(lt[0], lt[1], n_scenes))).astype(np.int64)
    n_rays = np.round(np.exp(rng.uniform(lr[0], lr[1], n_scenes))).astype(np.int64)
    scenes, rays = [], []
    for i in range(n_scenes):
        s = seed * 1000 + i
        if i % 2 == 0:
            scenes.append(soup_scene(int(n_tris[i]), seed=s))
        else:
            scenes.append(sphere_cluster_exact(int(n_tris[i]), seed=s))
        rays.append(uniform_rays(int(n_rays[i]), seed=s, tag=2))
    offsets = np.zeros(n_scenes + 1, np.int64)
    offsets[1:] = np.cumsum(n_rays)
    return dict(name=f"batch-{n_scenes}", scenes=scenes, rays=np.concatenate(rays),
                offsets=offsets, n_tris=n_tris, n_rays=n_rays)
