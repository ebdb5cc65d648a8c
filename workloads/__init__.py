"""Seeded synthetic scenes and rays for the hierarchy-cut-code ray-reordering path.

This module is shared by the tests, the benchmark and the smoke check.  It only
*generates* inputs: triangles, camera rays, and the diffuse/shadow rays a path
tracer spawns at hit points (Section 5 of the paper: a wavefront path tracer with
next-event estimation).  It contains none of the method's arithmetic -- no BVH,
no cut, no key, no sort, no traversal.  Hits needed to spawn secondary rays are
passed in by the caller (from the oracle in tests, from the GPU trace in the
benchmark).

Randomness is counter based (SplitMix64 finaliser keyed by seed, stream and
index), so any subset of a workload can be regenerated independently.

Ray layout (shared with the C ABI): float32 rows of 8 values
``[ox, oy, oz, tmin, dx, dy, dz, tmax]`` (32 bytes per ray).
Triangle layout: float32 rows of 9 values ``[v0xyz, v1xyz, v2xyz]``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "u64_hash", "uniform01", "room_box", "tiny_scene", "frame_scene", "cluster_scene",
    "icosphere", "torus", "pinhole_rays", "spawn_diffuse", "spawn_shadow", "scene_extent",
    "SceneSpec", "TINY", "FRAME", "DRIFT", "BATCH_SCENES",
]

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def _mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser (Steele, Lea, Flood 2014), vectorised, wrapping."""
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def u64_hash(seed: int, stream: int, idx) -> np.ndarray:
    """Counter-based 64-bit random value for (seed, stream, index)."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        key = _mix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * np.uint64(0x9E3779B97F4A7C15)
                     + np.uint64(stream & 0xFFFFFFFFFFFFFFFF) * np.uint64(0xD1B54A32D192ED03))
        return _mix64(key + (idx + np.uint64(1)) * np.uint64(0x9E3779B97F4A7C15))


def uniform01(seed: int, stream: int, idx) -> np.ndarray:
    """Uniform float64 in [0, 1) with 53 random bits."""
    return (u64_hash(seed, stream, idx) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# --------------------------------------------------------------------------- geometry

def room_box(lo, hi) -> np.ndarray:
    """Closed axis-aligned box as 12 triangles (two per face)."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    c = np.array([[lo[0] if (i >> 0) & 1 == 0 else hi[0],
                   lo[1] if (i >> 1) & 1 == 0 else hi[1],
                   lo[2] if (i >> 2) & 1 == 0 else hi[2]] for i in range(8)])
    quads = [(0, 2, 6, 4), (1, 5, 7, 3),   # x = lo, x = hi
             (0, 4, 5, 1), (2, 3, 7, 6),   # y = lo, y = hi
             (0, 1, 3, 2), (4, 6, 7, 5)]   # z = lo, z = hi
    tris = []
    for a, b, cc, d in quads:
        tris.append(np.concatenate([c[a], c[b], c[cc]]))
        tris.append(np.concatenate([c[a], c[cc], c[d]]))
    return np.asarray(tris, np.float32)


def _unit_sphere_dirs(u1: np.ndarray, u2: np.ndarray) -> np.ndarray:
    z = 1.0 - 2.0 * u1
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = 2.0 * math.pi * u2
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=-1)


def icosphere(subdiv: int) -> np.ndarray:
    """Unit icosphere, ``20 * 4**subdiv`` triangles, float64 (T, 3, 3)."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    verts = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t),
             (0, -1, -t), (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    faces = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
             (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
             (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    v = np.asarray(verts, np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    tri = v[np.asarray(faces)]                       # (20, 3, 3)
    for _ in range(subdiv):
        a, b, c = tri[:, 0], tri[:, 1], tri[:, 2]
        ab = a + b; ab /= np.linalg.norm(ab, axis=1, keepdims=True)
        bc = b + c; bc /= np.linalg.norm(bc, axis=1, keepdims=True)
        ca = c + a; ca /= np.linalg.norm(ca, axis=1, keepdims=True)
        tri = np.concatenate([np.stack([a, ab, ca], 1), np.stack([ab, b, bc], 1),
                              np.stack([ca, bc, c], 1), np.stack([ab, bc, ca], 1)], 0)
    return tri


def torus(nu: int, nv: int, major: float, minor: float) -> np.ndarray:
    """Torus around the z axis, ``2 * nu * nv`` triangles, float64 (T, 3, 3)."""
    i = np.arange(nu)
    j = np.arange(nv)
    u = 2 * math.pi * i / nu
    v = 2 * math.pi * j / nv
    U, V = np.meshgrid(u, v, indexing="ij")
    P = np.stack([(major + minor * np.cos(V)) * np.cos(U),
                  (major + minor * np.cos(V)) * np.sin(U),
                  minor * np.sin(V)], -1)             # (nu, nv, 3)
    p00 = P
    p10 = np.roll(P, -1, axis=0)
    p01 = np.roll(P, -1, axis=1)
    p11 = np.roll(np.roll(P, -1, axis=0), -1, axis=1)
    t1 = np.stack([p00, p10, p11], 2).reshape(-1, 3, 3)
    t2 = np.stack([p00, p11, p01], 2).reshape(-1, 3, 3)
    return np.concatenate([t1, t2], 0)


def _rotations(seed: int, stream: int, n: int) -> np.ndarray:
    """n uniformly random rotation matrices (random unit quaternions, Shoemake 1992)."""
    idx = np.arange(n, dtype=np.uint64) * np.uint64(3)
    u1 = uniform01(seed, stream, idx)
    u2 = uniform01(seed, stream, idx + np.uint64(1))
    u3 = uniform01(seed, stream, idx + np.uint64(2))
    a = np.sqrt(1 - u1); b = np.sqrt(u1)
    w = a * np.sin(2 * math.pi * u2); x = a * np.cos(2 * math.pi * u2)
    y = b * np.sin(2 * math.pi * u3); z = b * np.cos(2 * math.pi * u3)
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z); R[:, 0, 1] = 2 * (x * y - z * w); R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w); R[:, 1, 1] = 1 - 2 * (x * x + z * z); R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w); R[:, 2, 1] = 2 * (y * z + x * w); R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def scene_extent(tris: np.ndarray) -> float:
    """Largest extent of the bounding box of all vertices."""
    v = np.asarray(tris, np.float32).reshape(-1, 3)
    return float((v.max(0).astype(np.float64) - v.min(0).astype(np.float64)).max())


# --------------------------------------------------------------------------- scenes

@dataclass
class SceneSpec:
    """Scene plus the camera / light constants that go with it."""
    name: str
    tris: np.ndarray                      # (N, 9) float32
    cam_pos: tuple
    cam_dir: tuple
    cam_up: tuple
    vfov_deg: float
    lights: list = field(default_factory=list)


def tiny_scene(seed: int = 1, n_random: int = 2000) -> SceneSpec:
    """Closed room [-0.05, 1.05]^3 (12 tris) + ``n_random`` random triangles.

    v0 ~ U[0,1]^3; v1, v2 = v0 + l*w with l ~ U[0.01, 0.05] and w uniform on the sphere.
    """
    idx = np.arange(n_random, dtype=np.uint64)
    v0 = np.stack([uniform01(seed, s, idx) for s in (0, 1, 2)], -1)
    l1 = 0.01 + 0.04 * uniform01(seed, 3, idx)
    l2 = 0.01 + 0.04 * uniform01(seed, 4, idx)
    w1 = _unit_sphere_dirs(uniform01(seed, 5, idx), uniform01(seed, 6, idx))
    w2 = _unit_sphere_dirs(uniform01(seed, 7, idx), uniform01(seed, 8, idx))
    v1 = v0 + l1[:, None] * w1
    v2 = v0 + l2[:, None] * w2
    rnd = np.concatenate([v0, v1, v2], 1).astype(np.float32)
    tris = np.concatenate([room_box((-0.05,) * 3, (1.05,) * 3), rnd], 0)
    return SceneSpec("tiny", np.ascontiguousarray(tris), (0.5, 0.5, 1.0), (0.0, 0.0, -1.0),
                     (0.0, 1.0, 0.0), 60.0, lights=[(0.5, 0.95, 0.5)])


def frame_scene(seed: int = 3, n_spheres: int = 100, n_tori: int = 100, sphere_subdiv: int = 4,
                torus_res: int = 50) -> SceneSpec:
    """Paper-shaped frame: room [0,1]^3 + instanced icospheres and tori.

    Defaults give 12 + 100*5120 + 100*5000 = 1,012,012 triangles.  Each instance has
    radius r ~ U[0.02, 0.10], a uniform centre in [r + 0.01, 0.99 - r]^3 (so it stays inside
    the room; re-drawn if it comes near the camera) and a uniformly random rotation.
    """
    cam = np.array([0.5, 0.5, 0.97])
    sph = icosphere(sphere_subdiv)
    tor = torus(torus_res, torus_res, 0.7, 0.3)       # outer radius 1.0
    n_inst = n_spheres + n_tori
    centres = np.empty((n_inst, 3))
    radii = 0.02 + 0.08 * uniform01(seed, 10, np.arange(n_inst, dtype=np.uint64))
    for k in range(n_inst):
        draw = 0
        while True:
            idx = np.uint64(k * 64 + draw)
            u = np.array([uniform01(seed, 11 + a, idx) for a in range(3)]).reshape(3)
            c = (radii[k] + 0.01) + (0.98 - 2 * radii[k]) * u
            if np.linalg.norm(c - cam) > radii[k] + 0.03:
                break
            draw += 1
        centres[k] = c
    R = _rotations(seed, 20, n_inst)
    parts = [room_box((0.0,) * 3, (1.0,) * 3).reshape(-1, 3, 3).astype(np.float64)]
    for k in range(n_inst):
        base = sph if k < n_spheres else tor
        parts.append(np.einsum("ij,tvj->tvi", R[k], base) * radii[k] + centres[k])
    tris = np.concatenate(parts, 0).reshape(-1, 9).astype(np.float32)
    lights = [(0.3, 0.95, 0.5), (0.7, 0.95, 0.5)]
    return SceneSpec("frame", np.ascontiguousarray(tris), tuple(cam), (0.0, 0.0, -1.0),
                     (0.0, 1.0, 0.0), 60.0, lights=lights)


def cluster_scene(n_tris: int, seed: int = 5, n_clusters: int = 64, sigma: float = 0.05) -> SceneSpec:
    """Gaussian clusters of thin triangles inside the unit room.

    Cluster centres U[0.15, 0.85]^3, positions N(centre, sigma^2); each triangle has a long
    edge of length U[0.0005, 0.003] and aspect ratio U[1, 20] (short edge = long / aspect).
    """
    n = n_tris - 12
    idx = np.arange(n, dtype=np.uint64)
    cidx = np.arange(n_clusters, dtype=np.uint64)
    cc = 0.15 + 0.7 * np.stack([uniform01(seed, 30 + a, cidx) for a in range(3)], -1)
    which = (u64_hash(seed, 33, idx) % np.uint64(n_clusters)).astype(np.int64)
    # Box-Muller normals
    g = []
    for a in range(3):
        u1 = np.maximum(uniform01(seed, 34 + 2 * a, idx), 1e-300)
        u2 = uniform01(seed, 35 + 2 * a, idx)
        g.append(np.sqrt(-2 * np.log(u1)) * np.cos(2 * math.pi * u2))
    v0 = cc[which] + sigma * np.stack(g, -1)
    v0 = np.clip(v0, 0.001, 0.999)
    long_len = 0.0005 + 0.0025 * uniform01(seed, 40, idx)
    aspect = 1.0 + 19.0 * uniform01(seed, 41, idx)
    w1 = _unit_sphere_dirs(uniform01(seed, 42, idx), uniform01(seed, 43, idx))
    w2 = _unit_sphere_dirs(uniform01(seed, 44, idx), uniform01(seed, 45, idx))
    w2 = w2 - (w2 * w1).sum(-1, keepdims=True) * w1          # orthogonal to w1
    w2 /= np.maximum(np.linalg.norm(w2, axis=-1, keepdims=True), 1e-12)
    v1 = v0 + long_len[:, None] * w1
    v2 = v0 + 0.5 * long_len[:, None] * w1 + (long_len / aspect)[:, None] * w2
    tris = np.concatenate([room_box((0.0,) * 3, (1.0,) * 3),
                           np.concatenate([v0, v1, v2], 1).astype(np.float32)], 0)
    return SceneSpec(f"cluster{n_tris}", np.ascontiguousarray(tris), (0.5, 0.5, 0.97), (0.0, 0.0, -1.0),
                     (0.0, 1.0, 0.0), 60.0, lights=[(0.3, 0.95, 0.5), (0.7, 0.95, 0.5)])


# --------------------------------------------------------------------------- rays

def pinhole_rays(spec: SceneSpec, width: int, height: int, spp: int = 1, seed: int = 2,
                 jitter: bool | None = None) -> np.ndarray:
    """Primary rays of a pinhole camera, sample-major then row-major pixel order.

    With ``spp == 1`` and no jitter the rays pass through pixel centres.  Directions are
    normalised; tmin = 0, tmax = +inf.
    """
    if jitter is None:
        jitter = spp > 1
    fwd = np.asarray(spec.cam_dir, np.float64); fwd /= np.linalg.norm(fwd)
    up = np.asarray(spec.cam_up, np.float64)
    right = np.cross(fwd, up); right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    th = math.tan(math.radians(spec.vfov_deg) / 2)
    aspect = width / height
    n = width * height * spp
    k = np.arange(n, dtype=np.int64)
    s = k // (width * height)
    pix = k % (width * height)
    py = pix // width
    px = pix % width
    if jitter:
        jx = uniform01(seed, 50, k.astype(np.uint64))
        jy = uniform01(seed, 51, k.astype(np.uint64))
    else:
        jx = jy = 0.5
    sx = (2.0 * (px + jx) / width - 1.0) * th * aspect
    sy = (1.0 - 2.0 * (py + jy) / height) * th
    d = fwd[None] + sx[:, None] * right[None] + sy[:, None] * up[None]
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    out = np.empty((n, 8), np.float32)
    out[:, 0:3] = np.asarray(spec.cam_pos, np.float32)
    out[:, 3] = 0.0
    out[:, 4:7] = d
    out[:, 7] = np.inf
    del s
    return out


def _hit_frame(rays: np.ndarray, t: np.ndarray, prim: np.ndarray, tris: np.ndarray):
    o = rays[:, 0:3].astype(np.float64)
    d = rays[:, 4:7].astype(np.float64)
    p = o + t.astype(np.float64)[:, None] * d
    tr = tris[prim].astype(np.float64).reshape(-1, 3, 3)
    n = np.cross(tr[:, 1] - tr[:, 0], tr[:, 2] - tr[:, 0])
    n /= np.maximum(np.linalg.norm(n, axis=1, keepdims=True), 1e-300)
    flip = (n * d).sum(1) > 0
    n[flip] *= -1.0
    return p, n


def spawn_diffuse(rays: np.ndarray, t: np.ndarray, prim: np.ndarray, tris: np.ndarray,
                  seed: int, bounce: int) -> tuple[np.ndarray, np.ndarray]:
    """Cosine-weighted diffuse rays at the hit points of ``rays`` (misses dropped).

    Returns ``(new_rays, parent_index)``; order follows the parent rays.  tmin = 1e-4 * L
    (L = largest scene extent), tmax = +inf.
    """
    valid = np.nonzero(prim != np.uint32(0xFFFFFFFF))[0]
    p, n = _hit_frame(rays[valid], t[valid], prim[valid], tris)
    k = valid.astype(np.uint64)
    r1 = uniform01(seed, 100 + 2 * bounce, k)
    r2 = uniform01(seed, 101 + 2 * bounce, k)
    # branchless orthonormal basis (Duff et al. 2017)
    sign = np.where(n[:, 2] >= 0, 1.0, -1.0)
    a = -1.0 / (sign + n[:, 2])
    b = n[:, 0] * n[:, 1] * a
    b1 = np.stack([1.0 + sign * n[:, 0] ** 2 * a, sign * b, -sign * n[:, 0]], -1)
    b2 = np.stack([b, sign + n[:, 1] ** 2 * a, -n[:, 1]], -1)
    phi = 2 * math.pi * r1
    sr = np.sqrt(r2)
    d = (sr * np.cos(phi))[:, None] * b1 + (sr * np.sin(phi))[:, None] * b2 + np.sqrt(1 - r2)[:, None] * n
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    L = scene_extent(tris)
    out = np.empty((valid.size, 8), np.float32)
    out[:, 0:3] = p
    out[:, 3] = np.float32(1e-4 * L)
    out[:, 4:7] = d
    out[:, 7] = np.inf
    return out, valid


def spawn_shadow(rays: np.ndarray, t: np.ndarray, prim: np.ndarray, tris: np.ndarray,
                 lights: list) -> tuple[np.ndarray, np.ndarray]:
    """One shadow ray per (hit, light), hit-major order; segment ends 1e-4*L short of the light."""
    valid = np.nonzero(prim != np.uint32(0xFFFFFFFF))[0]
    p, _ = _hit_frame(rays[valid], t[valid], prim[valid], tris)
    L = scene_extent(tris)
    eps = 1e-4 * L
    nl = len(lights)
    out = np.empty((valid.size, nl, 8), np.float32)
    for j, lp in enumerate(lights):
        d = np.asarray(lp, np.float64)[None] - p
        dist = np.linalg.norm(d, axis=1)
        d /= np.maximum(dist, 1e-300)[:, None]
        out[:, j, 0:3] = p
        out[:, j, 3] = np.float32(eps)
        out[:, j, 4:7] = d
        out[:, j, 7] = (dist - eps).astype(np.float32)
    parent = np.repeat(valid, nl)
    return out.reshape(-1, 8), parent


def batch_plan(n_batches: int = 64, seed: int = 21, lo: int = 1024, hi: int = 2_097_152, n_scenes: int = 4,
               frac_closest: float = 0.7) -> list[dict]:
    """Uneven ray batches: size floor(exp(U[ln lo, ln hi])), scene uniform, closest hit with
    probability frac_closest (diffuse rays) else any hit (shadow rays), and an offset into the
    scene's ray pool."""
    k = np.arange(n_batches, dtype=np.uint64)
    size = np.floor(np.exp(np.log(lo) + (np.log(hi) - np.log(lo)) * uniform01(seed, 60, k))).astype(np.int64)
    scene = (u64_hash(seed, 61, k) % np.uint64(n_scenes)).astype(np.int64)
    closest = uniform01(seed, 62, k) < frac_closest
    offset = u64_hash(seed, 63, k)
    return [dict(n=int(size[i]), scene=int(scene[i]), closest=bool(closest[i]), offset=int(offset[i] % (1 << 40)))
            for i in range(n_batches)]


def take_rays(pool: np.ndarray, n: int, offset: int) -> np.ndarray:
    """n consecutive rays of a pool starting at offset (wrapping around)."""
    m = pool.shape[0]
    idx = (np.arange(n, dtype=np.int64) + (offset % m)) % m
    return np.ascontiguousarray(pool[idx])


# Named workload sizes (scene generator, camera resolution, samples, bounces).
TINY = dict(scene=tiny_scene, width=64, height=64, spp=1, bounces=1, cut=64, key_bits=32)
FRAME = dict(scene=frame_scene, width=1920, height=1080, spp=8, bounces=3, cut=(256, 4096), key_bits=32)
DRIFT = dict(scene=lambda seed=5: cluster_scene(10_000_000, seed), width=1920, height=1080, spp=4,
             bounces=2, key_bits=(16, 24, 32, 48, 64))
BATCH_SCENES = (10_000, 100_000, 1_000_000, 2_000_000)
