"""Python front of the plain CPU oracle (test infrastructure only).

The oracle is the slow, obviously correct reference the GPU path is checked
against.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
may import it; the product package never does.  All arithmetic lives in
``hcc_oracle.c`` (plain C, no FMA contraction); this file only marshals numpy
arrays.  Every function cites the passage of the paper it follows in the C file.
"""
from __future__ import annotations

import ctypes as C
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

MISS = 0xFFFFFFFF


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    P = C.c_void_p
    u32 = C.c_uint32
    lib.oracle_scene_box.argtypes = [P, u32, P]
    lib.oracle_morton3.argtypes = [u32, u32, u32]
    lib.oracle_morton3.restype = u32
    lib.oracle_morton_codes.argtypes = [P, u32, P]
    lib.oracle_build_bvh.argtypes = [P, u32, P, P, P, P]
    lib.oracle_build_bvh.restype = C.c_int
    lib.oracle_had.argtypes = [u32, P, P, C.c_double, P]
    lib.oracle_select_cut.argtypes = [u32, P, P, u32, P]
    lib.oracle_select_cut.restype = C.c_int
    lib.oracle_slab.argtypes = [P, P]
    lib.oracle_slab.restype = C.c_int
    lib.oracle_encode_hcc.argtypes = [P, u32, P, u32, u32, P]
    lib.oracle_encode_twopoint.argtypes = [P, u32, P, u32, P]
    lib.oracle_sort.argtypes = [P, u32, P]
    lib.oracle_sort.restype = C.c_int
    lib.oracle_trace.argtypes = [u32, P, P, P, P, P, P, u32, u32, C.c_int, P, P, P, P]
    lib.oracle_brute_force.argtypes = [P, u32, P, u32, C.c_int, P, P]
    lib.oracle_anc.argtypes = [P, P, u32, u32]
    lib.oracle_anc.restype = C.c_double
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a, cols):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a.reshape(-1, cols)


class OracleBVH:
    """LBVH produced by the oracle (unified node ids: internal i, leaf n-1+j)."""

    def __init__(self, tris, child, leaf_prim, boxes, codes):
        self.tris = tris
        self.n = tris.shape[0]
        self.child = child          # (n-1, 2) uint32
        self.leaf_prim = leaf_prim  # (n,) uint32
        self.boxes = boxes          # (2n-1, 6) float32
        self.codes = codes          # (n,) uint32, Morton codes in sorted order

    def is_leaf(self, node_id: int) -> bool:
        return self.n == 1 or node_id >= self.n - 1


def scene_box(tris) -> np.ndarray:
    tris = _f32(tris, 9)
    out = np.empty(6, np.float32)
    _load().oracle_scene_box(_ptr(tris), tris.shape[0], _ptr(out))
    return out


def morton3(qx: int, qy: int, qz: int) -> int:
    return int(_load().oracle_morton3(qx, qy, qz))


def morton_codes(tris) -> np.ndarray:
    tris = _f32(tris, 9)
    out = np.empty(tris.shape[0], np.uint32)
    _load().oracle_morton_codes(_ptr(tris), tris.shape[0], _ptr(out))
    return out


def build_bvh(tris) -> OracleBVH:
    tris = _f32(tris, 9)
    n = tris.shape[0]
    if n == 0:
        raise ValueError("empty scene")
    child = np.zeros((max(n - 1, 0), 2), np.uint32)
    leaf_prim = np.empty(n, np.uint32)
    boxes = np.empty((2 * n - 1, 6), np.float32)
    codes = np.empty(n, np.uint32)
    rc = _load().oracle_build_bvh(_ptr(tris), n, _ptr(child), _ptr(leaf_prim), _ptr(boxes), _ptr(codes))
    if rc != 0:
        raise MemoryError(f"oracle_build_bvh failed ({rc})")
    return OracleBVH(tris, child, leaf_prim, boxes, codes)


def had(bvh: OracleBVH, lam: float = 0.125) -> np.ndarray:
    out = np.empty(2 * bvh.n - 1, np.float64)
    _load().oracle_had(bvh.n, _ptr(bvh.child), _ptr(bvh.boxes), float(lam), _ptr(out))
    return out


def select_cut(bvh: OracleBVH, had_values: np.ndarray, cut_size: int) -> np.ndarray:
    ids = np.empty(cut_size + 2, np.uint32)
    had_values = np.ascontiguousarray(had_values, np.float64)
    m = _load().oracle_select_cut(bvh.n, _ptr(bvh.child), _ptr(had_values), cut_size, _ptr(ids))
    if m < 0:
        raise ValueError(f"oracle_select_cut failed ({m})")
    return ids[:m].copy()


def slab(ray, box) -> bool:
    ray = np.ascontiguousarray(ray, np.float32).reshape(8)
    box = np.ascontiguousarray(box, np.float32).reshape(6)
    return bool(_load().oracle_slab(_ptr(ray), _ptr(box)))


def _chunks(n: int, threads: int):
    threads = max(1, min(threads, n))
    step = (n + threads - 1) // threads if n else 0
    return [(k, min(n, k + step)) for k in range(0, n, step)] if n else []


def _key_dtype(key_bits: int):
    return np.uint32 if key_bits <= 32 else np.uint64


def encode_hcc(rays, cut_boxes, key_bits: int, threads: int = 1) -> np.ndarray:
    rays = _f32(rays, 8)
    cb = _f32(cut_boxes, 6)
    n = rays.shape[0]
    out = np.empty(n, np.uint64)
    lib = _load()

    def run(rng):
        k0, k1 = rng
        lib.oracle_encode_hcc(_ptr(rays[k0:k1]), k1 - k0, _ptr(cb), cb.shape[0], key_bits, _ptr(out[k0:k1]))

    with ThreadPoolExecutor(max(1, threads)) as ex:
        list(ex.map(run, _chunks(n, threads)))
    return out.astype(_key_dtype(key_bits))


def encode_twopoint(rays, scene_lohi, key_bits: int, threads: int = 1) -> np.ndarray:
    rays = _f32(rays, 8)
    lohi = np.ascontiguousarray(scene_lohi, np.float32).reshape(6)
    n = rays.shape[0]
    out = np.empty(n, np.uint64)
    lib = _load()

    def run(rng):
        k0, k1 = rng
        lib.oracle_encode_twopoint(_ptr(rays[k0:k1]), k1 - k0, _ptr(lohi), key_bits, _ptr(out[k0:k1]))

    with ThreadPoolExecutor(max(1, threads)) as ex:
        list(ex.map(run, _chunks(n, threads)))
    return out.astype(_key_dtype(key_bits))


def sort(keys) -> np.ndarray:
    keys64 = np.ascontiguousarray(keys, np.uint64)
    perm = np.empty(keys64.shape[0], np.uint32)
    rc = _load().oracle_sort(_ptr(keys64), keys64.shape[0], _ptr(perm))
    if rc != 0:
        raise MemoryError("oracle_sort failed")
    return perm


class Hits:
    """Closest-hit results indexed by original ray id."""

    def __init__(self, raw: np.ndarray):
        self.raw = raw                                   # (n, 4) float32 words
        self.t = raw[:, 0].copy()
        self.prim = raw[:, 1].copy().view(np.uint32)
        self.u = raw[:, 2].copy()
        self.v = raw[:, 3].copy()


def trace(bvh: OracleBVH, rays, perm=None, closest: bool = True, threads: int = 1,
          counters: bool = False, subset=None):
    """Trace every ray (or the rays listed in ``subset``) through the oracle BVH.

    Returns ``Hits`` (closest) or a uint8 occlusion array (any); with ``counters``
    also per-ray (boxes passed, triangle tests).  Results are by original ray id;
    rays outside ``subset`` are left zero.
    """
    rays = _f32(rays, 8)
    n = rays.shape[0]
    if subset is not None:
        perm = np.ascontiguousarray(subset, np.uint32)
    elif perm is not None:
        perm = np.ascontiguousarray(perm, np.uint32)
    m = n if perm is None else perm.shape[0]
    hits = np.zeros((n, 4), np.float32) if closest else None
    occ = None if closest else np.zeros(n, np.uint8)
    nn = np.zeros(n, np.uint32) if counters else None
    nt = np.zeros(n, np.uint32) if counters else None
    lib = _load()
    tris = bvh.tris

    def run(rng):
        k0, k1 = rng
        lib.oracle_trace(bvh.n, _ptr(bvh.child), _ptr(bvh.leaf_prim), _ptr(bvh.boxes), _ptr(tris),
                         _ptr(rays), _ptr(perm), k0, k1, 1 if closest else 0, _ptr(hits), _ptr(occ),
                         _ptr(nn), _ptr(nt))

    with ThreadPoolExecutor(max(1, threads)) as ex:
        list(ex.map(run, _chunks(m, max(1, threads) * 8 if threads > 1 else 1)))
    res = Hits(hits) if closest else occ
    if counters:
        return res, nn, nt
    return res


def brute_force(tris, rays, closest: bool = True):
    tris = _f32(tris, 9)
    rays = _f32(rays, 8)
    n = rays.shape[0]
    hits = np.zeros((n, 4), np.float32) if closest else None
    occ = None if closest else np.zeros(n, np.uint8)
    _load().oracle_brute_force(_ptr(tris), tris.shape[0], _ptr(rays), n, 1 if closest else 0,
                               _ptr(hits), _ptr(occ))
    return Hits(hits) if closest else occ


def anc(keys, perm=None, width: int = 32) -> float:
    keys64 = np.ascontiguousarray(keys, np.uint64)
    p = None if perm is None else np.ascontiguousarray(perm, np.uint32)
    return float(_load().oracle_anc(_ptr(keys64), _ptr(p), keys64.shape[0], width))


def cut_boxes(bvh: OracleBVH, ids) -> np.ndarray:
    return np.ascontiguousarray(bvh.boxes[np.asarray(ids, np.int64)])


def _load_extra():
    lib = _load()
    if getattr(lib, "_extra", False):
        return lib
    P, u32 = C.c_void_p, C.c_uint32
    lib.oracle_select_mlhcc_cut.argtypes = [u32, P, P, u32, u32, P, P]
    lib.oracle_select_mlhcc_cut.restype = C.c_int
    lib.oracle_encode_mlhcc.argtypes = [P, u32, P, u32, P, u32, u32, P]
    lib.oracle_grid_boxes.argtypes = [P, u32, u32, u32, P]
    lib.oracle_encode_ppc.argtypes = [P, u32, u32, P, P, u32, P]
    lib._extra = True
    return lib


def select_mlhcc_cut(bvh: OracleBVH, had_values, top: int, low: int):
    """Two-level cut (Section 4.3, Alg. 3): (top_ids (T',), low_ids (T', low))."""
    had_values = np.ascontiguousarray(had_values, np.float64)
    top_ids = np.empty(top + 2, np.uint32)
    low_ids = np.empty((top + 2) * low, np.uint32)
    m = _load_extra().oracle_select_mlhcc_cut(bvh.n, _ptr(bvh.child), _ptr(had_values), top, low, _ptr(top_ids),
                                              _ptr(low_ids))
    if m < 0:
        raise ValueError(f"oracle_select_mlhcc_cut failed ({m})")
    return top_ids[:m].copy(), low_ids[: m * low].reshape(m, low).copy()


def encode_mlhcc(rays, top_boxes, low_boxes, low: int, key_bits: int, threads: int = 1) -> np.ndarray:
    rays = _f32(rays, 8)
    tb = _f32(top_boxes, 6)
    lb = _f32(low_boxes, 6)
    n = rays.shape[0]
    out = np.empty(n, np.uint64)
    lib = _load_extra()

    def run(rng):
        k0, k1 = rng
        lib.oracle_encode_mlhcc(_ptr(rays[k0:k1]), k1 - k0, _ptr(tb), tb.shape[0], _ptr(lb), low, key_bits,
                                _ptr(out[k0:k1]))

    with ThreadPoolExecutor(max(1, threads)) as ex:
        list(ex.map(run, _chunks(n, threads)))
    return out.astype(_key_dtype(key_bits))


def encode_ppc(bvh: OracleBVH, rays, key_bits: int, threads: int = 1) -> np.ndarray:
    """Prefix path code (Section 4.1): the first key_bits box tests of a forced-order walk."""
    rays = _f32(rays, 8)
    n = rays.shape[0]
    out = np.empty(n, np.uint64)
    lib = _load_extra()

    def run(rng):
        k0, k1 = rng
        lib.oracle_encode_ppc(_ptr(rays[k0:k1]), k1 - k0, bvh.n, _ptr(bvh.child), _ptr(bvh.boxes), key_bits,
                              _ptr(out[k0:k1]))

    with ThreadPoolExecutor(max(1, threads)) as ex:
        list(ex.map(run, _chunks(n, threads)))
    return out.astype(_key_dtype(key_bits))


def sort_prefix(keys, key_bits: int, skip_bits: int) -> np.ndarray:
    """Early-terminated sort (Sections 6.5 and 6.6.1: the order inside one warp does not matter, so the last bits may be skipped): the stable
    ascending permutation by the key's top key_bits - skip_bits bits; the low skip_bits bits do
    not take part."""
    k = np.ascontiguousarray(keys).astype(np.uint64) >> np.uint64(skip_bits)
    return sort(k)


def sort_tiles(keys, tile: int) -> np.ndarray:
    """Tile-local sort: consecutive groups of `tile` rays (the last one ragged) are each sorted
    stably by key on their own; no ray leaves its group."""
    k = np.ascontiguousarray(keys).astype(np.uint64)
    perm = np.empty(k.shape[0], np.uint32)
    for t0 in range(0, k.shape[0], tile):
        t1 = min(k.shape[0], t0 + tile)
        perm[t0:t1] = t0 + sort(k[t0:t1])
    return perm


def grid_dims(key_bits: int):
    """Most cubic gx >= gy >= gz with gx*gy*gz == key_bits (the regular-grid control)."""
    best = None
    for gz in range(1, key_bits + 1):
        for gy in range(gz, key_bits + 1):
            if key_bits % (gy * gz):
                continue
            gx = key_bits // (gy * gz)
            if gx < gy:
                continue
            score = gx - gz
            if best is None or score < best[0]:
                best = (score, gx, gy, gz)
    return best[1:]


def grid_boxes(scene_lohi, gx: int, gy: int, gz: int) -> np.ndarray:
    lohi = np.ascontiguousarray(scene_lohi, np.float32).reshape(6)
    out = np.empty((gx * gy * gz, 6), np.float32)
    _load_extra().oracle_grid_boxes(_ptr(lohi), gx, gy, gz, _ptr(out))
    return out


def wave_fetches(bvh: OracleBVH, rays, perm=None, width: int = 64, closest: bool = True, order: int = 1,
                 waves=None, threads: int = 1):
    """Lockstep wave model (the per-warp coherence argument of Section 3.1; Table 6 in
    Section 6.5): rays in trace order, waves of ``width`` consecutive rays; per wave the
    distinct nodes and distinct triangles fetched at each lockstep step, summed over the
    steps.  ``order`` 0 is the traversal of ``trace``; 1 the child-test traversal (see
    ``oracle_wave_fetches`` in the C file).  ``waves`` lists the wave indices to model
    (default: all).  Returns (nodes, tris, steps), one entry per listed wave."""
    rays = _f32(rays, 8)
    n = rays.shape[0] if perm is None else len(perm)
    p = None if perm is None else np.ascontiguousarray(perm, np.uint32)
    n_w = (n + width - 1) // width
    w = np.arange(n_w, dtype=np.uint32) if waves is None else np.ascontiguousarray(waves, np.uint32)
    nodes = np.zeros(w.shape[0], np.uint64)
    trisf = np.zeros(w.shape[0], np.uint64)
    steps = np.zeros(w.shape[0], np.uint32)
    lib = _load()
    if not getattr(lib, "_wave", False):
        P, u32 = C.c_void_p, C.c_uint32
        lib.oracle_wave_fetches.argtypes = [u32, P, P, P, P, P, P, u32, u32, C.c_int, C.c_int, P, u32, P, P, P]
        lib.oracle_wave_fetches.restype = C.c_int
        lib._wave = True

    def run(rng):
        k0, k1 = rng
        rc = lib.oracle_wave_fetches(bvh.n, _ptr(bvh.child), _ptr(bvh.leaf_prim), _ptr(bvh.boxes), _ptr(bvh.tris),
                                     _ptr(rays), _ptr(p), n, width, 1 if closest else 0, order, _ptr(w[k0:k1]),
                                     k1 - k0, _ptr(nodes[k0:k1]), _ptr(trisf[k0:k1]), _ptr(steps[k0:k1]))
        if rc != 0:
            raise RuntimeError(f"oracle_wave_fetches failed ({rc})")

    with ThreadPoolExecutor(max(1, threads)) as ex:
        list(ex.map(run, _chunks(w.shape[0], max(1, threads) * 8 if threads > 1 else 1)))
    return nodes, trisf, steps
