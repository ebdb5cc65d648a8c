"""Python binding of the gfx950 hierarchy-cut-code library (``libhcc.so``).

Argument marshalling only: every step of the path runs in the library's HIP kernels;
PyTorch provides device memory and the stream.  The C declarations and their
documentation are in ``include/hcc.h``.  If the library has not been built this
module raises on import -- there is no fallback.

Tensor conventions (all on the current CUDA/HIP device):
  triangles: (N, 9) float32          rays: (R, 8) float32 [ox oy oz tmin dx dy dz tmax]
  keys: int32 (key_bits <= 32) or int64 tensors holding the unsigned key bits
  perm: int32 tensor holding uint32 ray indices
  closest hits: (R, 4) float32 = (t, prim bits, u, v); ``hits_prim`` views the prim ids
  any hits: (R,) uint8
"""
from __future__ import annotations

import ctypes as C
import os

import torch

__all__ = [
    "lib", "HCCError", "BVH", "Cut", "build_bvh", "select_cut", "encode", "sort", "sort_workspace_bytes",
    "trace", "trace_stats", "hits_prim", "KEY_HCC", "KEY_TWOPOINT", "STACK_LDS", "STACK_SCRATCH",
    "STACK_SHORT", "TraceOpts", "LIB_PATH",
]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhcc.so")

KEY_NONE, KEY_HCC, KEY_TWOPOINT = 0, 1, 2
CLOSEST, ANY = 0, 1
STACK_SCRATCH, STACK_LDS, STACK_SHORT = 0, 1, 2
_STATUS = {0: "HCC_OK", 1: "HCC_ERR_INVALID", 2: "HCC_ERR_OOM", 3: "HCC_ERR_DEVICE", 4: "HCC_ERR_UNSUPPORTED",
           5: "HCC_ERR_BUDGET"}


class HCCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class TraceOpts(C.Structure):
    """hcc_trace_opts: block, stack, xcd_remap, persistent, refill, chunk, waves, flags (0 = default)."""
    _fields_ = [("block", C.c_uint32), ("stack", C.c_uint32), ("xcd_remap", C.c_uint32),
                ("persistent", C.c_uint32), ("refill", C.c_uint32), ("chunk", C.c_uint32),
                ("waves", C.c_uint32), ("flags", C.c_uint32)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2305_16652_amd/build.py "
                      "(or __graft_entry__.build()); there is no fallback path")
lib = C.CDLL(LIB_PATH)

_P = C.c_void_p
_U32 = C.c_uint32
_H = C.c_void_p
_SIGS = {
    "hcc_build_bvh": [_P, _U32, _P, C.POINTER(_H)],
    "hcc_bvh_info": [_H, C.POINTER(_U32), C.POINTER(_U32), _P, C.POINTER(C.c_size_t)],
    "hcc_bvh_export": [_H, _P, _P, _P, _P],
    "hcc_bvh_export_wide": [_H, C.POINTER(_U32), _P, _P, C.POINTER(_U32)],
    "hcc_select_cut": [_H, _U32, C.c_double, _P, C.POINTER(_H)],
    "hcc_cut_info": [_H, C.POINTER(_U32)],
    "hcc_cut_export": [_H, _P, _P, _P],
    "hcc_encode": [_H, _H, C.c_int, _U32, _P, _U32, _P, _P],
    "hcc_sort_workspace": [_U32, _U32, C.POINTER(C.c_size_t)],
    "hcc_sort": [_P, _U32, _U32, _P, _P, _P, C.c_size_t, _P],
    "hcc_trace": [_H, _P, _P, _U32, C.c_int, _P, _P, _P],
    "hcc_trace_ex": [_H, _P, _P, _U32, C.c_int, _P, _P, C.POINTER(TraceOpts), _P],
    "hcc_trace_stats": [_H, _P, _P, _U32, C.c_int, _P, _P, _P, _P, _P, _P, _P],
}
for _name, _args in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
lib.hcc_bvh_destroy.argtypes = [_H]
lib.hcc_bvh_destroy.restype = None
lib.hcc_cut_destroy.argtypes = [_H]
lib.hcc_cut_destroy.restype = None
lib.hcc_last_error.restype = C.c_char_p
lib.hcc_version.restype = C.c_char_p


def _check(status: int):
    if status != 0:
        raise HCCError(status, lib.hcc_last_error().decode())


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)
lib.hcc_set_allocator.argtypes = [_P, _P, _P]
lib.hcc_set_allocator.restype = C.c_int
_HOOKS = []   # every installed callback pair stays alive: objects made under it free through it


def set_allocator(alloc=None, free=None):
    """Route the library's own device memory (handles, build temporaries, server workspaces)
    through ``alloc(nbytes, stream_ptr) -> int`` and ``free(ptr, stream_ptr)``.  With no
    arguments the library goes back to hipMalloc / hipFree for objects created afterwards."""
    if alloc is None and free is None:
        _check(lib.hcc_set_allocator(None, None, None))
        return
    if alloc is None or free is None:
        raise ValueError("give both alloc and free, or neither")

    def _a(nbytes, stream, ctx):
        try:
            return alloc(int(nbytes), stream or 0) or None
        except Exception:       # an exception cannot cross the C boundary: report OOM instead
            return None

    def _f(ptr, stream, ctx):
        try:
            free(ptr, stream or 0)
        except Exception:
            pass

    pair = (ALLOC_FN(_a), FREE_FN(_f))
    _HOOKS.append(pair)
    _check(lib.hcc_set_allocator(C.cast(pair[0], _P), C.cast(pair[1], _P), None))


def use_torch_allocator(device=None):
    """Back the library's device memory with PyTorch's caching allocator."""
    dev = torch.cuda.current_device() if device is None else device
    set_allocator(lambda n, s: torch.cuda.caching_allocator_alloc(max(n, 1), dev, s),
                  lambda p, s: torch.cuda.caching_allocator_delete(p))


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return C.c_void_p(t.data_ptr())


def _key_dtype(key_bits: int):
    return torch.int32 if key_bits <= 32 else torch.int64


class BVH:
    """Library-owned BVH handle (immutable after the build)."""

    def __init__(self, handle: int, tris: torch.Tensor):
        self._h = C.c_void_p(handle)
        self.tris = tris                      # kept alive only for callers' convenience
        n, nodes, size = _U32(), _U32(), C.c_size_t()
        box = (C.c_float * 6)()
        _check(lib.hcc_bvh_info(self._h, C.byref(n), C.byref(nodes), box, C.byref(size)))
        self.n = n.value
        self.n_nodes = nodes.value
        self.scene_box = list(box)
        self.device_bytes = size.value

    @property
    def handle(self):
        return self._h

    def export(self):
        """(child (n-1,2) u32, leaf_prim (n,) u32, boxes (2n-1,6) f32, had (2n-1,) f64) as numpy."""
        import numpy as np
        n = self.n
        child = np.zeros((max(n - 1, 0), 2), np.uint32)
        leaf = np.empty(n, np.uint32)
        boxes = np.empty((2 * n - 1, 6), np.float32)
        had = np.empty(2 * n - 1, np.float64)
        _check(lib.hcc_bvh_export(self._h, child.ctypes.data_as(_P), leaf.ctypes.data_as(_P),
                                  boxes.ctypes.data_as(_P), had.ctypes.data_as(_P)))
        return child, leaf, boxes, had

    def export_wide(self):
        """The 4-wide traversal nodes as numpy: (planes (w,6,4) f32, refs (w,4) u32) of the exact
        nodes, (corner_step (w,6) f32, steps (w,6) u32, refs (w,4) u32) of the quantised ones, and
        whether the quantised traversal is offered."""
        import numpy as np
        nw, ok = _U32(), _U32()
        _check(lib.hcc_bvh_export_wide(self._h, C.byref(nw), None, None, C.byref(ok)))
        w = nw.value
        wide = np.zeros((w, 32), np.uint32)
        quant = np.zeros((w, 16), np.uint32)
        _check(lib.hcc_bvh_export_wide(self._h, C.byref(nw), wide.ctypes.data_as(_P), quant.ctypes.data_as(_P),
                                       C.byref(ok)))
        planes = wide[:, :24].copy().view(np.float32).reshape(w, 6, 4)
        exact_refs = wide[:, 24:28].copy()
        corner_step = quant[:, :6].copy().view(np.float32)
        steps = quant[:, 6:12].copy()
        quant_refs = quant[:, 12:16].copy()
        return (planes, exact_refs), (corner_step, steps, quant_refs), bool(ok.value)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.hcc_bvh_destroy(h)
            self._h = C.c_void_p(0)


class Cut:
    def __init__(self, handle: int, bvh: BVH):
        self._h = C.c_void_p(handle)
        self.bvh = bvh
        c = _U32()
        _check(lib.hcc_cut_info(self._h, C.byref(c)))
        self.c_eff = c.value

    @property
    def handle(self):
        return self._h

    def export(self):
        import numpy as np
        ids = np.empty(self.c_eff, np.uint32)
        had = np.empty(self.c_eff, np.float64)
        boxes = np.empty((self.c_eff, 6), np.float32)
        _check(lib.hcc_cut_export(self._h, ids.ctypes.data_as(_P), had.ctypes.data_as(_P),
                                  boxes.ctypes.data_as(_P)))
        return ids, had, boxes

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.hcc_cut_destroy(h)
            self._h = C.c_void_p(0)


def build_bvh(tris: torch.Tensor, stream=None) -> BVH:
    if tris.dtype != torch.float32 or tris.dim() != 2 or tris.shape[1] != 9:
        raise ValueError("triangles must be an (N, 9) float32 tensor")
    h = _H()
    _check(lib.hcc_build_bvh(_dptr(tris), tris.shape[0], _stream(stream), C.byref(h)))
    return BVH(h.value, tris)


def select_cut(bvh: BVH, cut_size: int, lam: float = 0.125, stream=None) -> Cut:
    h = _H()
    _check(lib.hcc_select_cut(bvh.handle, cut_size, float(lam), _stream(stream), C.byref(h)))
    return Cut(h.value, bvh)


KEY_MLHCC = 3
KEY_PPC = 4
lib.hcc_select_mlhcc_cut.argtypes = [_H, _U32, _U32, C.c_double, _P, C.POINTER(_H)]
lib.hcc_grid_cut.argtypes = [_H, _U32, _U32, _U32, _P, C.POINTER(_H)]
lib.hcc_cut_shape.argtypes = [_H, C.POINTER(_U32), C.POINTER(_U32), C.POINTER(_U32)]
lib.hcc_cut_export_low.argtypes = [_H, _P, _P]
for _f in (lib.hcc_select_mlhcc_cut, lib.hcc_grid_cut, lib.hcc_cut_shape, lib.hcc_cut_export_low):
    _f.restype = C.c_int


def select_mlhcc_cut(bvh: BVH, top: int, low: int, lam: float = 0.125, stream=None) -> Cut:
    """Two-level cut of the multi-level hierarchy cut code (encode with KEY_MLHCC)."""
    h = _H()
    _check(lib.hcc_select_mlhcc_cut(bvh.handle, top, low, float(lam), _stream(stream), C.byref(h)))
    return Cut(h.value, bvh)


def grid_dims(cells: int):
    """The most cubic factorisation gx >= gy >= gz of a cell count (one key bit per cell)."""
    best = None
    for gz in range(1, cells + 1):
        if cells % gz:
            continue
        for gy in range(gz, cells // gz + 1):
            if (cells // gz) % gy or cells // (gz * gy) < gy:
                continue
            gx = cells // (gz * gy)
            if best is None or gx - gz < best[0] - best[2]:
                best = (gx, gy, gz)
    return best


def grid_cut(bvh: BVH, gx: int, gy: int, gz: int, stream=None) -> Cut:
    """Regular-grid control encoding: grid cells in place of cut nodes (encode with KEY_HCC)."""
    h = _H()
    _check(lib.hcc_grid_cut(bvh.handle, gx, gy, gz, _stream(stream), C.byref(h)))
    return Cut(h.value, bvh)


def cut_shape(cut: Cut):
    k, t, l = _U32(), _U32(), _U32()
    _check(lib.hcc_cut_shape(cut.handle, C.byref(k), C.byref(t), C.byref(l)))
    return k.value, t.value, l.value


def cut_export_low(cut: Cut):
    import numpy as np
    _, t, l = cut_shape(cut)
    ids = np.empty((t, l), np.uint32)
    boxes = np.empty((t, l, 6), np.float32)
    _check(lib.hcc_cut_export_low(cut.handle, ids.ctypes.data_as(_P), boxes.ctypes.data_as(_P)))
    return ids, boxes


def _check_rays(rays: torch.Tensor):
    if rays.dtype != torch.float32 or rays.dim() != 2 or rays.shape[1] != 8:
        raise ValueError("rays must be an (R, 8) float32 tensor")


def encode(bvh: BVH, cut: Cut | None, mode: int, key_bits: int, rays: torch.Tensor, out=None,
           stream=None) -> torch.Tensor:
    _check_rays(rays)
    n = rays.shape[0]
    if out is None:
        out = torch.empty(n, dtype=_key_dtype(key_bits), device=rays.device)
    _check(lib.hcc_encode(bvh.handle, cut.handle if cut is not None else None, mode, key_bits, _dptr(rays), n,
                          _dptr(out), _stream(stream)))
    return out


def sort_workspace_bytes(n: int, key_bits: int) -> int:
    b = C.c_size_t()
    _check(lib.hcc_sort_workspace(n, key_bits, C.byref(b)))
    return b.value


def sort(keys: torch.Tensor, key_bits: int, perm=None, sorted_keys=None, ws=None, stream=None) -> torch.Tensor:
    n = keys.shape[0]
    if perm is None:
        perm = torch.empty(n, dtype=torch.int32, device=keys.device)
    need = sort_workspace_bytes(n, key_bits)
    if ws is None:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=keys.device)
    _check(lib.hcc_sort(_dptr(keys), key_bits, n, _dptr(perm), _dptr(sorted_keys), _dptr(ws), ws.numel(),
                        _stream(stream)))
    return perm


lib.hcc_sort_ex.argtypes = [_P, _U32, _U32, _U32, _U32, _P, _P, _P, C.c_size_t, _P]
lib.hcc_sort_ex.restype = C.c_int


def sort_ex(keys: torch.Tensor, key_bits: int, skip_bits: int = 0, tile: int = 0, perm=None, sorted_keys=None,
            ws=None, stream=None) -> torch.Tensor:
    """Stable sort by the key's bits [skip_bits, key_bits), over all keys (tile 0) or within
    consecutive tiles of `tile` keys (256 ... 4096, no workspace)."""
    n = keys.shape[0]
    if perm is None:
        perm = torch.empty(n, dtype=torch.int32, device=keys.device)
    if tile == 0 and ws is None:
        ws = torch.empty(max(sort_workspace_bytes(n, key_bits), 256), dtype=torch.uint8, device=keys.device)
    _check(lib.hcc_sort_ex(_dptr(keys), key_bits, skip_bits, tile, n, _dptr(perm), _dptr(sorted_keys), _dptr(ws),
                           ws.numel() if ws is not None else 0, _stream(stream)))
    return perm


lib.hcc_sort_static.argtypes = [_P, _U32, _U32, _P, _P, _P]
lib.hcc_sort_static.restype = C.c_int
lib.hcc_sort_static_bytes.argtypes = [C.POINTER(C.c_size_t)]
lib.hcc_sort_static_bytes.restype = C.c_int
SORT_STATIC_MAX_KEYS = 1 << 20


def sort_static_bytes() -> int:
    b = C.c_size_t()
    _check(lib.hcc_sort_static_bytes(C.byref(b)))
    return b.value


def sort_static(keys: torch.Tensor, key_bits: int, perm: torch.Tensor, sorted_keys=None, stream=None) -> torch.Tensor:
    """hcc_sort with the library's static workspace (allocates nothing; perm is the caller's)."""
    _check(lib.hcc_sort_static(_dptr(keys), key_bits, keys.shape[0], _dptr(perm), _dptr(sorted_keys),
                               _stream(stream)))
    return perm


def trace(bvh: BVH, rays: torch.Tensor, perm=None, closest: bool = True, out=None, opts: TraceOpts | None = None,
          stream=None) -> torch.Tensor:
    _check_rays(rays)
    n = rays.shape[0]
    if out is None:
        out = (torch.empty((n, 4), dtype=torch.float32, device=rays.device) if closest
               else torch.empty(n, dtype=torch.uint8, device=rays.device))
    hits, occ = (out, None) if closest else (None, out)
    _check(lib.hcc_trace_ex(bvh.handle, _dptr(rays), _dptr(perm), n, CLOSEST if closest else ANY, _dptr(hits),
                            _dptr(occ), C.byref(opts) if opts is not None else None, _stream(stream)))
    return out


TRACE_SPECULATE, TRACE_WIDE, TRACE_SLAB, TRACE_SPREAD, TRACE_QUANT, TRACE_PACKET = 1, 2, 4, 8, 16, 32
BATCH_STACK_SCRATCH = 3
lib.hcc_trace_count.argtypes = [_H, _P, _P, _U32, C.c_int, _P, _P, C.POINTER(TraceOpts), _P, _P]
lib.hcc_trace_count.restype = C.c_int


def trace_count(bvh: BVH, rays: torch.Tensor, perm=None, closest: bool = True, opts: TraceOpts | None = None,
                out=None, stream=None):
    """Trace with a persistent or 4-wide launch that also counts the wavefront-distinct node and
    triangle fetches.  Returns (results, node_fetches, triangle_fetches)."""
    _check_rays(rays)
    n = rays.shape[0]
    if out is None:
        out = (torch.empty((n, 4), dtype=torch.float32, device=rays.device) if closest
               else torch.empty(n, dtype=torch.uint8, device=rays.device))
    hits, occ = (out, None) if closest else (None, out)
    counts = torch.zeros(2, dtype=torch.int64, device=rays.device)
    _check(lib.hcc_trace_count(bvh.handle, _dptr(rays), _dptr(perm), n, CLOSEST if closest else ANY, _dptr(hits),
                               _dptr(occ), C.byref(opts) if opts is not None else None, _dptr(counts),
                               _stream(stream)))
    c = counts.cpu().tolist()
    return out, int(c[0]), int(c[1])


def trace_stats(bvh: BVH, rays: torch.Tensor, perm=None, closest: bool = True, stream=None):
    """Trace with per-ray and per-wavefront fetch counters (measurement only)."""
    _check_rays(rays)
    n = rays.shape[0]
    dev = rays.device
    out = (torch.empty((n, 4), dtype=torch.float32, device=dev) if closest
           else torch.empty(n, dtype=torch.uint8, device=dev))
    hits, occ = (out, None) if closest else (None, out)
    nodes = torch.empty(n, dtype=torch.int32, device=dev)
    tris = torch.empty(n, dtype=torch.int32, device=dev)
    waves = (n + 63) // 64
    wn = torch.empty(max(waves, 1), dtype=torch.int32, device=dev)
    wt = torch.empty(max(waves, 1), dtype=torch.int32, device=dev)
    _check(lib.hcc_trace_stats(bvh.handle, _dptr(rays), _dptr(perm), n, CLOSEST if closest else ANY, _dptr(hits),
                               _dptr(occ), _dptr(nodes), _dptr(tris), _dptr(wn), _dptr(wt), _stream(stream)))
    return out, nodes, tris, wn[:waves], wt[:waves]


def hits_prim(hits: torch.Tensor) -> torch.Tensor:
    """The prim-id column of closest-hit results as int32 (0xFFFFFFFF shows as -1)."""
    return hits[:, 1].contiguous().view(torch.int32)


# ------------------------------------------------------------------------------ batched engine

class BatchDesc(C.Structure):
    _fields_ = [("bvh", C.c_void_p), ("cut", C.c_void_p), ("d_rays", C.c_void_p), ("n", C.c_uint32),
                ("mode", C.c_uint32), ("d_hits", C.c_void_p), ("d_occluded", C.c_void_p)]


class BatchOpts(C.Structure):
    """hcc_batch_opts: chunk (rays per trace item), refill, waves (0 = default), flags (TRACE_WIDE),
    direct_min (0 = one engine launch for all; else batches of at least this many rays, >= 65536,
    run through the full-device kernels), stack (4-wide trace phase: 0 / STACK_SHORT 12 LDS
    entries, STACK_LDS 24, BATCH_STACK_SCRATCH none)."""
    _fields_ = [("chunk", C.c_uint32), ("refill", C.c_uint32), ("waves", C.c_uint32), ("flags", C.c_uint32),
                ("direct_min", C.c_uint32), ("stack", C.c_uint32)]


lib.hcc_batch_workspace.argtypes = [C.c_void_p, C.c_uint32, C.c_int, C.c_uint32, C.POINTER(C.c_size_t)]
lib.hcc_batch_workspace.restype = C.c_int
lib.hcc_batch_run.argtypes = [C.c_void_p, C.c_uint32, C.c_int, C.c_uint32, C.c_void_p, C.c_void_p, C.c_size_t,
                              C.c_void_p]
lib.hcc_batch_run.restype = C.c_int


class Batch:
    """One ray batch for the engine: scene (BVH + cut), rays, trace mode and output tensor."""

    def __init__(self, bvh: BVH, rays: torch.Tensor, closest: bool = True, cut: Cut | None = None, out=None):
        _check_rays(rays)
        self.bvh, self.cut, self.rays, self.closest = bvh, cut, rays, closest
        n = rays.shape[0]
        if out is None:
            out = (torch.empty((n, 4), dtype=torch.float32, device=rays.device) if closest
                   else torch.empty(n, dtype=torch.uint8, device=rays.device))
        self.out = out

    def desc(self) -> BatchDesc:
        n = self.rays.shape[0]
        return BatchDesc(self.bvh.handle.value, self.cut.handle.value if self.cut is not None else None,
                         self.rays.data_ptr() if n else None, n, CLOSEST if self.closest else ANY,
                         self.out.data_ptr() if (self.closest and n) else None,
                         self.out.data_ptr() if (not self.closest and n) else None)


def _descs(batches):
    arr = (BatchDesc * len(batches))(*[b.desc() for b in batches])
    return arr


def batch_workspace_bytes(batches, mode: int, key_bits: int) -> int:
    arr = _descs(batches)
    b = C.c_size_t()
    _check(lib.hcc_batch_workspace(C.cast(arr, C.c_void_p), len(batches), mode, key_bits, C.byref(b)))
    return b.value


def batch_run(batches, mode: int, key_bits: int = 32, opts: BatchOpts | None = None, ws=None, stream=None):
    """Run every batch (encode + sort + trace, or trace only for KEY_NONE) in one persistent
    launch.  Results land in each Batch's ``out``.  Returns the workspace tensor (reusable)."""
    arr = _descs(batches)
    need = batch_workspace_bytes(batches, mode, key_bits)
    dev = batches[0].rays.device
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    _check(lib.hcc_batch_run(C.cast(arr, C.c_void_p), len(batches), mode, key_bits,
                             C.byref(opts) if opts is not None else None, C.c_void_p(ws.data_ptr()), ws.numel(),
                             _stream(stream)))
    return ws


lib.hcc_batch_export.argtypes = [C.c_void_p, C.c_uint32, C.c_int, C.c_uint32, C.c_void_p, C.c_void_p, C.c_size_t,
                                 C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p]
lib.hcc_batch_export.restype = C.c_int


def batch_export(batches, mode: int, key_bits: int, ws, index: int, opts: BatchOpts | None = None, stream=None):
    """Batch ``index``'s final permutation and sorted keys from the workspace of the last
    batch_run with the same batches, mode, key length and options: (perm int32, keys)."""
    arr = _descs(batches)
    n = batches[index].rays.shape[0]
    dev = batches[index].rays.device
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    keys = torch.empty(max(n, 1), dtype=torch.int32 if key_bits <= 32 else torch.int64, device=dev)
    _check(lib.hcc_batch_export(C.cast(arr, C.c_void_p), len(batches), mode, key_bits,
                                C.byref(opts) if opts is not None else None, C.c_void_p(ws.data_ptr()), ws.numel(),
                                index, _dptr(perm), _dptr(keys), _stream(stream)))
    return perm[:n], keys[:n]


lib.hcc_batch_check.argtypes = [_P, _P, C.POINTER(C.c_uint32)]
lib.hcc_batch_check.restype = C.c_int


def batch_check(ws, stream=None) -> bool:
    """Wait for the stream; True when the last batch_run on this workspace resolved every
    dependency inside its launch."""
    ok = C.c_uint32()
    _check(lib.hcc_batch_check(C.c_void_p(ws.data_ptr()), _stream(stream), C.byref(ok)))
    return bool(ok.value)


# ------------------------------------------------------------------------------ request server

class ServerOpts(C.Structure):
    _fields_ = [("budget_bytes", C.c_uint64), ("max_inflight", C.c_uint32), ("max_group", C.c_uint32),
                ("streams", C.c_uint32), ("key_mode", C.c_uint32), ("key_bits", C.c_uint32), ("plain", C.c_uint32),
                ("graphs", C.c_uint32), ("direct_min", C.c_uint32), ("batch", BatchOpts)]


class ServerCounters(C.Structure):
    _fields_ = [("launches", C.c_uint64), ("completed", C.c_uint64), ("queued", C.c_uint64),
                ("running", C.c_uint64), ("used_bytes", C.c_uint64)]


REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_CANCELLED, REQ_FAILED = 0, 1, 2, 3, 4

lib.hcc_server_create.argtypes = [C.POINTER(ServerOpts), C.POINTER(C.c_void_p)]
lib.hcc_server_submit.argtypes = [C.c_void_p, C.POINTER(BatchDesc), C.POINTER(C.c_uint64)]
lib.hcc_server_poll.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_uint32), C.POINTER(C.c_double)]
lib.hcc_server_cancel.argtypes = [C.c_void_p, C.c_uint64]
lib.hcc_server_drain.argtypes = [C.c_void_p]
lib.hcc_server_stats.argtypes = [C.c_void_p, C.POINTER(ServerCounters)]
for _f in (lib.hcc_server_create, lib.hcc_server_submit, lib.hcc_server_poll, lib.hcc_server_cancel,
           lib.hcc_server_drain, lib.hcc_server_stats):
    _f.restype = C.c_int
lib.hcc_server_destroy.argtypes = [C.c_void_p]
lib.hcc_server_destroy.restype = None


class Server:
    """Continuous-batching request server (native worker thread in libhcc)."""

    def __init__(self, key_mode: int = KEY_HCC, key_bits: int = 32, budget_bytes: int = 64 << 30,
                 max_inflight: int = 64, max_group: int = 16, streams: int = 4, plain: bool = False,
                 batch: BatchOpts | None = None, graphs: bool = True, direct_min: int = 0):
        o = ServerOpts(budget_bytes, max_inflight, max_group, streams, key_mode, key_bits, 1 if plain else 0,
                       1 if graphs else 0, direct_min, batch if batch is not None else BatchOpts())
        h = C.c_void_p()
        _check(lib.hcc_server_create(C.byref(o), C.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, batch: Batch) -> int:
        d = batch.desc()
        rid = C.c_uint64()
        _check(lib.hcc_server_submit(self._h, C.byref(d), C.byref(rid)))
        self._keep[rid.value] = batch          # buffers must outlive the request
        return rid.value

    def poll(self, rid: int):
        st, lat = C.c_uint32(), C.c_double()
        _check(lib.hcc_server_poll(self._h, rid, C.byref(st), C.byref(lat)))
        return st.value, lat.value

    def cancel(self, rid: int):
        _check(lib.hcc_server_cancel(self._h, rid))

    def drain(self):
        _check(lib.hcc_server_drain(self._h))

    def counters(self) -> dict:
        c = ServerCounters()
        _check(lib.hcc_server_stats(self._h, C.byref(c)))
        return {name: int(getattr(c, name)) for name, _ in c._fields_}

    def close(self):
        if self._h is not None and self._h.value and lib is not None:
            lib.hcc_server_destroy(self._h)
            self._h = C.c_void_p(0)
        self._keep = {}

    def __del__(self):
        self.close()
