"""Autotuner for the trace launch options and the HCC cut size / key length.

Times candidate configurations on the device with HIP events (through the C ABI) and keeps
the fastest.  The search space covers what the trace kernels expose: one-ray-per-lane blocks
(64/128/256 lanes) vs persistent wavefronts, the stack placement (scratch, LDS, split), the
persistent refill threshold, chunk size and speculative descent, and for the 4-wide traversal
the wavefront count, the child-box test (selected planes or slab, whichever suits the
scene's size against the caches), exact or quantised nodes, and whether the chunk counter deals
chunks in order or spread over the order; for HCC additionally the cut size C and key length K (the
paper's configuration is C = K).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import torch

from . import (KEY_HCC, KEY_TWOPOINT, TraceOpts, encode, select_cut, sort_ex, sort_workspace_bytes,
               trace)

PLAIN = [TraceOpts(b, s, 0, 0, 0, 0, 0, 0) for b in (64, 128) for s in (0, 2)]
PERSISTENT = [TraceOpts(64, s, 0, 1, r, c, 8192, f)
              for s in (0,) for r in (24, 32) for c in (64, 128, 256) for f in (0, 1)]
# 4-wide: LDS short stack, both child-box tests (selected planes / slab, flags 2 / 6) on the exact
# or the quantised nodes (flag 16), chunks dealt in order or spread over the order (flag 8)
WIDE = [TraceOpts(64, 2, 0, 1, r, c, 8192, f | q | sp) for f in (2, 6) for q in (0, 16) for sp in (0, 8)
        for r in (24, 32) for c in (64, 128, 256)]
# wavefront packets over the 4-wide nodes (flag 32): exact or quantised nodes, chunks in order or
# spread.  A packet costs one step per node of the union of its 64 rays' traversals, so these pay
# only on coherent rays (primary rays, shadow rays towards one light, well ordered rays); on
# diffuse secondary rays they are several times slower than the per-lane launches
PACKET = [TraceOpts(0, 0, 0, 1, 0, 0, 8192, 2 | q | sp | 32) for q in (0, 16) for sp in (0, 8)]
DEFAULT_CANDIDATES = PLAIN + PERSISTENT + WIDE + PACKET


def opts_dict(o: TraceOpts) -> dict:
    return {name: int(getattr(o, name)) for name, _ in o._fields_}


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def tune_trace(bvh, rays, perm=None, closest: bool = True, candidates=None, reps: int = 2):
    """Fastest trace options for these rays in this order: (TraceOpts, ms, table)."""
    n = rays.shape[0]
    out = (torch.empty((n, 4), dtype=torch.float32, device=rays.device) if closest
           else torch.empty(n, dtype=torch.uint8, device=rays.device))
    table = []
    for o in candidates or DEFAULT_CANDIDATES:
        ms = _time(lambda: trace(bvh, rays, perm, closest=closest, out=out, opts=o), reps)
        table.append((ms, opts_dict(o)))
    table.sort(key=lambda x: x[0])
    best = TraceOpts(*table[0][1].values())
    return best, table[0][0], table


@dataclass
class Choice:
    mode: str
    cut: int
    key_bits: int
    opts: TraceOpts
    encode_ms: float
    sort_ms: float
    trace_ms: float
    skip: int = 0          # low key bits the sort leaves out (a stable sort by key >> skip)

    @property
    def total_ms(self) -> float:
        return self.encode_ms + self.sort_ms + self.trace_ms

    def as_dict(self) -> dict:
        return dict(mode=self.mode, cut=self.cut, key_bits=self.key_bits, skip=self.skip, opts=opts_dict(self.opts),
                    encode_ms=round(self.encode_ms, 4), sort_ms=round(self.sort_ms, 4),
                    trace_ms=round(self.trace_ms, 4), total_ms=round(self.total_ms, 4))


def tune_reorder(bvh, rays, mode: str, cuts=(32, 64), key_bits=(32, 64), closest: bool = True,
                 candidates=None, reps: int = 2, paper_exact: bool = True, skips=(0,),
                 min_sorted_frac: float = 0.0) -> tuple[Choice, list]:
    """Best (cut, key length, skipped low bits, trace options) for a reordering method, by total
    encode + sort + trace time.  mode: 'hcc' or 'twopoint' (cut ignored).  With paper_exact only
    C = K pairs, otherwise every pair with C >= K (the key then holds the K cut nodes of highest
    HAD).  skips: numbers of low key bits the sort may leave out (the paper's shortened sort),
    limited to those that keep at least min_sorted_frac of the key's bits in the sort; the trace
    options are tuned on the first of them and reused for the others."""
    n = rays.shape[0]
    dev = rays.device
    results = []
    if mode == "hcc":
        pairs = [(c, k) for c, k in itertools.product(cuts, key_bits) if (c == k or (not paper_exact and c >= k))]
    else:
        pairs = [(0, k) for k in key_bits]
    out = (torch.empty((n, 4), dtype=torch.float32, device=dev) if closest
           else torch.empty(n, dtype=torch.uint8, device=dev))
    for c, k in pairs:
        cut = select_cut(bvh, c) if mode == "hcc" else None
        keys = torch.empty(n, dtype=torch.int32 if k <= 32 else torch.int64, device=dev)
        perm = torch.empty(n, dtype=torch.int32, device=dev)
        ws = torch.empty(sort_workspace_bytes(n, k), dtype=torch.uint8, device=dev)
        m = KEY_HCC if mode == "hcc" else KEY_TWOPOINT
        enc_ms = _time(lambda: encode(bvh, cut, m, k, rays, out=keys), reps)
        o = None
        for s in skips:
            if s >= k or (k - s) < min_sorted_frac * k:
                continue
            sort_ms = _time(lambda: sort_ex(keys, k, s, 0, perm=perm, ws=ws), reps)
            if o is None:
                o, tr_ms, _ = tune_trace(bvh, rays, perm, closest, candidates, reps)
            else:
                tr_ms = _time(lambda: trace(bvh, rays, perm, closest=closest, out=out, opts=o), reps)
            results.append(Choice(mode, c, k, o, enc_ms, sort_ms, tr_ms, s))
    results.sort(key=lambda ch: ch.total_ms)
    return results[0], results
