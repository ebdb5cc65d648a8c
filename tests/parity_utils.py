"""Comparison rules shared by the GPU parity tests.

Bars: keys, permutations, BVH topology, boxes and HAD bit-exact; closest-hit t within
1e-5 relative; triangle ids equal except at near-ties (|dt| < 1e-6, and the GPU's
triangle really is hit at its t); at most 1e-5 of the rays may disagree; any-hit flags
disagree on at most 1e-5 of the rays.  Between two traversals of which one tests a superset
of the other's triangles: the superset's hit is never farther, and where it differs it is a
real hit of its triangle.
"""
import numpy as np

import oracle as O

MISS = 0xFFFFFFFF
T_REL = 1e-5
TIE_DT = 1e-6
MAX_RATE = 1e-5


def compare_closest(gpu_hits: np.ndarray, ref: "O.Hits", rays: np.ndarray, tris: np.ndarray, idx=None):
    """Returns (mismatch count, rays compared, details).  gpu_hits: (n, 4) float32."""
    g = np.ascontiguousarray(gpu_hits, np.float32)
    if idx is None:
        idx = np.arange(g.shape[0])
    gt = g[idx, 0]
    gp = g[idx, 1].copy().view(np.uint32)
    gu, gv = g[idx, 2], g[idx, 3]
    rt, rp = ref.t[idx], ref.prim[idx]
    ru, rv = ref.u[idx], ref.v[idx]
    bad = []
    miss_g, miss_r = gp == MISS, rp == MISS
    bad.extend(idx[miss_g != miss_r].tolist())
    both = ~miss_g & ~miss_r
    with np.errstate(invalid="ignore"):
        t_bad = both & ~(np.abs(gt - rt) <= T_REL * np.abs(rt))
    bad.extend(idx[t_bad].tolist())
    pd = both & ~t_bad & (gp != rp)
    for k in np.nonzero(pd)[0]:
        r = idx[k]
        near_tie = abs(float(gt[k]) - float(rt[k])) < TIE_DT
        if near_tie:
            # the GPU's triangle must itself be hit at the reported distance
            h = O.brute_force(tris[int(gp[k])][None], rays[r][None])
            if h.prim[0] == 0 and h.t[0] == gt[k]:
                continue
        bad.append(int(r))
    same = both & (gp == rp) & ~t_bad
    uv_bad = same & ~((np.abs(gu - ru) <= 1e-5) & (np.abs(gv - rv) <= 1e-5))
    bad.extend(idx[uv_bad].tolist())
    # misses must report t = +inf and zero barycentrics
    mg = miss_g & miss_r
    bad.extend(idx[mg & ~(np.isinf(gt) & (gu == 0) & (gv == 0))].tolist())
    bad = sorted(set(bad))
    return len(bad), len(idx), bad[:10]


def assert_closest(gpu_hits, ref, rays, tris, idx=None):
    nbad, n, ex = compare_closest(gpu_hits, ref, rays, tris, idx)
    assert nbad <= MAX_RATE * n, f"{nbad} of {n} closest hits disagree, e.g. rays {ex}"


def assert_any(gpu_occ: np.ndarray, ref_occ: np.ndarray, idx=None):
    g = np.asarray(gpu_occ, np.uint8)
    r = np.asarray(ref_occ, np.uint8)
    if idx is not None:
        g, r = g[idx], r[idx]
    assert set(np.unique(g).tolist()) <= {0, 1}
    nbad = int((g != r).sum())
    assert nbad <= MAX_RATE * g.size, f"{nbad} of {g.size} any-hit flags disagree"


def _key(t, prim):
    return (float("inf") if prim == MISS else float(t), int(prim))


def assert_no_worse_closest(got: np.ndarray, base: np.ndarray, rays: np.ndarray, tris: np.ndarray, max_rate=MAX_RATE):
    """`got` comes from a traversal that tests every triangle `base`'s traversal tests and maybe
    more (quantised boxes contain the exact ones; 4-wide nodes skip intermediate boxes).  The
    Moller-Trumbore test can accept a ray passing just outside a triangle (and outside its box)
    by rounding, so such a traversal may find a hit the other one culled: on every ray got's
    distance is at most base's, and where the hits differ got's triangle is really hit at got's
    distance (the same test on that triangle alone).  At equal distances the triangles may differ:
    which of two triangles hit at the same t survives depends on the visiting order (a box whose
    entry distance rounds above the current hit's is culled).  max_rate bounds the share of rays
    that differ (None: no bound, for rays aimed at vertices and edges on purpose)."""
    g = np.ascontiguousarray(got, np.float32)
    b = np.ascontiguousarray(base, np.float32)
    diff = np.nonzero((g.view(np.uint32) != b.view(np.uint32)).any(1))[0]
    if max_rate is not None:
        assert diff.size <= max_rate * g.shape[0], f"{diff.size} of {g.shape[0]} hits differ, e.g. rays {diff[:10]}"
    for r in diff:
        gp, bp = int(g[r, 1:2].view(np.uint32)[0]), int(b[r, 1:2].view(np.uint32)[0])
        assert _key(g[r, 0], gp)[0] <= _key(b[r, 0], bp)[0] and gp != MISS, f"ray {r}: {g[r]} is farther than {b[r]}"
        h = O.brute_force(tris[gp][None], rays[r][None])
        assert h.prim[0] == 0 and h.t[0] == g[r, 0] and h.u[0] == g[r, 2] and h.v[0] == g[r, 3], f"ray {r}"


def assert_no_fewer_any(got: np.ndarray, base: np.ndarray, upper=None, max_rate=MAX_RATE):
    """Any-hit flags of a traversal testing a superset of base's triangles: every ray base
    finds occluded is occluded in got; got differs from base on at most max_rate of the rays
    (None: no bound) and, given `upper` (brute force), never reports a ray no triangle hits."""
    g = np.asarray(got, np.uint8)
    b = np.asarray(base, np.uint8)
    assert not (b & ~g).any(), "a ray occluded in the base traversal is not occluded"
    if max_rate is not None:
        assert int((g != b).sum()) <= max_rate * g.size
    if upper is not None:
        assert not (g & ~np.asarray(upper, np.uint8)).any(), "occluded without any triangle hit"


def assert_stable_sort(keys: np.ndarray, perm: np.ndarray):
    """A stable ascending sort is unique: bijection + non-decreasing keys + equal keys in
    input order fixes it completely (exact check at any size)."""
    n = keys.shape[0]
    perm = np.asarray(perm, np.uint32).astype(np.int64)
    assert perm.shape[0] == n
    seen = np.zeros(n, bool)
    seen[perm] = True
    assert seen.all(), "not a permutation"
    ks = np.asarray(keys)[perm].astype(np.uint64)
    assert (ks[1:] >= ks[:-1]).all(), "keys not ascending"
    eq = ks[1:] == ks[:-1]
    assert (perm[1:][eq] > perm[:-1][eq]).all(), "equal keys out of input order"
