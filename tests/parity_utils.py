"""Comparison rules shared by the GPU parity tests.

Bars: keys, permutations, BVH topology, boxes and HAD bit-exact; closest-hit t within
1e-5 relative; triangle ids equal except at near-ties (|dt| < 1e-6, and the GPU's
triangle really is hit at its t); at most 1e-5 of the rays may disagree; any-hit flags
disagree on at most 1e-5 of the rays.
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
