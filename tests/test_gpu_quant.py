"""Quantised 4-wide nodes (HCC_TRACE_QUANT) on geometry that strains 8-bit steps.

Every slot box of a quantised node is stored as steps from the node's corner, rounded outwards,
so the traversal tests a superset of the boxes the exact nodes pass and must return the same hits.
The scenes below make the rounding matter: all triangles in one plane (every node has zero extent
on that axis), coordinates far from the origin (steps of a few float ulps), triangles a million
times smaller than their neighbours (decoded boxes far looser than the boxes they hold), negative
coordinates, and rays with zero direction components or running inside the plane of the triangles
(the slab form of the child test).  Each launch is compared with the oracle and, bit for bit, with
the same launch on the exact nodes."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from parity_utils import assert_any, assert_closest, assert_no_fewer_any, assert_no_worse_closest

pytestmark = pytest.mark.gpu

N_TRIS = 20_000
N_RAYS = 6_000


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _u(seed, stream, n):
    return W.uniform01(seed, stream, np.arange(n, dtype=np.uint64))


def _tris(centres, size, seed):
    n = centres.shape[0]
    e1 = (np.stack([_u(seed, 10 + a, n) for a in range(3)], -1) - 0.5) * size
    e2 = (np.stack([_u(seed, 13 + a, n) for a in range(3)], -1) - 0.5) * size
    return np.concatenate([centres, centres + e1, centres + e2], 1)


def scene(kind: str) -> np.ndarray:
    s = {"flat": 1, "far": 2, "scales": 3, "negative": 4}[kind]
    c = np.stack([_u(s, a, N_TRIS) for a in range(3)], -1)
    if kind == "flat":                      # every vertex at z = 0.5
        t = _tris(c, 0.02, s)
        t[:, 2::3] = 0.5
    elif kind == "far":                     # around (3e4, -2e4, 1e4): float steps of 2^-9 .. 2^-8
        t = _tris(c * 40.0 + np.array([3e4, -2e4, 1e4]), 0.2, s)
    elif kind == "scales":                  # triangles of size 1e-5 next to triangles of size 1
        t = _tris(c, 1e-5, s)
        t[: N_TRIS // 20] = _tris(c[: N_TRIS // 20], 1.0, s + 7)
    else:                                   # all coordinates negative
        t = _tris(-1.0 - c * 3.0, 0.05, s)
    return t.astype(np.float32)


def rays_for(tris: np.ndarray, kind: str, seed: int) -> np.ndarray:
    lo, hi = tris.reshape(-1, 3).min(0), tris.reshape(-1, 3).max(0)
    ext = np.maximum(hi - lo, 0.25 * float((hi - lo).max()))   # origins off a flat scene's plane too
    lo = (lo + hi) / 2 - ext / 2
    n = N_RAYS
    o = lo - 0.1 * ext + 1.2 * ext * np.stack([_u(seed, a, n) for a in range(3)], -1)
    d = np.stack([_u(seed, 3 + a, n) for a in range(3)], -1) - 0.5
    # a quarter of the rays along the axes (zero direction components), a quarter towards triangles
    q = n // 4
    ax = (np.arange(q) % 3)
    d[:q] = 0.0
    d[np.arange(q), ax] = np.where(_u(seed, 7, q) < 0.5, -1.0, 1.0)
    target = tris[(np.arange(q) * 7919) % tris.shape[0], 0:3]
    d[q:2 * q] = target[: q] - o[q:2 * q]
    if kind == "flat":                      # rays inside the plane of the triangles
        o[2 * q:2 * q + q // 2, 2] = 0.5
        d[2 * q:2 * q + q // 2, 2] = 0.0
    d /= np.maximum(np.linalg.norm(d, axis=1, keepdims=True), 1e-30)
    r = np.zeros((n, 8), np.float64)
    r[:, 0:3] = o
    r[:, 4:7] = d
    r[:, 7] = np.where(np.arange(n) % 3 == 0, 0.5 * float(ext.max()), np.inf)
    return r.astype(np.float32)


@pytest.fixture(scope="module")
def H():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2305_16652_amd as H
    return H


@pytest.mark.parametrize("kind", ["flat", "far", "scales", "negative"])
def test_quantised_nodes_against_exact_nodes_and_oracle(H, kind):
    """A quarter of the rays aim at triangle vertices: there Moller-Trumbore's rounding can
    accept a ray that passes just outside the triangle and its box, which brute force finds and
    a traversal may cull (the oracle's BVH2 traversal does so on 30 of the flat scene's rays).
    Every launch therefore has to lie between the oracle's traversal and brute force: never a
    farther hit than the oracle's, and every other hit a real one (brute force is the nearest
    real hit).  The quantised nodes keep the same relation to the exact 4-wide nodes."""
    _say(f"quantised nodes, scene {kind}")
    tris = scene(kind)
    rays = rays_for(tris, kind, seed=5)
    ob = O.build_bvh(tris)
    ref_c = O.trace(ob, rays, threads=8)
    ref_a = O.trace(ob, rays, closest=False, threads=8)
    bf_a = O.brute_force(tris, rays, closest=False)
    assert (ref_c.prim != O.MISS).mean() > 0.03
    bvh = H.build_bvh(torch.from_numpy(tris).cuda())
    rd = torch.from_numpy(rays).cuda()
    perm = torch.from_numpy(np.random.default_rng(3).permutation(N_RAYS).astype(np.int32)).cuda()
    for base in (H.TRACE_WIDE, H.TRACE_WIDE | H.TRACE_SLAB):
        exact_o = H.TraceOpts(64, 2, 0, 1, 32, 64, 0, base)
        quant_o = H.TraceOpts(64, 2, 0, 1, 32, 64, 0, base | H.TRACE_QUANT)
        exact = H.trace(bvh, rd, perm, opts=exact_o).cpu().numpy()
        quant = H.trace(bvh, rd, perm, opts=quant_o).cpu().numpy()
        assert_no_worse_closest(exact, ref_c.raw, rays, tris, max_rate=None)
        assert_no_worse_closest(quant, ref_c.raw, rays, tris, max_rate=None)
        assert_no_worse_closest(quant, exact, rays, tris, max_rate=None)
        occ_e = H.trace(bvh, rd, perm, closest=False, opts=exact_o).cpu().numpy()
        occ_q = H.trace(bvh, rd, perm, closest=False, opts=quant_o).cpu().numpy()
        assert_no_fewer_any(occ_e, ref_a, upper=bf_a, max_rate=None)
        assert_no_fewer_any(occ_q, occ_e, upper=bf_a, max_rate=None)
        # rays that do not aim at a vertex: the usual parity bar against the oracle
        rest = np.r_[0:N_RAYS // 4, N_RAYS // 2:N_RAYS]
        assert_closest(quant, ref_c, rays, tris, idx=rest)
        assert_any(occ_q, ref_a, idx=rest)


def test_quantised_nodes_single_triangle_and_small_scenes(H):
    """One triangle (no wide nodes: the launch falls back to the one-ray-per-lane kernel) and
    scenes of 2..9 triangles (one or two wide nodes with empty slots)."""
    for n in (1, 2, 3, 5, 9):
        tris = scene("negative")[:n]
        rays = rays_for(tris, "negative", seed=n)
        ob = O.build_bvh(tris)
        ref = O.trace(ob, rays)
        bvh = H.build_bvh(torch.from_numpy(tris).cuda())
        got = H.trace(bvh, torch.from_numpy(rays).cuda(),
                      opts=H.TraceOpts(64, 2, 0, 1, 32, 64, 0, H.TRACE_WIDE | H.TRACE_QUANT)).cpu().numpy()
        # the vertex-aimed quarter: between the oracle's traversal and brute force; the rest: parity
        assert_no_worse_closest(got, ref.raw, rays, tris, max_rate=None)
        assert_closest(got, ref, rays, tris, idx=np.r_[0:N_RAYS // 4, N_RAYS // 2:N_RAYS])


def test_quantised_nodes_need_the_wide_traversal(H):
    tris = scene("far")[:100]
    bvh = H.build_bvh(torch.from_numpy(tris).cuda())
    rd = torch.from_numpy(rays_for(tris, "far", seed=1)).cuda()
    with pytest.raises(H.HCCError):
        H.trace(bvh, rd, opts=H.TraceOpts(0, 0, 0, 1, 32, 64, 0, H.TRACE_QUANT))
    with pytest.raises(H.HCCError):
        H.trace(bvh, rd, opts=H.TraceOpts(64, 0, 0, 0, 0, 0, 0, H.TRACE_QUANT))


def _decode(q, s, p):
    """The traversal's decode, fmaf(q, s, p): q * s is exact in float32, so one float32 add."""
    return (q.astype(np.float32) * s.astype(np.float32)).astype(np.float32) + p.astype(np.float32)


@pytest.mark.parametrize("kind", ["tiny", "cluster", "flat", "far", "scales", "negative"])
def test_wide_and_quantised_nodes_structure(H, kind):
    """The 4-wide nodes against the exported BVH2, and the quantised nodes against the 4-wide
    ones, on the host: every triangle is the leaf slot of exactly one wide node, with its BVH2
    leaf box bit for bit; an internal slot's box is the exact union of its wide node's slot boxes
    and every wide node but the root is one slot's; the root's slots cover the BVH2 root box.
    Quantised: the same refs; per axis the corner is the least lower plane and the step a power of
    two whose step 255 reaches the node's upper plane; every slot's decoded lower plane is the
    largest step at most its lower plane, its decoded upper plane the smallest step at least its
    upper plane; empty slots hold steps 255 / 0."""
    _say(f"wide node structure, scene {kind}")
    if kind == "tiny":
        tris = W.tiny_scene().tris
    elif kind == "cluster":
        tris = W.cluster_scene(50_000, seed=7).tris
    else:
        tris = scene(kind)
    bvh = H.build_bvh(torch.from_numpy(np.ascontiguousarray(tris, np.float32)).cuda())
    child, leaf_prim, boxes, had = bvh.export()
    (planes, refs), (cs, steps, qrefs), ok = bvh.export_wide()
    n = tris.shape[0]
    ni = n - 1
    EMPTY, LEAF = np.uint32(0xFFFFFFFF), np.uint32(0x80000000)
    w = planes.shape[0]
    assert ok and w > 0
    full = refs != EMPTY
    is_leaf = full & ((refs & LEAF) != 0)
    is_int = full & ~is_leaf
    # leaves: each triangle once, with its BVH2 leaf box
    li = (refs[is_leaf] & ~LEAF).astype(np.int64)
    assert np.array_equal(np.sort(li), np.arange(n))
    wl, jl = np.nonzero(is_leaf)
    got = planes[wl, :, jl]                           # (k, 6): lo.xyz, hi.xyz
    assert np.array_equal(got.view(np.uint32), boxes[ni + li].view(np.uint32))
    # internal slots: wide nodes 1..w-1 once each, box = union of that node's slot boxes
    ci = refs[is_int].astype(np.int64)
    assert np.array_equal(np.sort(ci), np.arange(1, w))
    lo = np.where(full[:, None, :], planes[:, 0:3, :], np.float32(np.inf)).min(axis=2)
    hi = np.where(full[:, None, :], planes[:, 3:6, :], np.float32(-np.inf)).max(axis=2)
    wi, ji = np.nonzero(is_int)
    assert np.array_equal(planes[wi, 0:3, ji], lo[ci]) and np.array_equal(planes[wi, 3:6, ji], hi[ci])
    assert np.array_equal(np.concatenate([lo[0], hi[0]]), boxes[0])
    # quantised copy
    assert np.array_equal(qrefs, refs)
    p, s = cs[:, 0:3], cs[:, 3:6]
    assert np.array_equal(p, lo)
    m, e = np.frexp(s.astype(np.float64))
    assert (m == 0.5).all()                           # powers of two
    assert (_decode(np.full_like(p, 255), s, p) >= hi).all()
    for a in range(3):
        for j in range(4):
            ql = (steps[:, 2 * a] >> np.uint32(8 * j)) & np.uint32(255)
            qh = (steps[:, 2 * a + 1] >> np.uint32(8 * j)) & np.uint32(255)
            f = full[:, j]
            assert (ql[~f] == 255).all() and (qh[~f] == 0).all()
            L, U = planes[f, a, j], planes[f, 3 + a, j]
            qlf, qhf, pf, sf = ql[f], qh[f], p[f, a], s[f, a]
            dl, dh = _decode(qlf, sf, pf), _decode(qhf, sf, pf)
            assert (dl <= L).all() and (dh >= U).all()
            up = qlf < 255
            assert (_decode(qlf[up] + 1, sf[up], pf[up]) > L[up]).all()
            down = qhf > 0
            assert (_decode(qhf[down] - 1, sf[down], pf[down]) < U[down]).all()
