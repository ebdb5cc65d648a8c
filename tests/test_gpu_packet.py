"""Wavefront packets (HCC_TRACE_PACKET): one walk of the 4-wide tree per 64 consecutive rays.

A packet visits every node some lane's child-box test passes, so each lane tests a superset of
the triangles its own traversal tests and keeps the same closest (t, triangle) rule: the hits are
the per-lane traversal's, except that Moller-Trumbore's rounding may accept a ray passing just
outside a triangle whose box only other lanes pass.  The checks: against the oracle at the usual
parity bar, never farther than the per-lane traversal (and every differing hit a real one),
any-hit flags a superset of the per-lane ones; on the frame's ray kinds (primary, diffuse
secondary, shadow) in pixel order, through an HCC permutation and through a random one; on
packets cut short by the end of the rays; and on the scenes built to strain the quantised nodes.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from parity_utils import assert_any, assert_closest, assert_no_fewer_any, assert_no_worse_closest
from test_gpu_quant import N_RAYS, rays_for, scene

pytestmark = pytest.mark.gpu

PACKET_FLAGS = [2 | 32, 2 | 16 | 32, 2 | 16 | 4 | 32, 2 | 16 | 8 | 32]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def H():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2305_16652_amd as H
    return H


@pytest.fixture(scope="module")
def cluster(H):
    spec = W.cluster_scene(60_000, seed=11)
    ob = O.build_bvh(spec.tris)
    prim = W.pinhole_rays(spec, 160, 120, 2, seed=4)
    ph = O.trace(ob, prim, threads=8)
    sec, _ = W.spawn_diffuse(prim, ph.t, ph.prim, spec.tris, seed=9, bounce=0)
    shd, _ = W.spawn_shadow(prim, ph.t, ph.prim, spec.tris, spec.lights)
    bvh = H.build_bvh(torch.from_numpy(spec.tris).cuda())
    rays = dict(primary=prim, secondary=sec, shadow=shd)
    ref = {k: (O.trace(ob, r, threads=8), O.trace(ob, r, closest=False, threads=8)) for k, r in rays.items()}
    return dict(spec=spec, ob=ob, bvh=bvh, rays=rays, ref=ref)


def _perms(H, bvh, rays_d, n):
    cut = H.select_cut(bvh, 32)
    hcc = H.sort(H.encode(bvh, cut, H.KEY_HCC, 32, rays_d), 32)
    rnd = torch.from_numpy(np.random.default_rng(n).permutation(n).astype(np.int32)).cuda()
    return dict(pixel=None, hcc=hcc, random=rnd)


@pytest.mark.parametrize("flags", PACKET_FLAGS)
def test_packets_on_cluster_scene(H, cluster, flags):
    tris = cluster["spec"].tris
    bvh = cluster["bvh"]
    per_lane = H.TraceOpts(64, 2, 0, 1, 32, 64, 0, flags & ~32 & ~8)
    o = H.TraceOpts(0, 0, 0, 1, 0, 0, 0, flags)
    for kind, rays in cluster["rays"].items():
        _say(f"packets flags {flags}, {kind} rays")
        ref_c, ref_a = cluster["ref"][kind]
        rd = torch.from_numpy(rays).cuda()
        base_c = H.trace(bvh, rd, opts=per_lane).cpu().numpy()
        base_a = H.trace(bvh, rd, closest=False, opts=per_lane).cpu().numpy()
        for name, perm in _perms(H, bvh, rd, rays.shape[0]).items():
            got = H.trace(bvh, rd, perm, opts=o).cpu().numpy()
            assert_closest(got, ref_c, rays, tris)
            assert_no_worse_closest(got, base_c, rays, tris)
            occ = H.trace(bvh, rd, perm, closest=False, opts=o).cpu().numpy()
            assert_any(occ, ref_a)
            assert_no_fewer_any(occ, base_a)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 127, 129, 1000])
def test_partial_packets(H, cluster, n):
    """Ray counts that leave the last packet partly empty, through a permutation of the prefix."""
    rays = cluster["rays"]["secondary"][:n]
    ref_c, ref_a = cluster["ref"]["secondary"]
    rd = torch.from_numpy(np.ascontiguousarray(rays)).cuda()
    perm = torch.from_numpy(np.random.default_rng(n).permutation(n).astype(np.int32)).cuda()
    for flags in (2 | 32, 2 | 16 | 32):
        o = H.TraceOpts(0, 0, 0, 1, 0, 0, 5, flags)
        got = H.trace(cluster["bvh"], rd, perm, opts=o).cpu().numpy()
        assert_closest(got, O.Hits(ref_c.raw[:n]), rays, cluster["spec"].tris)
        occ = H.trace(cluster["bvh"], rd, perm, closest=False, opts=o).cpu().numpy()
        assert_any(occ, ref_a[:n])


@pytest.mark.parametrize("kind", ["flat", "far", "scales", "negative"])
def test_packets_on_strained_scenes(H, kind):
    """As the quantised-node test on the same scenes: a quarter of the rays aim at vertices, so
    every launch must lie between the oracle's traversal and brute force there, and meet the
    parity bar on the other rays."""
    _say(f"packets, scene {kind}")
    tris = scene(kind)
    rays = rays_for(tris, kind, seed=6)
    ob = O.build_bvh(tris)
    ref_c = O.trace(ob, rays, threads=8)
    ref_a = O.trace(ob, rays, closest=False, threads=8)
    bf_a = O.brute_force(tris, rays, closest=False)
    bvh = H.build_bvh(torch.from_numpy(tris).cuda())
    rd = torch.from_numpy(rays).cuda()
    perm = torch.from_numpy(np.random.default_rng(4).permutation(N_RAYS).astype(np.int32)).cuda()
    rest = np.r_[0:N_RAYS // 4, N_RAYS // 2:N_RAYS]
    for flags in PACKET_FLAGS:
        o = H.TraceOpts(0, 0, 0, 1, 0, 0, 0, flags)
        per_lane = H.TraceOpts(64, 2, 0, 1, 32, 64, 0, flags & ~32)
        got = H.trace(bvh, rd, perm, opts=o).cpu().numpy()
        base = H.trace(bvh, rd, perm, opts=per_lane).cpu().numpy()
        assert_no_worse_closest(got, ref_c.raw, rays, tris, max_rate=None)
        assert_no_worse_closest(got, base, rays, tris, max_rate=None)
        assert_closest(got, ref_c, rays, tris, idx=rest)
        occ = H.trace(bvh, rd, perm, closest=False, opts=o).cpu().numpy()
        base_a = H.trace(bvh, rd, perm, closest=False, opts=per_lane).cpu().numpy()
        assert_no_fewer_any(occ, base_a, upper=bf_a, max_rate=None)
        assert_any(occ, ref_a, idx=rest)
