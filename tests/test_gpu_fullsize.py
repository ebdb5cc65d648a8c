"""Full-size parity on the benchmark's workload (frame scene, 1,012,012 triangles, 1920x1080x8
primary rays, bounce-1 secondary rays) in the launch configuration bench.py times.

Every primary hit and every key is compared; the permutation is checked by the properties that
fix a stable sort uniquely; secondary and shadow traces are compared on a deterministic sample
the oracle traces ray by ray.  Secondary rays are spawned from the oracle's primary hits.
"""
import os
import sys
import time

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from parity_utils import assert_any, assert_closest, assert_no_fewer_any, assert_no_worse_closest, assert_stable_sort

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))
# bench.py's default launch configuration (block, stack, remap, persistent, refill, chunk, waves, flags);
# the autotuner picks among these and the one-ray-per-lane launch, which test_gpu_parity covers
BENCH_OPTS = (64, 0, 0, 1, 32, 64, 8192, 1)
WIDE_OPTS = (64, 2, 0, 1, 32, 64, 8192, 2)        # the 4-wide traversal, LDS short stack (bench's pick)


def WIDE_FLAGS(H):
    """4-wide variants checked against each other: child test, quantised nodes, spread dealing
    (the exact nodes give the same hits bit for bit; the quantised ones test a superset of the
    boxes, see assert_no_worse_closest)."""
    w, q = H.TRACE_WIDE, H.TRACE_QUANT
    return (w, w | H.TRACE_SLAB, w | q, w | q | H.TRACE_SLAB, w | q | H.TRACE_SPREAD)


def _say(msg):
    print(f"[fullsize {time.strftime('%H:%M:%S')}] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def frame():
    import paper_2305_16652_amd as H
    assert torch.cuda.is_available()
    spec = W.frame_scene()
    _say(f"frame scene {spec.tris.shape[0]} triangles")
    ob = O.build_bvh(spec.tris)
    had = O.had(ob)
    bvh = H.build_bvh(torch.from_numpy(spec.tris).cuda())
    prim = W.pinhole_rays(spec, 1920, 1080, 8, seed=2)
    _say(f"{prim.shape[0]} primary rays; oracle trace with {THREADS} threads")
    ph = O.trace(ob, prim, threads=THREADS)
    sec, _ = W.spawn_diffuse(prim, ph.t, ph.prim, spec.tris, seed=7, bounce=0)
    shd, _ = W.spawn_shadow(prim, ph.t, ph.prim, spec.tris, spec.lights)
    _say(f"{sec.shape[0]} secondary, {shd.shape[0]} shadow rays")
    return dict(H=H, spec=spec, ob=ob, had=had, bvh=bvh, prim=prim, ph=ph, sec=sec, shd=shd)


def _opts(H):
    return H.TraceOpts(*BENCH_OPTS)


def test_fullsize_bvh_and_cut(frame):
    H, ob, had, bvh = frame["H"], frame["ob"], frame["had"], frame["bvh"]
    child, leaf, boxes, ghad = bvh.export()
    assert np.array_equal(leaf, ob.leaf_prim)
    assert np.array_equal(child, ob.child)
    assert np.array_equal(boxes.view(np.uint32), ob.boxes.view(np.uint32))
    assert np.array_equal(ghad.view(np.uint64), had.view(np.uint64))
    for c in (32, 64, 1024, 4096):
        assert np.array_equal(H.select_cut(bvh, c).export()[0], O.select_cut(ob, had, c))


# wavefront packets on the exact and the quantised nodes (bench.py's packet candidates)
PACKET_OPTS = [(0, 0, 0, 1, 0, 0, 8192, 2 | 32), (0, 0, 0, 1, 0, 0, 8192, 2 | 16 | 8 | 32)]


@pytest.mark.parametrize("opts", [BENCH_OPTS, WIDE_OPTS] + PACKET_OPTS)
def test_fullsize_primary_hits_all_rays(frame, opts):
    H = frame["H"]
    hits = H.trace(frame["bvh"], torch.from_numpy(frame["prim"]).cuda(), opts=H.TraceOpts(*opts)).cpu().numpy()
    assert_closest(hits, frame["ph"], frame["prim"], frame["spec"].tris)


@pytest.mark.parametrize("cut_size,key_bits", [(32, 32), (64, 64)])
def test_fullsize_hcc_keys_sort_trace(frame, cut_size, key_bits):
    H, ob, bvh, sec = frame["H"], frame["ob"], frame["bvh"], frame["sec"]
    rays = torch.from_numpy(sec).cuda()
    cut = H.select_cut(bvh, cut_size)
    keys = H.encode(bvh, cut, H.KEY_HCC, key_bits, rays)
    cb = O.cut_boxes(ob, O.select_cut(ob, frame["had"], cut_size))
    ref = O.encode_hcc(sec, cb, key_bits, threads=THREADS)
    k = keys.cpu().numpy()
    k = k.view(np.uint32) if key_bits <= 32 else k.view(np.uint64)
    assert np.array_equal(k, ref)
    _say(f"HCC keys C={cut_size} K={key_bits} equal on {k.size} rays")
    perm = H.sort(keys, key_bits)
    p = perm.cpu().numpy().view(np.uint32)
    assert_stable_sort(ref, p)
    hits = H.trace(bvh, rays, perm, opts=_opts(H)).cpu().numpy()
    sample = np.arange(0, sec.shape[0], 997)
    oh = O.trace(ob, sec, subset=sample, threads=THREADS)
    assert_closest(hits, oh, sec, frame["spec"].tris, idx=sample)
    # the 4-wide traversal returns the same closest hits on every ray, with either child test, on
    # the exact and on the quantised nodes
    for flags in WIDE_FLAGS(H):
        wide = H.trace(bvh, rays, perm, opts=H.TraceOpts(*WIDE_OPTS[:7], flags)).cpu().numpy()
        if flags & H.TRACE_QUANT:
            assert_no_worse_closest(wide, hits, sec, frame["spec"].tris)
        else:
            assert np.array_equal(wide.view(np.uint32), hits.view(np.uint32))


def test_fullsize_twopoint_keys(frame):
    H, bvh, sec = frame["H"], frame["bvh"], frame["sec"]
    rays = torch.from_numpy(sec).cuda()
    keys = H.encode(bvh, None, H.KEY_TWOPOINT, 32, rays).cpu().numpy().view(np.uint32)
    assert np.array_equal(keys, O.encode_twopoint(sec, O.scene_box(frame["spec"].tris), 32, threads=THREADS))


def test_fullsize_shadow_any_hit(frame):
    H, ob, bvh, shd = frame["H"], frame["ob"], frame["bvh"], frame["shd"]
    rays = torch.from_numpy(shd).cuda()
    cut = H.select_cut(bvh, 32)
    perm = H.sort(H.encode(bvh, cut, H.KEY_HCC, 32, rays), 32)
    occ = H.trace(bvh, rays, perm, closest=False, opts=_opts(H)).cpu().numpy()
    sample = np.arange(0, shd.shape[0], 1999)
    ref = O.trace(ob, shd, subset=sample, closest=False, threads=THREADS)
    assert_any(occ, ref, idx=sample)
    for flags in WIDE_FLAGS(H):
        wide = H.trace(bvh, rays, perm, closest=False, opts=H.TraceOpts(*WIDE_OPTS[:7], flags)).cpu().numpy()
        if flags & H.TRACE_QUANT:
            assert_no_fewer_any(wide, occ)
        else:
            assert np.array_equal(wide, occ)
    # packets test a superset of each ray's triangles: never fewer occluded rays than the per-lane
    # launch, in the HCC order and in pixel order
    for o in PACKET_OPTS:
        for p in (perm, None):
            pk = H.trace(bvh, rays, p, closest=False, opts=H.TraceOpts(*o)).cpu().numpy()
            assert_no_fewer_any(pk, occ)
            assert_any(pk, ref, idx=sample)
