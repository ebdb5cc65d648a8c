"""Parity on the boundary-drift workload at its full scene size: 10,000,000 thin triangles in 64
Gaussian clusters inside the unit room (the benchmark's drift scene, seed 90), in the launch
configuration its tuner picks there (4-wide persistent traversal with the slab child test).

The BVH (topology, boxes, HAD) is compared bit for bit; bounce-1 diffuse rays are spawned from the
oracle's hits of every 4th primary ray of the benchmark's 1920x1080x4 camera (about 2.07M rays);
HCC keys (C = K = 16 and 64) and TwoPoint keys (K = 64) are compared on all of them, with their
permutations; primary hits are compared on every traced ray, secondary and shadow hits on a
deterministic sample the oracle traces ray by ray."""
import os
import sys
import time

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from parity_utils import assert_any, assert_closest, assert_no_fewer_any, assert_no_worse_closest

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))
DRIFT_OPTS = (64, 2, 0, 1, 32, 64, 8192, 6)     # 4-wide, LDS short stack, slab child test


def _say(msg):
    print(f"[drift {time.strftime('%H:%M:%S')}] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def drift():
    import paper_2305_16652_amd as H
    assert torch.cuda.is_available()
    spec = W.cluster_scene(10_000_000, seed=90)
    _say(f"drift scene {spec.tris.shape[0]} triangles")
    ob = O.build_bvh(spec.tris)
    had = O.had(ob)
    bvh = H.build_bvh(torch.from_numpy(spec.tris).cuda())
    torch.cuda.synchronize()
    prim = np.ascontiguousarray(W.pinhole_rays(spec, 1920, 1080, 4, seed=91)[::4])
    _say(f"{prim.shape[0]} primary rays; oracle trace with {THREADS} threads")
    ph = O.trace(ob, prim, threads=THREADS)
    sec, _ = W.spawn_diffuse(prim, ph.t, ph.prim, spec.tris, seed=92, bounce=0)
    shd, _ = W.spawn_shadow(prim, ph.t, ph.prim, spec.tris, spec.lights)
    _say(f"{sec.shape[0]} secondary, {shd.shape[0]} shadow rays")
    return dict(H=H, spec=spec, ob=ob, had=had, bvh=bvh, prim=prim, ph=ph, sec=sec, shd=shd)


def test_drift_bvh_bit_exact(drift):
    H, ob, had, bvh = drift["H"], drift["ob"], drift["had"], drift["bvh"]
    child, leaf, boxes, ghad = bvh.export()
    assert np.array_equal(leaf, ob.leaf_prim)
    assert np.array_equal(child, ob.child)
    assert np.array_equal(boxes.view(np.uint32), ob.boxes.view(np.uint32))
    assert np.array_equal(ghad.view(np.uint64), had.view(np.uint64))
    for c in (16, 64, 4096):
        assert np.array_equal(H.select_cut(bvh, c).export()[0], O.select_cut(ob, had, c))
    _say("BVH and cuts equal")


def test_drift_primary_hits_all_rays(drift):
    H = drift["H"]
    hits = H.trace(drift["bvh"], torch.from_numpy(drift["prim"]).cuda(), opts=H.TraceOpts(*DRIFT_OPTS))
    assert_closest(hits.cpu().numpy(), drift["ph"], drift["prim"], drift["spec"].tris)


@pytest.mark.parametrize("mode,key_bits", [("hcc", 16), ("hcc", 64), ("twopoint", 64)])
def test_drift_keys_sort_trace(drift, mode, key_bits):
    H, ob, bvh, sec = drift["H"], drift["ob"], drift["bvh"], drift["sec"]
    rays = torch.from_numpy(sec).cuda()
    if mode == "hcc":
        keys = H.encode(bvh, H.select_cut(bvh, key_bits), H.KEY_HCC, key_bits, rays)
        ref = O.encode_hcc(sec, O.cut_boxes(ob, O.select_cut(ob, drift["had"], key_bits)), key_bits, threads=THREADS)
    else:
        keys = H.encode(bvh, None, H.KEY_TWOPOINT, key_bits, rays)
        ref = O.encode_twopoint(sec, O.scene_box(drift["spec"].tris), key_bits, threads=THREADS)
    k = keys.cpu().numpy()
    assert np.array_equal(k.view(np.uint32) if key_bits <= 32 else k.view(np.uint64), ref)
    perm = H.sort(keys, key_bits)
    ref_perm = O.sort(ref)
    assert np.array_equal(perm.cpu().numpy().view(np.uint32), ref_perm)
    _say(f"{mode} K={key_bits}: keys and permutation equal on {sec.shape[0]} rays")
    hits = H.trace(bvh, rays, perm, opts=H.TraceOpts(*DRIFT_OPTS)).cpu().numpy()
    sample = np.arange(0, sec.shape[0], 97)
    oh = O.trace(ob, sec, subset=sample, threads=THREADS)
    assert_closest(hits, oh, sec, drift["spec"].tris, idx=sample)
    # the selected-plane child test and the quantised nodes return the same hits on every ray
    wide = H.trace(bvh, rays, perm, opts=H.TraceOpts(*DRIFT_OPTS[:7], H.TRACE_WIDE)).cpu().numpy()
    assert np.array_equal(wide.view(np.uint32), hits.view(np.uint32))
    # the quantised nodes test a superset of the boxes: never a farther hit, every other hit real
    for flags in (H.TRACE_WIDE | H.TRACE_QUANT, H.TRACE_WIDE | H.TRACE_QUANT | H.TRACE_SLAB):
        quant = H.trace(bvh, rays, perm, opts=H.TraceOpts(*DRIFT_OPTS[:7], flags)).cpu().numpy()
        assert_no_worse_closest(quant, hits, sec, drift["spec"].tris)


def test_drift_shadow_any_hit(drift):
    H, ob, bvh, shd = drift["H"], drift["ob"], drift["bvh"], drift["shd"]
    rays = torch.from_numpy(shd).cuda()
    perm = H.sort(H.encode(bvh, H.select_cut(bvh, 32), H.KEY_HCC, 32, rays), 32)
    occ = H.trace(bvh, rays, perm, closest=False, opts=H.TraceOpts(*DRIFT_OPTS)).cpu().numpy()
    sample = np.arange(0, shd.shape[0], 199)
    assert_any(occ, O.trace(ob, shd, subset=sample, closest=False, threads=THREADS), idx=sample)
    occ_q = H.trace(bvh, rays, perm, closest=False, opts=H.TraceOpts(*DRIFT_OPTS[:7], DRIFT_OPTS[7] | H.TRACE_QUANT))
    assert_no_fewer_any(occ_q.cpu().numpy(), occ)
