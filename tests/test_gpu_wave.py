"""The trace kernel's own fetch counters against the oracle's lockstep wave model.

hcc_trace_stats runs the one-ray-per-lane BVH2 kernel (64-lane wavefronts over consecutive
trace positions, child-test traversal) and counts, per wavefront and lockstep iteration, the
distinct nodes and triangles its lanes fetch.  The oracle's wave model with the child-test
order and waves of 64 describes exactly that, so the per-wavefront counts must agree exactly,
and so must the per-ray step and triangle-test counts (the model with one ray per wave)."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    import paper_2305_16652_amd as H
    return H


def _scene_rays(spec, w, h, seed):
    ob = O.build_bvh(spec.tris)
    prim = W.pinhole_rays(spec, w, h, 1, seed=seed)
    ph = O.trace(ob, prim, threads=8)
    sec, _ = W.spawn_diffuse(prim, ph.t, ph.prim, spec.tris, seed=seed + 1, bounce=0)
    shd, _ = W.spawn_shadow(prim, ph.t, ph.prim, spec.tris, spec.lights)
    return ob, sec, shd


def _orders(ob, rays, n_cut=32):
    """NoSort, HCC (C = K = 32) and TwoPoint (K = 32) trace orders, all from the oracle."""
    cb = O.cut_boxes(ob, O.select_cut(ob, O.had(ob), n_cut))
    hcc = O.sort(O.encode_hcc(rays, cb, 32, threads=8))
    tp = O.sort(O.encode_twopoint(rays, O.scene_box(ob.tris), 32, threads=8))
    return {"nosort": None, "hcc": hcc, "twopoint": tp}


def _check(H, ob, rays, closest, label):
    bvh = H.build_bvh(torch.from_numpy(ob.tris).cuda())
    rd = torch.from_numpy(rays).cuda()
    for name, perm in _orders(ob, rays).items():
        pd = None if perm is None else torch.from_numpy(perm.view(np.int32)).cuda()
        _, nodes, tris, wn, wt = H.trace_stats(bvh, rd, pd, closest=closest)
        torch.cuda.synchronize()
        mn, mt, _ = O.wave_fetches(ob, rays, perm, 64, closest, order=1, threads=8)
        assert np.array_equal(wn.cpu().numpy().astype(np.uint64), mn), f"{label} {name}: wave node fetches"
        assert np.array_equal(wt.cpu().numpy().astype(np.uint64), mt), f"{label} {name}: wave triangle fetches"
        # per ray (one ray per wave, in any order) the kernel's iteration and test counts
        rn, rt, _ = O.wave_fetches(ob, rays, None, 1, closest, order=1, threads=8)
        assert np.array_equal(nodes.cpu().numpy().astype(np.uint64), rn), f"{label} {name}: per-ray steps"
        assert np.array_equal(tris.cpu().numpy().astype(np.uint64), rt), f"{label} {name}: per-ray tests"


def test_wave_counts_tiny(H):
    spec = W.tiny_scene()
    ob, sec, shd = _scene_rays(spec, 64, 64, 2)
    _check(H, ob, sec, True, "tiny secondary")
    _check(H, ob, shd, False, "tiny shadow")


def test_wave_counts_cluster_ragged(H):
    spec = W.cluster_scene(100_000, seed=41)
    ob, sec, shd = _scene_rays(spec, 256, 128, 12)
    n = sec.shape[0] - 37          # a ragged last wavefront
    _check(H, ob, np.ascontiguousarray(sec[:n]), True, "cluster secondary")
    _check(H, ob, np.ascontiguousarray(shd[: shd.shape[0] - 5]), False, "cluster shadow")
