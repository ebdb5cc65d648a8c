"""The autotuner (trace launch options; reordering method's cut size, key length and skipped low
key bits) on the tiny workload: every candidate it times is a correct launch, and whatever it
picks reproduces the oracle's keys, shortened-sort permutation and hits."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from parity_utils import assert_closest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2305_16652_amd as H
    return H


@pytest.fixture(scope="module")
def tiny(H):
    spec = W.tiny_scene()
    ob = O.build_bvh(spec.tris)
    prim = W.pinhole_rays(spec, 64, 64)
    ph = O.trace(ob, prim)
    sec, _ = W.spawn_diffuse(prim, ph.t, ph.prim, spec.tris, seed=2, bounce=0)
    bvh = H.build_bvh(torch.from_numpy(spec.tris).cuda())
    return dict(spec=spec, ob=ob, sec=sec, rays=torch.from_numpy(sec).cuda(), bvh=bvh, ref=O.trace(ob, sec))


def test_every_trace_candidate_gives_the_oracle_hits(H, tiny):
    from paper_2305_16652_amd import autotune as AT
    best, ms, table = AT.tune_trace(tiny["bvh"], tiny["rays"], None, reps=1)
    assert len(table) == len(AT.DEFAULT_CANDIDATES) and ms > 0
    # the 4-wide candidates cover both child-box tests, with chunks dealt in order and spread
    assert {o.flags for o in AT.WIDE} == {H.TRACE_WIDE | s | q | sp for s in (0, H.TRACE_SLAB)
                                          for q in (0, H.TRACE_QUANT) for sp in (0, H.TRACE_SPREAD)}
    assert {o.flags for o in AT.PACKET} == {H.TRACE_WIDE | H.TRACE_PACKET | q | sp for q in (0, H.TRACE_QUANT)
                                            for sp in (0, H.TRACE_SPREAD)}
    for o in AT.DEFAULT_CANDIDATES + [best]:
        hits = H.trace(tiny["bvh"], tiny["rays"], opts=o).cpu().numpy()
        assert_closest(hits, tiny["ref"], tiny["sec"], tiny["spec"].tris)


@pytest.mark.parametrize("mode", ["hcc", "twopoint"])
def test_reorder_choice_reproduces_the_oracle(H, tiny, mode):
    from paper_2305_16652_amd import autotune as AT
    ch, results = AT.tune_reorder(tiny["bvh"], tiny["rays"], mode, cuts=(16, 64), key_bits=(16, 32),
                                  paper_exact=False, skips=(0, 8), reps=1, candidates=AT.WIDE[:2])
    # every (C >= K, skip < K) combination was timed, and the pick is the fastest of them
    if mode == "hcc":
        assert sorted((r.cut, r.key_bits, r.skip) for r in results) == [
            (16, 16, 0), (16, 16, 8), (64, 16, 0), (64, 16, 8), (64, 32, 0), (64, 32, 8)]
    else:
        assert sorted((r.key_bits, r.skip) for r in results) == [(16, 0), (16, 8), (32, 0), (32, 8)]
    assert ch.total_ms == min(r.total_ms for r in results)
    assert ch.as_dict()["skip"] == ch.skip
    # the picked configuration, run through the library, against the oracle step by step
    k = ch.key_bits
    if mode == "hcc":
        cut = H.select_cut(tiny["bvh"], ch.cut)
        keys = H.encode(tiny["bvh"], cut, H.KEY_HCC, k, tiny["rays"])
        ob = tiny["ob"]
        ref_keys = O.encode_hcc(tiny["sec"], O.cut_boxes(ob, O.select_cut(ob, O.had(ob), ch.cut)), k)
    else:
        keys = H.encode(tiny["bvh"], None, H.KEY_TWOPOINT, k, tiny["rays"])
        ref_keys = O.encode_twopoint(tiny["sec"], O.scene_box(tiny["spec"].tris), k)
    assert np.array_equal(keys.cpu().numpy().view(np.uint32), ref_keys)
    perm = H.sort_ex(keys, k, ch.skip)
    assert np.array_equal(perm.cpu().numpy().view(np.uint32), O.sort_prefix(ref_keys, k, ch.skip))
    hits = H.trace(tiny["bvh"], tiny["rays"], perm, opts=ch.opts).cpu().numpy()
    assert_closest(hits, tiny["ref"], tiny["sec"], tiny["spec"].tris)
