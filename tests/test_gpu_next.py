"""GPU parity of the multi-level hierarchy cut code (two-level cut + MLHCC keys) and of the
regular-grid control encoding against the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    assert torch.cuda.is_available()
    import paper_2305_16652_amd as H
    return H


@pytest.fixture(scope="module")
def tiny(H):
    spec = W.tiny_scene()
    ob = O.build_bvh(spec.tris)
    prim = W.pinhole_rays(spec, 64, 64)
    ph = O.trace(ob, prim)
    sec, _ = W.spawn_diffuse(prim, ph.t, ph.prim, spec.tris, seed=2, bounce=0)
    shd, _ = W.spawn_shadow(prim, ph.t, ph.prim, spec.tris, spec.lights)
    bvh = H.build_bvh(torch.from_numpy(spec.tris).cuda())
    return dict(spec=spec, ob=ob, had=O.had(ob), bvh=bvh, rays=np.concatenate([sec, shd, prim]))


def _keys(t, kb):
    a = t.cpu().numpy()
    return a.view(np.uint32) if kb <= 32 else a.view(np.uint64)


@pytest.mark.parametrize("top,low", [(8, 8), (16, 16), (4, 32), (30, 2), (1, 64), (64, 32)])
def test_mlhcc_cut_and_keys_bit_exact(H, tiny, top, low):
    cut = H.select_mlhcc_cut(tiny["bvh"], top, low)
    kind, t_eff, l = H.cut_shape(cut)
    rt, rl = O.select_mlhcc_cut(tiny["ob"], tiny["had"], top, low)
    assert kind == 1 and l == low and t_eff == rt.size
    ids, had, boxes = cut.export()
    assert np.array_equal(ids, rt) and np.array_equal(boxes, tiny["ob"].boxes[rt])
    low_ids, low_boxes = H.cut_export_low(cut)
    assert np.array_equal(low_ids, rl)
    assert np.array_equal(low_boxes.reshape(-1, 6), tiny["ob"].boxes[rl.reshape(-1)])
    kb = min(64, top + low)
    if t_eff + low > kb:
        pytest.skip("key too short for this cut")
    rays = tiny["rays"]
    keys = H.encode(tiny["bvh"], cut, H.KEY_MLHCC, kb, torch.from_numpy(rays).cuda())
    ref = O.encode_mlhcc(rays, tiny["ob"].boxes[rt], tiny["ob"].boxes[rl.reshape(-1)], low, kb)
    assert np.array_equal(_keys(keys, kb), ref)


@pytest.mark.parametrize("key_bits", [16, 24, 32, 48, 64])
def test_grid_keys_bit_exact(H, tiny, key_bits):
    gx, gy, gz = O.grid_dims(key_bits)
    cut = H.grid_cut(tiny["bvh"], gx, gy, gz)
    kind, cells, _ = H.cut_shape(cut)
    assert kind == 2 and cells == key_bits
    ref_boxes = O.grid_boxes(O.scene_box(tiny["spec"].tris), gx, gy, gz)
    assert np.array_equal(cut.export()[2], ref_boxes)
    rays = tiny["rays"]
    keys = H.encode(tiny["bvh"], cut, H.KEY_HCC, key_bits, torch.from_numpy(rays).cuda())
    assert np.array_equal(_keys(keys, key_bits), O.encode_hcc(rays, ref_boxes, key_bits))


def test_mode_and_cut_kind_must_match(H, tiny):
    rays = torch.from_numpy(tiny["rays"][:100]).cuda()
    ml = H.select_mlhcc_cut(tiny["bvh"], 8, 8)
    with pytest.raises(H.HCCError):
        H.encode(tiny["bvh"], ml, H.KEY_HCC, 32, rays)
    with pytest.raises(H.HCCError):
        H.encode(tiny["bvh"], H.select_cut(tiny["bvh"], 32), H.KEY_MLHCC, 32, rays)
    with pytest.raises(H.HCCError):
        H.encode(tiny["bvh"], ml, H.KEY_MLHCC, 8, rays)          # 8 top + 8 low bits do not fit in 8
    with pytest.raises(H.HCCError):
        H.select_mlhcc_cut(tiny["bvh"], 64, 64)                  # more than 2048 low-level boxes
    with pytest.raises(H.HCCError):
        H.grid_cut(tiny["bvh"], 8, 8, 2)
