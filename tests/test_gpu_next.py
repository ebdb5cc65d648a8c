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


@pytest.mark.parametrize("top,low", [(8, 8), (16, 16), (4, 32), (30, 2), (1, 64), (64, 32), (32, 32), (40, 24)])
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
    rays = tiny["rays"]
    if t_eff + low > kb:
        # the cut is valid, but its top bits and low bits cannot share one 64-bit key
        with pytest.raises(H.HCCError):
            H.encode(tiny["bvh"], cut, H.KEY_MLHCC, kb, torch.from_numpy(rays).cuda())
        return
    # (32, 32): 1,024 low-level boxes staged in LDS, the most a 64-bit key can use
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


@pytest.mark.parametrize("key_bits", [1, 7, 16, 32, 33, 64])
def test_ppc_keys_bit_exact(H, tiny, key_bits):
    rays = tiny["rays"]
    keys = H.encode(tiny["bvh"], None, H.KEY_PPC, key_bits, torch.from_numpy(rays).cuda())
    assert np.array_equal(_keys(keys, key_bits), O.encode_ppc(tiny["ob"], rays, key_bits))


def test_ppc_one_and_two_triangles(H):
    rng = np.random.default_rng(8)
    for n in (1, 2):
        tris = (rng.random((n, 9)) * 0.5 + 0.25).astype(np.float32)
        ob = O.build_bvh(tris)
        bvh = H.build_bvh(torch.from_numpy(tris).cuda())
        o = rng.random((300, 3)).astype(np.float32)
        d = (0.5 - o) + 0.2 * (rng.random((300, 3)) - 0.5)
        rays = np.concatenate([o, np.zeros((300, 1)), d, np.full((300, 1), np.inf)], 1).astype(np.float32)
        for kb in (1, 5, 40):
            keys = H.encode(bvh, None, H.KEY_PPC, kb, torch.from_numpy(rays).cuda())
            ref = O.encode_ppc(ob, rays, kb)
            assert np.array_equal(_keys(keys, kb), ref)
            assert ref.any()


@pytest.mark.parametrize("n", [1, 255, 4096, 4097, 70001])
@pytest.mark.parametrize("key_bits,skip", [(32, 8), (32, 16), (32, 31), (20, 3), (64, 24), (48, 40)])
def test_prefix_sort_bit_exact(H, n, key_bits, skip):
    rng = np.random.default_rng(n + key_bits + skip)
    hi = np.uint64((1 << key_bits) - 1)
    raw = rng.integers(0, 1 << 62, n, dtype=np.uint64) & hi
    raw[: n // 3] &= ~np.uint64((1 << (skip + 2)) - 1) & hi       # many equal prefixes
    keys = torch.from_numpy(raw.astype(np.uint32).view(np.int32) if key_bits <= 32 else raw.view(np.int64)).cuda()
    sk = torch.empty_like(keys)
    perm = H.sort_ex(keys, key_bits, skip_bits=skip, sorted_keys=sk)
    ref = O.sort_prefix(raw, key_bits, skip)
    assert np.array_equal(perm.cpu().numpy().view(np.uint32), ref)
    assert np.array_equal(_keys(sk, key_bits), raw[ref].astype(np.uint32 if key_bits <= 32 else np.uint64))
    # without sorted keys out (packed late passes)
    assert np.array_equal(H.sort_ex(keys, key_bits, skip_bits=skip).cpu().numpy().view(np.uint32), ref)


@pytest.mark.parametrize("tile", [256, 512, 1024, 2048, 4096])
@pytest.mark.parametrize("n", [1, 300, 4096, 10000])
@pytest.mark.parametrize("key_bits,skip", [(32, 0), (16, 4), (64, 0), (64, 32)])
def test_tile_sort_bit_exact(H, tile, n, key_bits, skip):
    rng = np.random.default_rng(tile + n + key_bits)
    raw = rng.integers(0, 1 << 62, n, dtype=np.uint64) & np.uint64((1 << key_bits) - 1)
    raw[::5] = raw[0]                                                    # repeated keys
    raw[1::7] = np.uint64((1 << key_bits) - 1)                           # the largest key, as the padding
    keys = torch.from_numpy(raw.astype(np.uint32).view(np.int32) if key_bits <= 32 else raw.view(np.int64)).cuda()
    sk = torch.empty_like(keys)
    perm = H.sort_ex(keys, key_bits, skip_bits=skip, tile=tile, sorted_keys=sk)
    ref = O.sort_tiles(raw >> np.uint64(skip), tile)
    assert np.array_equal(perm.cpu().numpy().view(np.uint32), ref)
    assert np.array_equal(_keys(sk, key_bits), raw[ref].astype(np.uint32 if key_bits <= 32 else np.uint64))


def test_sort_ex_rejects_bad_arguments(H):
    keys = torch.zeros(10, dtype=torch.int32, device="cuda")
    for kw in (dict(skip_bits=32), dict(tile=100), dict(tile=8192), dict(tile=3000)):
        with pytest.raises(H.HCCError):
            H.sort_ex(keys, 32, **kw)
