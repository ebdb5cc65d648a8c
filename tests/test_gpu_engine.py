"""Batched engine (one persistent launch over many uneven batches and several resident scenes)
against the oracle and against the plain per-batch path."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from parity_utils import assert_any, assert_closest, assert_no_fewer_any, assert_no_worse_closest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    assert torch.cuda.is_available()
    import paper_2305_16652_amd as H
    return H


@pytest.fixture(scope="module")
def scenes(H):
    """Three resident scenes with oracle BVHs and ray pools (diffuse + shadow) from oracle hits."""
    out = []
    specs = [W.tiny_scene(), W.cluster_scene(20_000, seed=9), W.tiny_scene(seed=3, n_random=1)]
    for si, spec in enumerate(specs):
        ob = O.build_bvh(spec.tris)
        prim = W.pinhole_rays(spec, 96, 96, 1)
        ph = O.trace(ob, prim)
        dif, _ = W.spawn_diffuse(prim, ph.t, ph.prim, spec.tris, seed=11 + si, bounce=0)
        shd, _ = W.spawn_shadow(prim, ph.t, ph.prim, spec.tris, spec.lights)
        bvh = H.build_bvh(torch.from_numpy(spec.tris).cuda())
        out.append(dict(spec=spec, ob=ob, bvh=bvh, cut32=H.select_cut(bvh, 32), cut64=H.select_cut(bvh, 64),
                        diffuse=dif, shadow=shd))
    return out


SIZES = [0, 1, 63, 64, 1023, 1024, 1025, 4097, 9000]
_ORACLE_CUTS = {}


def _oracle_keys(s, mode, key_bits, cut_size, rays):
    """The oracle's keys of a batch (its own cut of the scene for HCC)."""
    ob = s["ob"]
    if mode == "hcc":
        k = (id(ob), cut_size)
        if k not in _ORACLE_CUTS:
            _ORACLE_CUTS[k] = O.cut_boxes(ob, O.select_cut(ob, O.had(ob), cut_size))
        return O.encode_hcc(rays, _ORACLE_CUTS[k], key_bits)
    return O.encode_twopoint(rays, O.scene_box(ob.tris), key_bits)


def check_engine_order(H, items, mode, key_bits, cut_size, ws, opts=None):
    """Every batch's final permutation and sorted keys inside the engine workspace equal the
    oracle's stable sort of the oracle's keys, bit for bit."""
    key_mode = {"hcc": H.KEY_HCC, "twopoint": H.KEY_TWOPOINT}[mode]
    batches = [it[1] for it in items]
    for i, it in enumerate(items):
        s, b = it[0], it[1]
        rays = b.rays.cpu().numpy()
        if rays.shape[0] == 0:
            continue
        perm, keys = H.batch_export(batches, key_mode, key_bits, ws, i, opts=opts)
        ref_keys = _oracle_keys(s, mode, key_bits, cut_size, rays)
        ref_perm = O.sort(ref_keys)
        kd = np.uint32 if key_bits <= 32 else np.uint64
        assert np.array_equal(perm.cpu().numpy().view(np.uint32), ref_perm), f"batch {i}: permutation"
        assert np.array_equal(keys.cpu().numpy().view(kd), ref_keys[ref_perm]), f"batch {i}: sorted keys"


def _batches(H, scenes, seed, key_cut):
    rng = np.random.default_rng(seed)
    res = []
    for i, n in enumerate(SIZES + list(rng.integers(1, 9000, 6))):
        s = scenes[int(rng.integers(0, len(scenes)))]
        closest = bool(rng.random() < 0.7)
        pool = s["diffuse"] if closest else s["shadow"]
        start = int(rng.integers(0, max(1, pool.shape[0] - n))) if pool.shape[0] > n else 0
        sel = np.resize(pool[start:], (n, 8)) if n else np.zeros((0, 8), np.float32)
        rays = torch.from_numpy(np.ascontiguousarray(sel, np.float32)).cuda()
        res.append((s, H.Batch(s["bvh"], rays, closest, cut=s[key_cut] if key_cut else None), sel))
    return res


@pytest.mark.parametrize("mode,key_bits,cut", [("hcc", 32, "cut32"), ("hcc", 64, "cut64"), ("hcc", 16, "cut32"),
                                               ("twopoint", 32, None), ("twopoint", 64, None), ("none", 32, None)])
@pytest.mark.parametrize("opts", [None, (64, 1, 7, 0), (1000, 64, 3, 0), (256, 32, 0, 2), (64, 5, 11, 2),
                                  (128, 24, 0, 6), (256, 32, 0, 2, 0, 3), (64, 9, 13, 6, 0, 1),
                                  # quantised 4-wide nodes (flags bit 4), with each child test and stack
                                  (256, 32, 0, 18), (64, 9, 13, 22, 0, 1), (128, 24, 0, 18, 0, 3)])
def test_engine_matches_oracle_and_plain_path(H, scenes, mode, key_bits, cut, opts):
    key_mode = {"hcc": H.KEY_HCC, "twopoint": H.KEY_TWOPOINT, "none": 0}[mode]
    items = _batches(H, scenes, seed=key_bits + (opts[0] if opts else 0), key_cut=cut if mode == "hcc" else None)
    o = H.BatchOpts(*opts) if opts else None
    ws = H.batch_run([b for _, b, _ in items], key_mode, key_bits, opts=o)
    assert H.batch_check(ws)
    torch.cuda.synchronize()
    if mode != "none":
        check_engine_order(H, items, mode, key_bits, {"cut32": 32, "cut64": 64}.get(cut, 0), ws, o)
    for s, b, rays in items:
        n = rays.shape[0]
        if n == 0:
            continue
        got = b.out.cpu().numpy()
        # the plain path, batch by batch
        perm = None
        if mode != "none":
            keys = H.encode(s["bvh"], b.cut, key_mode, key_bits, b.rays)
            perm = H.sort(keys, key_bits)
        ref_gpu = H.trace(s["bvh"], b.rays, perm, closest=b.closest).cpu().numpy()
        quant = bool(opts and opts[3] & H.TRACE_QUANT)
        if b.closest:
            if quant:   # a superset of the boxes: see assert_no_worse_closest
                assert_no_worse_closest(got, ref_gpu, rays, s["spec"].tris)
            else:
                assert np.array_equal(got.view(np.uint32), ref_gpu.view(np.uint32))
            assert_closest(got, O.trace(s["ob"], rays), rays, s["spec"].tris)
        else:
            if quant:
                assert_no_fewer_any(got, ref_gpu)
            else:
                assert np.array_equal(got, ref_gpu)
            assert_any(got, O.trace(s["ob"], rays, closest=False))


@pytest.mark.parametrize("mode", ["hcc", "twopoint", "none"])
def test_engine_direct_launches_for_large_batches(H, scenes, mode):
    """With direct_min set, batches of that many rays go through the full-device kernels after
    the engine launch of the rest; results are those of the lone path either way."""
    key_mode = {"hcc": H.KEY_HCC, "twopoint": H.KEY_TWOPOINT, "none": 0}[mode]
    rng = np.random.default_rng(11)
    items = []
    for n in (70000, 100, 65536, 65535, 3000, 140000):
        s = scenes[int(rng.integers(0, len(scenes)))]
        closest = bool(rng.random() < 0.7)
        pool = s["diffuse"] if closest else s["shadow"]
        rays = np.ascontiguousarray(np.resize(pool, (n, 8)), np.float32)
        items.append((s, H.Batch(s["bvh"], torch.from_numpy(rays).cuda(), closest,
                                 cut=s["cut32"] if mode == "hcc" else None), rays))
    od = H.BatchOpts(0, 0, 0, 0, 65536)
    ws = H.batch_run([b for _, b, _ in items], key_mode, 32, opts=od)
    assert H.batch_check(ws)
    if mode != "none":   # engine batches and direct launches alike
        check_engine_order(H, items, mode, 32, 32, ws, od)
    big = [b for _, b, _ in items if b.rays.shape[0] >= 65536]
    assert H.batch_check(H.batch_run(big, key_mode, 32, opts=H.BatchOpts(0, 0, 0, 0, 65536)))   # no engine part
    torch.cuda.synchronize()
    for s, b, rays in items:
        perm = None
        if mode != "none":
            perm = H.sort(H.encode(s["bvh"], b.cut, key_mode, 32, b.rays), 32)
        ref = H.trace(s["bvh"], b.rays, perm, closest=b.closest).cpu().numpy()
        assert np.array_equal(b.out.cpu().numpy().view(np.uint8), ref.view(np.uint8))
    with pytest.raises(H.HCCError):
        H.batch_run([b for _, b, _ in items], key_mode, 32, opts=H.BatchOpts(0, 0, 0, 0, 1000))


def test_engine_reuses_workspace_and_is_deterministic(H, scenes):
    items = _batches(H, scenes, seed=5, key_cut="cut32")
    batches = [b for _, b, _ in items]
    ws = H.batch_run(batches, H.KEY_HCC, 32)
    first = [b.out.clone() for b in batches]
    for b in batches:
        b.out.zero_()
    H.batch_run(batches, H.KEY_HCC, 32, ws=ws)
    torch.cuda.synchronize()
    for a, b in zip(first, batches):
        # compare bits: a miss stores prim 0xFFFFFFFF, a NaN pattern in the float view
        if a.dtype == torch.float32:
            assert torch.equal(a.view(torch.int32), b.out.view(torch.int32))
        else:
            assert torch.equal(a, b.out)


def test_engine_invalid_arguments(H, scenes):
    s = scenes[0]
    rays = torch.from_numpy(s["diffuse"][:10]).cuda()
    with pytest.raises(H.HCCError):
        H.batch_run([H.Batch(s["bvh"], rays, True)], H.KEY_HCC, 32)          # HCC without a cut
    with pytest.raises(H.HCCError):
        H.batch_run([H.Batch(s["bvh"], rays, True, cut=scenes[1]["cut32"])], H.KEY_HCC, 32)   # cut of another BVH
    with pytest.raises(H.HCCError):
        H.batch_run([H.Batch(s["bvh"], rays, True)], H.KEY_TWOPOINT, 0)
    with pytest.raises(H.HCCError):
        H.batch_run([H.Batch(s["bvh"], rays, True)], H.KEY_TWOPOINT, 32, opts=H.BatchOpts(0, 0, 0, 1))
    with pytest.raises(H.HCCError):
        H.batch_run([H.Batch(s["bvh"], rays, True)], H.KEY_TWOPOINT, 32, opts=H.BatchOpts(0, 0, 0, 8))
    with pytest.raises(H.HCCError):
        H.batch_run([H.Batch(s["bvh"], rays, True)], H.KEY_TWOPOINT, 32, opts=H.BatchOpts(0, 0, 0, 32))
    with pytest.raises(H.HCCError):
        H.batch_run([H.Batch(s["bvh"], rays, True)], H.KEY_TWOPOINT, 32, opts=H.BatchOpts(0, 0, 0, 2, 0, 4))


@pytest.mark.parametrize("mode,key_bits,cut", [("hcc", 8, "cut32"), ("hcc", 16, "cut32"), ("twopoint", 32, None)])
def test_engine_large_batches_across_phases(H, scenes, mode, key_bits, cut):
    """Batches of hundreds of tiles, so that a batch's encode tiles, each sort pass's tiles and
    its trace chunks run on many wavefronts of every XCD and every phase reads what other
    wavefronts wrote in the launch: results equal the plain path's on every ray (outputs are
    filled with a pattern no result has before each run), on two runs in a row."""
    key_mode = {"hcc": H.KEY_HCC, "twopoint": H.KEY_TWOPOINT}[mode]
    rng = np.random.default_rng(key_bits)
    items = []
    for n in (400_000, 250_000, 1_000, 131_072, 300_001, 64):
        s = scenes[int(rng.integers(0, len(scenes)))]
        closest = bool(rng.random() < 0.7)
        pool = s["diffuse"] if closest else s["shadow"]
        rays = np.ascontiguousarray(np.resize(pool[int(rng.integers(0, 100)):], (n, 8)), np.float32)
        items.append((s, H.Batch(s["bvh"], torch.from_numpy(rays).cuda(), closest,
                                 cut=s[cut] if cut else None)))
    refs = []
    for s, b in items:
        perm = H.sort(H.encode(s["bvh"], b.cut, key_mode, key_bits, b.rays), key_bits)
        refs.append(H.trace(s["bvh"], b.rays, perm, closest=b.closest).cpu().numpy())
    ws = None
    for rep in range(3):
        for _, b in items:
            b.out.fill_(float("nan") if b.out.dtype == torch.float32 else 7)
        # default stack, then the scratch-only and 24-entry LDS stacks of the 4-wide trace phase
        o = H.BatchOpts(256, 32, 0, H.TRACE_WIDE, 0, (0, H.BATCH_STACK_SCRATCH, H.STACK_LDS)[rep])
        ws = H.batch_run([b for _, b in items], key_mode, key_bits, opts=o, ws=ws)
        assert H.batch_check(ws)
        check_engine_order(H, items, mode, key_bits, 32, ws, o)
        for (_, b), ref in zip(items, refs):
            assert np.array_equal(b.out.cpu().numpy().view(np.uint8), ref.view(np.uint8)), f"run {rep}"
