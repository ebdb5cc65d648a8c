"""GPU (gfx950) path vs the CPU oracle on the tiny workload and on edge cases.

Every GPU call goes through the C ABI (ctypes binding).  Inputs come from the seeded
workload generators and, for secondary rays, from the oracle's primary hits.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from parity_utils import MISS, assert_any, assert_closest, assert_stable_sort

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def H():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2305_16652_amd as H
    return H


@pytest.fixture(scope="module")
def tiny():
    """Tiny workload: scene, oracle BVH, primary/secondary/shadow rays from oracle hits."""
    spec = W.tiny_scene()
    ob = O.build_bvh(spec.tris)
    prim = W.pinhole_rays(spec, 64, 64)
    ph = O.trace(ob, prim)
    sec, _ = W.spawn_diffuse(prim, ph.t, ph.prim, spec.tris, seed=2, bounce=0)
    shd, _ = W.spawn_shadow(prim, ph.t, ph.prim, spec.tris, spec.lights)
    return dict(spec=spec, ob=ob, had=O.had(ob), primary=prim, primary_hits=ph, secondary=sec, shadow=shd)


@pytest.fixture(scope="module")
def gpu_bvh(H, tiny):
    _say("build tiny BVH on GPU")
    tris = torch.from_numpy(tiny["spec"].tris).cuda()
    b = H.build_bvh(tris)
    torch.cuda.synchronize()
    return b


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _keys_np(t, key_bits):
    a = t.cpu().numpy()
    return a.view(np.uint32) if key_bits <= 32 else a.view(np.uint64)


# ----------------------------------------------------------------------------- BVH, HAD, cut

def test_bvh_bit_exact(gpu_bvh, tiny):
    child, leaf, boxes, had = gpu_bvh.export()
    ob = tiny["ob"]
    assert np.array_equal(leaf, ob.leaf_prim)
    assert np.array_equal(child, ob.child)
    assert np.array_equal(boxes.view(np.uint32), ob.boxes.view(np.uint32))
    assert np.array_equal(had.view(np.uint64), tiny["had"].view(np.uint64))
    assert gpu_bvh.scene_box == O.scene_box(tiny["spec"].tris).tolist()


@pytest.mark.parametrize("cut_size", [1, 2, 7, 32, 64, 500, 2012, 5000])
def test_cut_bit_exact(H, gpu_bvh, tiny, cut_size):
    cut = H.select_cut(gpu_bvh, cut_size)
    ids, had, boxes = cut.export()
    ref = O.select_cut(tiny["ob"], tiny["had"], cut_size)
    assert cut.c_eff == len(ref)
    assert np.array_equal(ids, ref)
    assert np.array_equal(had, tiny["had"][ref])
    assert np.array_equal(boxes, tiny["ob"].boxes[ref])


def test_cut_other_lambda(H, tiny):
    tris = torch.from_numpy(tiny["spec"].tris).cuda()
    b = H.build_bvh(tris)
    for lam in (0.5, 0.0, 0.125):
        cut = H.select_cut(b, 64, lam)
        ids, had, _ = cut.export()
        ref_had = O.had(tiny["ob"], lam)
        assert np.array_equal(ids, O.select_cut(tiny["ob"], ref_had, 64))
        assert np.array_equal(had, ref_had[ids])
        assert np.array_equal(b.export()[3], ref_had)


# ----------------------------------------------------------------------------- keys

@pytest.mark.parametrize("key_bits", [1, 7, 16, 24, 32, 33, 48, 64])
@pytest.mark.parametrize("cut_size", [1, 16, 32, 64, 500])
def test_encode_hcc_bit_exact(H, gpu_bvh, tiny, key_bits, cut_size):
    cut = H.select_cut(gpu_bvh, cut_size)
    ids = O.select_cut(tiny["ob"], tiny["had"], cut_size)
    cb = O.cut_boxes(tiny["ob"], ids)
    for rays in (tiny["secondary"], tiny["shadow"], tiny["primary"]):
        keys = H.encode(gpu_bvh, cut, H.KEY_HCC, key_bits, _dev(rays))
        ref = O.encode_hcc(rays, cb, key_bits)
        assert np.array_equal(_keys_np(keys, key_bits), ref)


@pytest.mark.parametrize("key_bits", [1, 5, 6, 7, 16, 24, 32, 33, 48, 63, 64])
def test_encode_twopoint_bit_exact(H, gpu_bvh, tiny, key_bits):
    lohi = O.scene_box(tiny["spec"].tris)
    for rays in (tiny["secondary"], tiny["shadow"]):
        keys = H.encode(gpu_bvh, None, H.KEY_TWOPOINT, key_bits, _dev(rays))
        assert np.array_equal(_keys_np(keys, key_bits), O.encode_twopoint(rays, lohi, key_bits))


# ----------------------------------------------------------------------------- sort

def _rand_keys(n, key_bits, kind, seed):
    idx = np.arange(n, dtype=np.uint64)
    raw = W.u64_hash(seed, 7, idx)
    if kind == "uniform":
        k = raw >> np.uint64(64 - key_bits)
    elif kind == "few":
        k = (raw % np.uint64(5)) << np.uint64(max(0, key_bits - 3))
        k &= np.uint64((1 << key_bits) - 1) if key_bits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    elif kind == "equal":
        k = np.full(n, (1 << (key_bits - 1)), np.uint64)
    else:  # descending
        k = (np.uint64(n) - idx) & np.uint64((1 << min(key_bits, 63)) - 1)
    return k.astype(np.uint32) if key_bits <= 32 else k


# large sizes at three key widths only
SORT_CASES = [(n, k) for n in (1, 100, 4095, 4096, 4097, 65537, 1_000_003) for k in (1, 8, 9, 16, 30, 32, 33, 64)
              if n <= 100_000 or k in (16, 32, 64)]


@pytest.mark.parametrize("n,key_bits", SORT_CASES)
@pytest.mark.parametrize("kind", ["uniform", "few", "equal", "descending"])
def test_sort_bit_exact(H, n, key_bits, kind):
    keys = _rand_keys(n, key_bits, kind, seed=n + key_bits)
    dt = torch.from_numpy(keys.view(np.int32) if key_bits <= 32 else keys.view(np.int64)).cuda()
    sk = torch.empty_like(dt)
    perm = H.sort(dt, key_bits, sorted_keys=sk)
    p = perm.cpu().numpy().view(np.uint32)
    assert np.array_equal(p, O.sort(keys))
    assert np.array_equal(_keys_np(sk, key_bits), keys[p.astype(np.int64)])
    # without sorted keys out, the late passes move packed (key bits, index) words
    assert np.array_equal(H.sort(dt, key_bits).cpu().numpy().view(np.uint32), p)


@pytest.mark.parametrize("kind", ["few", "uniform"])
def test_sort_unaligned_keys(H, kind):
    """Keys starting 4 bytes past a 16-byte boundary (the histogram reads them one at a time)."""
    n = 70_001
    keys = _rand_keys(n, 32, kind, seed=11)
    buf = torch.from_numpy(np.concatenate([np.zeros(1, np.uint32), keys]).view(np.int32)).cuda()
    dt = buf[1:]
    assert dt.data_ptr() % 16 == 4
    perm = H.sort(dt, 32)
    assert np.array_equal(perm.cpu().numpy().view(np.uint32), O.sort(keys))


def test_sort_hcc_keys_match_oracle(H, gpu_bvh, tiny):
    cut = H.select_cut(gpu_bvh, 64)
    rays = _dev(tiny["secondary"])
    keys = H.encode(gpu_bvh, cut, H.KEY_HCC, 32, rays)
    perm = H.sort(keys, 32)
    ref = O.sort(O.encode_hcc(tiny["secondary"], O.cut_boxes(tiny["ob"], O.select_cut(tiny["ob"], tiny["had"], 64)), 32))
    assert np.array_equal(perm.cpu().numpy().view(np.uint32), ref)


def test_sort_empty(H):
    keys = torch.empty(0, dtype=torch.int32, device="cuda")
    perm = H.sort(keys, 32)
    assert perm.numel() == 0


# ----------------------------------------------------------------------------- trace

# (block, stack, remap, persistent, refill, chunk, waves); stack 0 scratch, 1 LDS, 2 LDS+scratch
OPTS = [(128, 1, 0, 0, 0, 0, 0), (64, 1, 1, 0, 0, 0, 0), (256, 1, 0, 0, 0, 0, 0), (64, 0, 0, 0, 0, 0, 0),
        (128, 0, 1, 0, 0, 0, 0), (256, 2, 0, 0, 0, 0, 0), (128, 2, 1, 0, 0, 0, 0),
        (0, 0, 0, 1, 16, 256, 0), (0, 1, 0, 1, 1, 64, 3), (0, 2, 0, 1, 64, 1000, 7), (0, 0, 0, 1, 33, 4096, 1),
        (0, 0, 0, 1, 32, 64, 0, 1), (0, 2, 0, 1, 5, 128, 11, 1),
        # 4-wide nodes (flags bit 1), with and without the persistent field, odd chunk / refill / waves
        (0, 0, 0, 1, 16, 256, 0, 2), (64, 1, 1, 0, 32, 64, 0, 2), (0, 0, 0, 1, 1, 64, 3, 2),
        (0, 2, 0, 1, 64, 1000, 7, 3), (0, 1, 0, 1, 16, 64, 0, 2), (0, 2, 0, 1, 1, 64, 5, 2),
        # XCD-contiguous chunk order for the persistent and 4-wide kernels
        (0, 2, 1, 1, 32, 64, 0, 2), (0, 0, 1, 1, 16, 256, 13, 1),
        # 4-wide with every child box through the slab test (flags bit 2)
        (0, 2, 0, 1, 32, 64, 0, 6), (0, 0, 1, 1, 16, 256, 9, 6), (0, 1, 0, 1, 1, 64, 3, 6),
        # chunks dealt spread over the order (flags bit 3), BVH2 and 4-wide
        (0, 2, 0, 1, 32, 64, 0, 8 | 2), (0, 0, 0, 1, 16, 256, 5, 8 | 1),
        # quantised 4-wide nodes (flags bit 4): selected planes, slab test, spread dealing, stacks
        (0, 2, 0, 1, 32, 64, 0, 16 | 2), (0, 0, 0, 1, 16, 256, 5, 16 | 2), (0, 1, 0, 1, 1, 64, 3, 16 | 4 | 2),
        (64, 2, 0, 1, 32, 64, 0, 16 | 8 | 2), (0, 2, 1, 1, 24, 128, 7, 16 | 2),
        # wavefront packets (flags bit 5) on the exact and quantised nodes, slab test, spread and
        # XCD-contiguous dealing, few wavefronts
        (0, 0, 0, 1, 0, 0, 0, 32 | 2), (0, 0, 0, 1, 0, 0, 3, 32 | 16 | 2), (0, 0, 0, 1, 0, 0, 0, 32 | 16 | 4 | 2),
        (0, 0, 1, 1, 0, 0, 5, 32 | 16 | 8 | 2), (0, 0, 0, 1, 0, 0, 1, 32 | 4 | 2)]
WIDE = (0, 0, 0, 1, 32, 64, 0, 2)
PACKET = (0, 0, 0, 1, 0, 0, 0, 32 | 2)
PACKET_Q = (0, 0, 0, 1, 0, 0, 0, 32 | 16 | 2)


@pytest.mark.parametrize("opt", OPTS)
def test_trace_closest(H, gpu_bvh, tiny, opt):
    o = H.TraceOpts(*opt)
    block, stack = opt[0], opt[1]
    tris = tiny["spec"].tris
    for name in ("primary", "secondary"):
        rays = tiny[name]
        ref = O.trace(tiny["ob"], rays)
        hits = H.trace(gpu_bvh, _dev(rays), opts=o).cpu().numpy()
        assert_closest(hits, ref, rays, tris)
        # reordered by the HCC permutation: same answers at the original indices
        perm = np.random.default_rng(block + stack).permutation(rays.shape[0]).astype(np.uint32)
        hits_p = H.trace(gpu_bvh, _dev(rays), perm=_dev(perm.view(np.int32)), opts=o).cpu().numpy()
        assert np.array_equal(hits_p.view(np.uint32), hits.view(np.uint32))


@pytest.mark.parametrize("opt", OPTS)
def test_trace_any(H, gpu_bvh, tiny, opt):
    o = H.TraceOpts(*opt)
    rays = tiny["shadow"]
    ref = O.trace(tiny["ob"], rays, closest=False)
    occ = H.trace(gpu_bvh, _dev(rays), closest=False, opts=o).cpu().numpy()
    assert_any(occ, ref)
    assert 0.05 < ref.mean() < 0.95
    sec = tiny["secondary"]
    assert_any(H.trace(gpu_bvh, _dev(sec), closest=False, opts=o).cpu().numpy(), O.trace(tiny["ob"], sec, closest=False))


def test_trace_stats_same_results(H, gpu_bvh, tiny):
    rays = tiny["secondary"]
    d = _dev(rays)
    hits = H.trace(gpu_bvh, d).cpu().numpy()
    out, nodes, ntri, wn, wt = H.trace_stats(gpu_bvh, d)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), hits.view(np.uint32))
    nodes = nodes.cpu().numpy()
    ntri = ntri.cpu().numpy()
    wn = wn.cpu().numpy()
    wt = wt.cpu().numpy()
    assert (nodes >= 1).all()
    assert wn.shape[0] == (rays.shape[0] + 63) // 64
    # per wavefront, distinct fetches are at most the lanes' total and at least the busiest lane's count
    for w in range(wn.shape[0]):
        lanes = slice(64 * w, 64 * (w + 1))
        assert nodes[lanes].max() <= wn[w] <= nodes[lanes].sum()
        assert wt[w] <= ntri[lanes].sum()
    occ, n2, t2, _, _ = H.trace_stats(gpu_bvh, _dev(tiny["shadow"]), closest=False)
    assert_any(occ.cpu().numpy(), O.trace(tiny["ob"], tiny["shadow"], closest=False))


@pytest.mark.parametrize("opt", [(0, 0, 0, 1, 32, 64, 0, 1), (0, 0, 0, 1, 16, 256, 0, 0), WIDE,
                                 (0, 0, 0, 1, 1, 64, 5, 2)])
def test_trace_count_same_results(H, gpu_bvh, tiny, opt):
    o = H.TraceOpts(*opt)
    for name, closest in (("secondary", True), ("shadow", False)):
        d = _dev(tiny[name])
        n = d.shape[0]
        plain = H.trace(gpu_bvh, d, closest=closest, opts=o).cpu().numpy()
        out, nodes, tris = H.trace_count(gpu_bvh, d, closest=closest, opts=o)
        assert np.array_equal(out.cpu().numpy().view(np.uint8), plain.view(np.uint8))
        again = H.trace_count(gpu_bvh, d, closest=closest, opts=o)
        assert (nodes, tris) == again[1:]                 # static chunk assignment: deterministic counts
        assert n / 64 <= nodes and 0 < tris <= nodes * 64 * 4
    with pytest.raises(H.HCCError):
        H.trace_count(gpu_bvh, _dev(tiny["secondary"]), opts=H.TraceOpts(64, 0, 0, 0, 0, 0, 0, 0))


# ----------------------------------------------------------------------------- edge cases

def test_single_and_two_triangle_scenes(H):
    for tris in (np.array([[0, 0, 1, 1, 0, 1, 0, 1, 1]], np.float32),
                 np.array([[0, 0, 1, 1, 0, 1, 0, 1, 1], [0, 0, 2, 1, 0, 2, 0, 1, 2]], np.float32)):
        ob = O.build_bvh(tris)
        b = H.build_bvh(_dev(tris))
        child, leaf, boxes, had = b.export()
        assert np.array_equal(child, ob.child) and np.array_equal(leaf, ob.leaf_prim)
        assert np.array_equal(boxes, ob.boxes) and np.array_equal(had, O.had(ob))
        for c in (1, 2, 5):
            assert np.array_equal(H.select_cut(b, c).export()[0], O.select_cut(ob, O.had(ob), c))
        rays = np.array([[0.2, 0.2, 0, 0, 0, 0, 1, np.inf], [2, 2, 0, 0, 0, 0, 1, np.inf],
                         [0.2, 0.2, 0, 1.5, 0, 0, 1, np.inf], [0.2, 0.2, 0, 0, 0, 0, 1, 0.5]], np.float32)
        for o in (None, H.TraceOpts(*WIDE), H.TraceOpts(*PACKET), H.TraceOpts(*PACKET_Q)):
            hits = H.trace(b, _dev(rays), opts=o).cpu().numpy()
            assert_closest(hits, O.trace(ob, rays), rays, tris)
            assert_any(H.trace(b, _dev(rays), closest=False, opts=o).cpu().numpy(), O.trace(ob, rays, closest=False))


def test_degenerate_rays(H, gpu_bvh, tiny):
    rng = np.random.default_rng(5)
    n = 3000
    rays = np.zeros((n, 8), np.float32)
    rays[:, 0:3] = rng.uniform(-0.1, 1.1, (n, 3))
    d = rng.normal(size=(n, 3))
    d[0::5, 0] = 0.0             # axis-parallel components, both zero signs
    d[1::5, 1] = -0.0
    d[2::5, 0:2] = 0.0
    rays[:, 4:7] = d
    rays[:, 3] = 0.0
    rays[:, 7] = np.inf
    rays[3::7, 3] = 5.0          # empty segments (tmin > tmax)
    rays[3::7, 7] = 1.0
    rays[4::7, 7] = 0.0          # zero-length segments
    rays[5::11, 4:7] = 0.0       # zero direction
    tris = tiny["spec"].tris
    for o in (None, H.TraceOpts(*WIDE), H.TraceOpts(*WIDE[:7], H.TRACE_WIDE | H.TRACE_SLAB),
              H.TraceOpts(0, 0, 0, 1, 32, 64, 0, 1), H.TraceOpts(*PACKET), H.TraceOpts(*PACKET_Q)):
        assert_closest(H.trace(gpu_bvh, _dev(rays), opts=o).cpu().numpy(), O.trace(tiny["ob"], rays), rays, tris)
        assert_any(H.trace(gpu_bvh, _dev(rays), closest=False, opts=o).cpu().numpy(),
                   O.trace(tiny["ob"], rays, closest=False))
    cut = H.select_cut(gpu_bvh, 64)
    cb = O.cut_boxes(tiny["ob"], O.select_cut(tiny["ob"], tiny["had"], 64))
    for kb in (32, 64):
        assert np.array_equal(_keys_np(H.encode(gpu_bvh, cut, H.KEY_HCC, kb, _dev(rays)), kb),
                              O.encode_hcc(rays, cb, kb))
        assert np.array_equal(_keys_np(H.encode(gpu_bvh, None, H.KEY_TWOPOINT, kb, _dev(rays)), kb),
                              O.encode_twopoint(rays, O.scene_box(tris), kb))


def test_nonfinite_origins(H, gpu_bvh, tiny):
    """Rays with an infinite or NaN origin component, in the same wavefronts as ordinary rays:
    the 4-wide kernels must give them the slab test (whose NaN handling the oracle shares), while
    the ordinary rays around them keep the selected-plane child test."""
    rays = tiny["secondary"][:2048].copy()
    rays[7::64, 0] = np.nan
    rays[21::64, 1] = np.inf
    rays[40::64, 2] = -np.inf
    tris = tiny["spec"].tris
    for o in (None, H.TraceOpts(*WIDE), H.TraceOpts(64, 2, 0, 1, 32, 64, 0, H.TRACE_WIDE), H.TraceOpts(*PACKET_Q)):
        assert_closest(H.trace(gpu_bvh, _dev(rays), opts=o).cpu().numpy(), O.trace(tiny["ob"], rays), rays, tris)
        assert_any(H.trace(gpu_bvh, _dev(rays), closest=False, opts=o).cpu().numpy(),
                   O.trace(tiny["ob"], rays, closest=False))


def test_empty_inputs(H, gpu_bvh):
    empty = torch.empty((0, 8), dtype=torch.float32, device="cuda")
    cut = H.select_cut(gpu_bvh, 8)
    assert H.encode(gpu_bvh, cut, H.KEY_HCC, 32, empty).numel() == 0
    assert H.trace(gpu_bvh, empty).shape == (0, 4)
    assert H.trace(gpu_bvh, empty, closest=False).numel() == 0


def test_invalid_arguments(H, gpu_bvh):
    rays = torch.zeros((4, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(H.HCCError):
        H.encode(gpu_bvh, None, H.KEY_HCC, 32, rays)            # HCC needs a cut
    with pytest.raises(H.HCCError):
        H.encode(gpu_bvh, None, H.KEY_TWOPOINT, 65, rays)
    with pytest.raises(H.HCCError):
        H.select_cut(gpu_bvh, 0)
    with pytest.raises(H.HCCError):
        H.select_cut(gpu_bvh, 8, float("nan"))
    with pytest.raises(H.HCCError):
        H.trace(gpu_bvh, rays, opts=H.TraceOpts(96, 0, 0, 0, 0, 0, 0, 0))
    with pytest.raises(H.HCCError):
        H.trace(gpu_bvh, rays, opts=H.TraceOpts(64, 7, 0, 0, 0, 0, 0, 0))
    with pytest.raises(H.HCCError):
        H.trace(gpu_bvh, rays, opts=H.TraceOpts(0, 0, 0, 1, 32, 64, 0, 64))     # unknown flag bit
    with pytest.raises(H.HCCError):
        H.trace(gpu_bvh, rays, opts=H.TraceOpts(0, 0, 0, 1, 32, 64, 0, 32))     # packets without 4-wide
    with pytest.raises(H.HCCError):
        H.trace_count(gpu_bvh, rays, opts=H.TraceOpts(*PACKET))                 # packets are not counted
    with pytest.raises(H.HCCError):
        H.trace(gpu_bvh, rays, opts=H.TraceOpts(0, 0, 0, 1, 32, 64, 0, 16))     # quantised nodes without 4-wide
    other = H.build_bvh(torch.tensor([[0, 0, 0, 1, 0, 0, 0, 1, 0]], dtype=torch.float32, device="cuda"))
    with pytest.raises(H.HCCError):
        H.encode(gpu_bvh, H.select_cut(other, 1), H.KEY_HCC, 32, rays)   # cut from another BVH
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(H.HCCError):
        H.sort(torch.zeros(1000, dtype=torch.int32, device="cuda"), 32, ws=ws)   # workspace too small


def test_run_to_run_determinism(H, tiny):
    tris = torch.from_numpy(tiny["spec"].tris).cuda()
    rays = _dev(tiny["secondary"])
    outs = []
    for _ in range(2):
        b = H.build_bvh(tris)
        cut = H.select_cut(b, 64)
        k = H.encode(b, cut, H.KEY_HCC, 32, rays)
        p = H.sort(k, 32)
        h = H.trace(b, rays, perm=p)
        outs.append((b.export(), k.cpu().numpy(), p.cpu().numpy(), h.cpu().numpy()))
    (e0, k0, p0, h0), (e1, k1, p1, h1) = outs
    for a, b2 in zip(e0, e1):
        assert np.array_equal(a, b2)
    assert np.array_equal(k0, k1) and np.array_equal(p0, p1) and np.array_equal(h0.view(np.uint32), h1.view(np.uint32))
