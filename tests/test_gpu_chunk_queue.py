"""Persistent trace launches that deal out their chunks through the per-stream device counter:
launches of changing sizes and launch shapes back to back on one stream (the counter must read
zero at each launch's start), launches overlapping on two streams (each stream its own slot),
and a launch captured into a graph (the static chunk order) replayed between eager launches.
Every result is checked against the oracle, or against the same rays traced eagerly."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from parity_utils import assert_any, assert_closest

pytestmark = pytest.mark.gpu

# (block, stack, xcd_remap, persistent, refill, chunk, waves, flags)
WIDE = (64, 2, 0, 1, 32, 64, 0, 2)
BVH2 = (64, 0, 0, 1, 32, 64, 0, 0)
WIDE_SPREAD = (64, 2, 0, 1, 32, 64, 0, 2 | 8)     # chunks dealt spread over the order
BVH2_SPREAD = (64, 0, 0, 1, 32, 64, 0, 8)
PACKET = (0, 0, 0, 1, 0, 0, 0, 2 | 32)           # wavefront packets (chunks of 64 rays)
PACKET_SPREAD = (0, 0, 0, 1, 0, 0, 0, 2 | 16 | 8 | 32)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


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
    shd, _ = W.spawn_shadow(prim, ph.t, ph.prim, spec.tris, spec.lights)
    bvh = H.build_bvh(torch.from_numpy(spec.tris).cuda())
    torch.cuda.synchronize()
    return dict(spec=spec, sec=sec, shd=shd, bvh=bvh, ref_sec=O.trace(ob, sec), ref_shd=O.trace(ob, shd, closest=False))


def _opts(H, base, chunk, waves):
    return H.TraceOpts(*base[:5], chunk, waves, base[7])


@pytest.mark.parametrize("base", [WIDE, BVH2, WIDE_SPREAD, BVH2_SPREAD, PACKET, PACKET_SPREAD],
                         ids=["wide", "bvh2", "wide-spread", "bvh2-spread", "packet", "packet-spread"])
def test_back_to_back_launches_of_changing_shape(H, tiny, base):
    sec, shd = torch.from_numpy(tiny["sec"]).cuda(), torch.from_numpy(tiny["shd"]).cuda()
    n = sec.shape[0]
    # sizes and launch shapes change from launch to launch with no synchronisation between them:
    # more wavefronts than chunks, fewer, one; a ragged last chunk; a single ray
    plan = [(n, 64, 0), (1000, 64, 3), (n, 128, 1), (65, 64, 8192), (1, 64, 0), (n, 256, 5), (n - 7, 64, 16)]
    outs = []
    for m, chunk, waves in plan:
        o = _opts(H, base, chunk, waves)
        outs.append((m, H.trace(tiny["bvh"], sec[:m], opts=o), H.trace(tiny["bvh"], shd[:m], closest=False, opts=o)))
    torch.cuda.synchronize()
    for (m, hits, occ), (_, chunk, waves) in zip(outs, plan):
        _say(f"{base[7]} n={m} chunk={chunk} waves={waves}")
        idx = np.arange(m)      # the launch traced the first m rays
        assert_closest(hits.cpu().numpy(), tiny["ref_sec"], tiny["sec"], tiny["spec"].tris, idx=idx)
        assert_any(occ.cpu().numpy(), tiny["ref_shd"], idx=idx)


def test_spread_and_ordered_dealing_alternate_on_one_stream(H, tiny):
    """Spread and in-order dealing share the stream's counter: alternating them back to back
    (chunk counts that do and do not fill the 64 interleaved streams) gives the same hits."""
    sec = torch.from_numpy(np.tile(tiny["sec"], (3, 1))).cuda()
    n = sec.shape[0]
    want = H.trace(tiny["bvh"], sec, opts=H.TraceOpts(*WIDE)).cpu().numpy()
    outs = []
    for i, (m, chunk) in enumerate([(n, 64), (n, 64), (4096, 64), (n - 1, 128), (200, 64), (n, 256)]):
        base = WIDE_SPREAD if i % 2 == 0 else WIDE
        outs.append((m, H.trace(tiny["bvh"], sec[:m], opts=_opts(H, base, chunk, 0))))
    torch.cuda.synchronize()
    for m, out in outs:
        assert np.array_equal(out.cpu().numpy().view(np.uint32), want[:m].view(np.uint32)), m


def test_overlapping_launches_on_two_streams(H, tiny):
    # 16 copies of the secondary rays, in two orders, traced at the same time on two streams
    rays = torch.from_numpy(np.tile(tiny["sec"], (16, 1))).cuda()
    n = rays.shape[0]
    rev = torch.arange(n - 1, -1, -1, dtype=torch.int32, device="cuda")
    o = H.TraceOpts(*WIDE)
    want = H.trace(tiny["bvh"], rays, opts=o).cpu().numpy()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    outs = []
    for rep in range(3):
        a = torch.empty((n, 4), dtype=torch.float32, device="cuda")
        b = torch.empty((n, 4), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        H.trace(tiny["bvh"], rays, out=a, opts=o, stream=s1)
        H.trace(tiny["bvh"], rays, rev, out=b, opts=o, stream=s2)
        H.trace(tiny["bvh"], rays, out=a, opts=o, stream=s1)
        outs.append((a, b))
    torch.cuda.synchronize()
    for a, b in outs:
        assert np.array_equal(a.cpu().numpy().view(np.uint32), want.view(np.uint32))
        assert np.array_equal(b.cpu().numpy().view(np.uint32), want.view(np.uint32))
    assert_closest(want[: tiny["sec"].shape[0]], tiny["ref_sec"], tiny["sec"], tiny["spec"].tris)


def test_graph_captured_launch_replays(H, tiny):
    rays = torch.from_numpy(tiny["sec"]).cuda()
    n = rays.shape[0]
    o = H.TraceOpts(*WIDE)
    eager = H.trace(tiny["bvh"], rays, opts=o).cpu().numpy()
    out = torch.full((n, 4), -1.0, dtype=torch.float32, device="cuda")
    H.trace(tiny["bvh"], rays, out=out, opts=o)          # warm-up on the current stream
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        H.trace(tiny["bvh"], rays, out=out, opts=o)
    for rep in range(4):
        out.fill_(-1.0)
        g.replay()
        # an eager launch of the same kernel on the same stream between the replays
        other = H.trace(tiny["bvh"], rays, opts=o)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy().view(np.uint32), eager.view(np.uint32)), f"replay {rep}"
        assert np.array_equal(other.cpu().numpy().view(np.uint32), eager.view(np.uint32))


def test_packet_and_per_lane_launches_share_the_counter(H, tiny):
    """Packet launches (chunks of 64 rays) and per-lane launches (chunks of 64-256) alternate back
    to back on one stream, through the stream's one counter slot: each must start from zero."""
    sec = torch.from_numpy(np.tile(tiny["sec"], (3, 1))).cuda()
    n = sec.shape[0]
    want = H.trace(tiny["bvh"], sec, opts=H.TraceOpts(*WIDE)).cpu().numpy()
    plan = [(PACKET, n, 0), (WIDE, n, 0), (PACKET_SPREAD, 4096, 0), (WIDE_SPREAD, n - 1, 0), (PACKET, 65, 3),
            (BVH2, n, 0), (PACKET, n, 1), (WIDE, 200, 0)]
    outs = [(m, H.trace(tiny["bvh"], sec[:m], opts=_opts(H, base, base[5], waves))) for base, m, waves in plan]
    torch.cuda.synchronize()
    for (m, out), (base, _, _) in zip(outs, plan):
        got = out.cpu().numpy()
        if base[7] & 32:
            # packets test a superset of each ray's triangles: the oracle's bar on every ray
            assert_closest(got, O.Hits(np.tile(tiny["ref_sec"].raw, (3, 1))[:m]), np.tile(tiny["sec"], (3, 1))[:m],
                           tiny["spec"].tris)
        else:
            assert np.array_equal(got.view(np.uint32), want[:m].view(np.uint32)), (base, m)


def test_graph_captured_packet_launch_replays(H, tiny):
    shd = torch.from_numpy(tiny["shd"]).cuda()
    n = shd.shape[0]
    o = H.TraceOpts(*PACKET)
    eager = H.trace(tiny["bvh"], shd, closest=False, opts=o).cpu().numpy()
    assert_any(eager, tiny["ref_shd"])
    out = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    H.trace(tiny["bvh"], shd, closest=False, out=out, opts=o)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        H.trace(tiny["bvh"], shd, closest=False, out=out, opts=o)
    for rep in range(4):
        out.fill_(7)
        g.replay()
        other = H.trace(tiny["bvh"], shd, closest=False, opts=o)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), f"replay {rep}"
        assert np.array_equal(other.cpu().numpy(), eager)
