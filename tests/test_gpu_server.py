"""Request server (continuous batching) against the lone per-request path and the oracle,
plus admission, cancellation and shutdown behaviour."""
import time

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from parity_utils import assert_any, assert_closest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    assert torch.cuda.is_available()
    import paper_2305_16652_amd as H
    return H


@pytest.fixture(scope="module")
def scenes(H):
    out = []
    for si, spec in enumerate([W.tiny_scene(), W.cluster_scene(30_000, seed=12)]):
        ob = O.build_bvh(spec.tris)
        prim = W.pinhole_rays(spec, 128, 128, 1)
        ph = O.trace(ob, prim)
        dif, _ = W.spawn_diffuse(prim, ph.t, ph.prim, spec.tris, seed=21 + si, bounce=0)
        shd, _ = W.spawn_shadow(prim, ph.t, ph.prim, spec.tris, spec.lights)
        bvh = H.build_bvh(torch.from_numpy(spec.tris).cuda())
        out.append(dict(spec=spec, ob=ob, bvh=bvh, cut=H.select_cut(bvh, 32), diffuse=dif, shadow=shd))
    return out


def _requests(H, scenes, n_req, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n_req):
        s = scenes[int(rng.integers(0, len(scenes)))]
        closest = bool(rng.random() < 0.7)
        pool = s["diffuse"] if closest else s["shadow"]
        n = int(min(pool.shape[0], np.exp(rng.uniform(np.log(1), np.log(pool.shape[0])))))
        off = int(rng.integers(0, pool.shape[0] - n + 1))
        rays = np.ascontiguousarray(pool[off:off + n])
        reqs.append((s, H.Batch(s["bvh"], torch.from_numpy(rays).cuda(), closest, cut=s["cut"]), rays))
    return reqs


def _lone(H, s, b, key_mode):
    perm = None
    if key_mode != 0:
        perm = H.sort(H.encode(s["bvh"], b.cut, key_mode, 32, b.rays), 32)
    return H.trace(s["bvh"], b.rays, perm, closest=b.closest).cpu().numpy()


# "graph" routes requests of 3,000+ rays through the full-device kernels, the rest through the
# engine; "engine-only" sends everything through the engine
VARIANTS = {"graph": dict(plain=False, graphs=True, direct_min=3000), "engine-only": dict(plain=False, direct_min=0xFFFFFFFF),
            "eager": dict(plain=False, graphs=False),
            "graph-wide": dict(plain=False, graphs=True, wide=True), "plain": dict(plain=True),
            "plain-wide": dict(plain=True, wide=True)}


def _server(H, key_mode, variant, **kw):
    v = dict(VARIANTS[variant])
    wide = v.pop("wide", False)
    batch = H.BatchOpts(0, 0, 0, H.TRACE_WIDE) if wide else None
    return H.Server(key_mode=key_mode, key_bits=32, batch=batch, **v, **kw)


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("key_mode", [1, 2, 0])
def test_server_results_equal_lone_requests(H, scenes, variant, key_mode):
    plain = VARIANTS[variant]["plain"]
    reqs = _requests(H, scenes, 40, seed=key_mode * 7 + plain)
    srv = _server(H, key_mode, variant, max_group=8, streams=3)
    ids = [srv.submit(b) for _, b, _ in reqs]
    srv.drain()
    for rid, (s, b, rays) in zip(ids, reqs):
        st, lat = srv.poll(rid)
        assert st == H.REQ_DONE and lat > 0
        got = b.out.cpu().numpy()
        ref = _lone(H, s, b, key_mode)
        if b.closest:
            assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
        else:
            assert np.array_equal(got, ref)
    # and against the oracle for a few of them
    for s, b, rays in reqs[:6]:
        got = b.out.cpu().numpy()
        if b.closest:
            assert_closest(got, O.trace(s["ob"], rays), rays, s["spec"].tris)
        else:
            assert_any(got, O.trace(s["ob"], rays, closest=False))
    c = srv.counters()
    assert c["completed"] == len(reqs) and c["running"] == 0 and c["used_bytes"] == 0
    srv.close()


def test_server_graph_replays_match_eager(H, scenes):
    """The captured launch graphs are replayed group after group; between rounds the test runs
    its own eager work (the lone path) and synchronises, and checks every round's results."""
    srv = _server(H, 1, "engine-only", max_group=4, streams=2)
    for rnd in range(4):
        reqs = _requests(H, scenes, 12, seed=100 + rnd)
        ids = [srv.submit(b) for _, b, _ in reqs]
        srv.drain()
        torch.cuda.synchronize()
        for rid, (s, b, rays) in zip(ids, reqs):
            assert srv.poll(rid)[0] == H.REQ_DONE
            ref = _lone(H, s, b, 1)
            got = b.out.cpu().numpy()
            assert np.array_equal(got.view(np.uint8), ref.view(np.uint8)), f"round {rnd}"
    assert srv.counters()["launches"] >= 4 * 3
    srv.close()


def test_server_budget_admission_and_refusal(H, scenes):
    s = scenes[1]
    small = [H.Batch(s["bvh"], torch.from_numpy(s["diffuse"][:2000]).cuda(), True, cut=s["cut"]) for _ in range(6)]
    big = H.Batch(s["bvh"], torch.from_numpy(s["diffuse"]).cuda(), True, cut=s["cut"])
    # budget for one small request at a time: all still complete, one after the other
    one = H.Server(key_mode=H.KEY_HCC, budget_bytes=250_000)
    ids = [one.submit(b) for b in small]
    with pytest.raises(H.HCCError) as e:
        one.submit(big)
    assert e.value.status == 5   # HCC_ERR_BUDGET
    one.drain()
    assert all(one.poll(i)[0] == H.REQ_DONE for i in ids)
    assert one.counters()["launches"] == len(small)
    ref = _lone(H, s, small[0], H.KEY_HCC)
    for b in small:
        assert np.array_equal(b.out.cpu().numpy().view(np.uint32), ref.view(np.uint32))
    one.close()


def test_server_cancel_queued_request(H, scenes):
    s = scenes[1]
    big_rays = torch.from_numpy(np.resize(s["diffuse"], (3_000_000, 8))).cuda()
    first = H.Batch(s["bvh"], big_rays, True, cut=s["cut"])
    later = [H.Batch(s["bvh"], torch.from_numpy(s["diffuse"][:1000]).cuda(), True, cut=s["cut"]) for _ in range(3)]
    for b in later:
        b.out.fill_(7.0)
    srv = H.Server(key_mode=H.KEY_HCC, max_inflight=1)
    f = srv.submit(first)
    ids = [srv.submit(b) for b in later]
    srv.cancel(ids[-1])                     # still queued behind the running 3M-ray request
    srv.drain()
    assert srv.poll(f)[0] == H.REQ_DONE
    assert srv.poll(ids[-1])[0] == H.REQ_CANCELLED
    assert torch.all(later[-1].out == 7.0)  # never touched
    assert all(srv.poll(i)[0] == H.REQ_DONE for i in ids[:-1])
    with pytest.raises(H.HCCError):
        srv.cancel(f)                       # already done
    srv.close()


def test_server_shutdown_with_pending(H, scenes):
    s = scenes[0]
    srv = H.Server(key_mode=H.KEY_TWOPOINT, max_inflight=1)
    bs = [H.Batch(s["bvh"], torch.from_numpy(s["diffuse"]).cuda(), True) for _ in range(20)]
    for b in bs:
        srv.submit(b)
    t0 = time.time()
    srv.close()                             # cancels the queued ones, waits for admitted ones
    assert time.time() - t0 < 30
