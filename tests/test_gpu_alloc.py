"""The device-memory hooks: with PyTorch's caching allocator installed every library-owned
buffer comes from it and goes back to it, and results are unchanged."""
import gc

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    assert torch.cuda.is_available()
    import paper_2305_16652_amd as H
    return H


def _run(H, bvh, cut, rays):
    keys = H.encode(bvh, cut, H.KEY_HCC, 32, rays)
    perm = H.sort(keys, 32)
    hits = H.trace(bvh, rays, perm)
    return keys.cpu().numpy(), perm.cpu().numpy(), hits.cpu().numpy()


def test_hooked_allocations_balance_and_results_match(H):
    spec = W.tiny_scene()
    tris = torch.from_numpy(spec.tris).cuda()
    rays = torch.from_numpy(W.pinhole_rays(spec, 48, 40)).cuda()
    H.set_allocator()
    b0 = H.build_bvh(tris)
    ref = _run(H, b0, H.select_cut(b0, 32), rays)
    ref_export = b0.export()

    dev = torch.cuda.current_device()
    live, counts = {}, dict(alloc=0, free=0, bad_free=0)

    def alloc(n, stream):
        p = torch.cuda.caching_allocator_alloc(max(n, 1), dev, stream)
        live[p] = n
        counts["alloc"] += 1
        return p

    def free(p, stream):
        if p not in live:
            counts["bad_free"] += 1
            return
        del live[p]
        counts["free"] += 1
        torch.cuda.caching_allocator_delete(p)

    try:
        H.set_allocator(alloc, free)
        b1 = H.build_bvh(tris)
        assert counts["alloc"] > 9 and len(live) == 9          # 9 BVH arrays kept (with the quantised nodes), temporaries returned
        c1 = H.select_cut(b1, 32)
        m1 = H.select_mlhcc_cut(b1, 8, 8)
        g1 = H.grid_cut(b1, 4, 4, 2)
        assert len(live) == 12
        out = _run(H, b1, c1, rays)
        for a, e in zip(out, ref):
            assert np.array_equal(a.view(np.uint32), e.view(np.uint32))
        for a, e in zip(b1.export(), ref_export):
            assert np.array_equal(a, e)
        # a server created under the hooks takes its workspaces from them too
        srv = H.Server(key_mode=H.KEY_HCC, key_bits=32, max_group=4, streams=2)
        batches = [H.Batch(b1, rays[i * 400:(i + 1) * 400], True, cut=c1) for i in range(4)]
        before = counts["alloc"]
        for batch in batches:
            srv.submit(batch)
        del batch
        srv.drain()
        srv.close()
        assert counts["alloc"] > before and len(live) == 12
        got = np.concatenate([b.out.cpu().numpy() for b in batches])
        assert np.array_equal(got.view(np.uint32), ref[2][:1600].view(np.uint32))
        del m1, g1, c1, b1, batches, srv
        gc.collect()
    finally:
        H.set_allocator()
    assert not live and counts["alloc"] == counts["free"] and counts["bad_free"] == 0
    # objects created after the reset use hipMalloc again
    n_before = counts["alloc"]
    b2 = H.build_bvh(tris)
    assert counts["alloc"] == n_before
    del b2


def test_failing_hook_reports_oom(H):
    spec = W.tiny_scene()
    tris = torch.from_numpy(spec.tris).cuda()
    try:
        H.set_allocator(lambda n, s: 0, lambda p, s: None)
        with pytest.raises(H.HCCError) as e:
            H.build_bvh(tris)
        assert e.value.status == 2
    finally:
        H.set_allocator()
