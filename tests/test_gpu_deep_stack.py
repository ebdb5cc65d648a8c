"""Traversal stacks deeper than every LDS part of the kernels' stacks.

A row of 2^20 small triangles along the x axis (all at y = z = 0.5, 1,024 distinct Morton codes
with 1,024 triangles on each) gives a BVH2 of depth 21.  A ray running along the row meets both
children of most nodes it visits, so a near-first traversal keeps pushing the far child on its
way down: a BVH2 traversal of these rays holds up to 19 entries at once (more than the 16 LDS
entries of the short stacks), and a 4-wide traversal pushes up to three entries per level, so
the kernels' spills to scratch are exercised.  Every launch kind is compared with the oracle,
closest and any hit, in generation order and through a permutation."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from parity_utils import assert_any, assert_closest

pytestmark = pytest.mark.gpu

N_ROW = 1 << 20
EPS = 1e-3


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def row_scene() -> np.ndarray:
    x = (np.arange(N_ROW, dtype=np.float64) + 0.5) / N_ROW
    t = np.zeros((N_ROW, 9), np.float64)
    t[:, 0], t[:, 1], t[:, 2] = x, 0.5 - EPS, 0.5 - EPS
    t[:, 3], t[:, 4], t[:, 5] = x, 0.5 + EPS, 0.5 - EPS
    t[:, 6], t[:, 7], t[:, 8] = x, 0.5, 0.5 + EPS
    corners = np.array([[0, 0, 0, 1, 0, 0, 0, 1, 1], [1, 1, 1, 0, 1, 1, 1, 0, 0]], np.float64)   # scene box [0,1]^3
    return np.concatenate([t, corners]).astype(np.float32)


def row_rays(n: int, seed: int) -> np.ndarray:
    """Rays along the row (either direction, slope below 5e-4 so that they stay inside the
    triangles' +-1e-3 band over the whole row), from before, inside and after it, half of them
    segments ending inside the row."""
    u = W.uniform01(seed, 0, np.arange(6 * n, dtype=np.uint64)).reshape(n, 6)
    r = np.zeros((n, 8), np.float64)
    sign = np.where(u[:, 0] < 0.5, 1.0, -1.0)
    r[:, 0] = -0.05 + 1.1 * u[:, 1]
    r[:, 1] = 0.5 + (u[:, 2] - 0.5) * 2e-4
    r[:, 2] = 0.5 + (u[:, 3] - 0.5) * 2e-4
    r[:, 4] = sign
    r[:, 5] = (u[:, 4] - 0.5) * 5e-4
    r[:, 6] = (u[:, 5] - 0.5) * 5e-4
    r[:, 3] = 0.0
    r[:, 7] = np.where(np.arange(n) % 2 == 0, np.inf, 0.25 + 0.5 * u[:, 2])
    return r.astype(np.float32)


def bvh2_depth(ob) -> int:
    n = ob.child.shape[0] + 1
    depth = {0: 0}
    stack = [0]
    while stack:
        x = stack.pop()
        if x < n - 1:
            for c in ob.child[x]:
                depth[int(c)] = depth[x] + 1
                stack.append(int(c))
    return max(depth.values())


@pytest.fixture(scope="module")
def H():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2305_16652_amd as H
    return H


@pytest.fixture(scope="module")
def scene(H):
    tris = row_scene()
    ob = O.build_bvh(tris)
    rays = row_rays(8192, seed=91)
    ref_c = O.trace(ob, rays, threads=8)
    ref_a = O.trace(ob, rays, closest=False, threads=8)
    bvh = H.build_bvh(torch.from_numpy(tris).cuda())
    torch.cuda.synchronize()
    return dict(tris=tris, ob=ob, rays=rays, ref_c=ref_c, ref_a=ref_a, bvh=bvh)


def test_scene_is_deep(scene):
    assert bvh2_depth(scene["ob"]) >= 20
    # most rays hit the row, and a closest hit is never behind the first triangle met
    assert (scene["ref_c"].prim != 0xFFFFFFFF).mean() > 0.9


# (block, stack, remap, persistent, refill, chunk, waves, flags)
DEEP_OPTS = [
    (64, 0, 0, 0, 0, 0, 0, 0),          # one ray per lane, scratch stack
    (64, 1, 0, 0, 0, 0, 0, 0),          # one ray per lane, whole stack in LDS
    (128, 2, 0, 0, 0, 0, 0, 0),         # one ray per lane, 16 LDS entries + scratch
    (0, 0, 0, 1, 32, 64, 0, 1),         # persistent BVH2, speculative descent, scratch
    (0, 1, 0, 1, 32, 64, 0, 0),         # persistent BVH2, LDS stack
    (0, 2, 0, 1, 24, 128, 0, 0),        # persistent BVH2, short stack
    (64, 2, 0, 1, 32, 64, 0, 2),        # 4-wide, 16 LDS entries + scratch
    (64, 1, 0, 1, 32, 64, 0, 2),        # 4-wide, 24 LDS entries + scratch
    (64, 0, 0, 1, 32, 64, 0, 2),        # 4-wide, scratch only
    (64, 2, 0, 1, 32, 64, 0, 6 | 8),    # 4-wide, slab child test, spread dealing
    (64, 2, 0, 1, 32, 64, 0, 2 | 16),   # quantised 4-wide nodes, 16 LDS entries + scratch
    (64, 0, 0, 1, 32, 64, 0, 6 | 16),   # quantised 4-wide nodes, slab child test, scratch only
    (0, 0, 0, 1, 0, 0, 0, 2 | 32),      # wavefront packets, shared register stack
    (0, 0, 0, 1, 0, 0, 0, 2 | 16 | 32), # wavefront packets on the quantised nodes
]


@pytest.mark.parametrize("opt", DEEP_OPTS)
def test_deep_traversal_matches_oracle(H, scene, opt):
    _say(f"deep stack, opts {opt}")
    o = H.TraceOpts(*opt)
    rays = scene["rays"]
    rd = torch.from_numpy(rays).cuda()
    perm = np.random.default_rng(5).permutation(rays.shape[0]).astype(np.uint32)
    pd = torch.from_numpy(perm.view(np.int32)).cuda()
    hits = H.trace(scene["bvh"], rd, opts=o)
    hits_p = H.trace(scene["bvh"], rd, perm=pd, opts=o)
    occ = H.trace(scene["bvh"], rd, closest=False, opts=o)
    torch.cuda.synchronize()
    h = hits.cpu().numpy()
    assert_closest(h, scene["ref_c"], rays, scene["tris"])
    assert np.array_equal(hits_p.cpu().numpy().view(np.uint32), h.view(np.uint32))
    assert_any(occ.cpu().numpy(), scene["ref_a"])


@pytest.mark.parametrize("wide,stack", [(False, 0), (True, 0), (True, 1), (True, 3)],
                         ids=["bvh2", "wide-12-lds", "wide-24-lds", "wide-scratch"])
def test_deep_traversal_in_the_engine(H, scene, wide, stack):
    """The batched engine's trace phase (BVH2 with its scratch stack, or 4-wide with 12 / 24 LDS
    entries or scratch only) on the same rays in two uneven batches, NoSort and HCC keys."""
    _say(f"deep stack engine, wide={wide} stack={stack}")
    rays = scene["rays"]
    rd = torch.from_numpy(rays).cuda()
    cut = H.select_cut(scene["bvh"], 16)
    split = 3001
    for mode in (0, H.KEY_HCC):
        bc = H.Batch(scene["bvh"], rd[:split], True, cut=cut)
        ba = H.Batch(scene["bvh"], rd[split:], False, cut=cut)
        o = H.BatchOpts(64, 32, 0, H.TRACE_WIDE if wide else 0, 0, stack)
        H.batch_run([bc, ba], mode, 16, opts=o)
        torch.cuda.synchronize()
        full = np.zeros((rays.shape[0], 4), np.float32)
        full[:split] = bc.out.cpu().numpy()
        assert_closest(full, scene["ref_c"], rays, scene["tris"], idx=np.arange(split))
        assert_any(ba.out.cpu().numpy(), np.asarray(scene["ref_a"])[split:])
