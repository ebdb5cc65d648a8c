"""Pins of the oracle's lockstep wave model (O8: distinct node and triangle fetches per wave and
lockstep step; the per-warp coherence argument of Section 3.1, Table 6 in Section 6.5).

The model is checked against counts made by hand on the four-triangle BVH, against a separate
pure-Python traversal and lockstep count written here from the model's definition, and against
properties any such count has (one copy of a ray per lane costs one ray; waves never cost more
than their rays traced alone; lane order inside a wave does not matter)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from test_oracle import _four_triangles, random_rays


def _ray(o, d, tmin=0.0, tmax=np.inf):
    return np.array([*o, tmin, *d, tmax], np.float32)


def _counts(bvh, rays, width, order, closest=True, perm=None):
    n, t, s = O.wave_fetches(bvh, np.stack(rays) if isinstance(rays, list) else rays, perm, width, closest, order)
    return n.astype(int).tolist(), t.astype(int).tolist(), s.astype(int).tolist()


# Four flat triangles at z = 0 (tests/golden/had_four_triangles.txt): root 0 -> internal 1
# (leaves 3 = T0 at (0, 0), 4 = T2 at (0, 0.875)) and internal 2 (leaves 5 = T1 at (0.875, 0),
# 6 = T3 at (0.875, 0.875)).
A = _ray((0.05, 0.05, 1.0), (0.0, 0.0, -1.0))     # straight down onto T0
B = _ray((0.9, 0.9, 1.0), (0.0, 0.0, -1.0))       # straight down onto T3
Cm = _ray((0.05, 0.5, 1.0), (0.0, 0.0, -1.0))     # inside internal 1's box, between its leaves
E = _ray((-1.0, 0.05, 0.0), (1.0, 0.0, 0.0))      # in the triangles' plane along +x: boxes 1, 3, 2, 5


def test_wave_model_hand_counts_child_test_order():
    bvh = O.build_bvh(_four_triangles())
    assert bvh.child.tolist() == [[1, 2], [3, 4], [5, 6]]
    # by hand: A steps (0), (1: leaf 3); B steps (0), (2: leaf 6); C steps (0), (1: no leaf);
    # E steps (0), (1: leaf 3, miss, det = 0), (2: leaf 5, miss)
    assert _counts(bvh, [A], 1, 1) == ([2], [1], [2])
    assert _counts(bvh, [B], 1, 1) == ([2], [1], [2])
    assert _counts(bvh, [Cm], 1, 1) == ([2], [0], [2])
    assert _counts(bvh, [E], 1, 1) == ([3], [2], [3])
    # a wave of two: step 0 shares the root; step 1 fetches nodes 1 and 2, triangles 3 and 6
    assert _counts(bvh, [A, B], 2, 1) == ([3], [2], [2])
    assert _counts(bvh, [A, A], 2, 1) == ([2], [1], [2])
    # A and E share node 1 and triangle 3 at step 1; E alone fetches node 2 and triangle 5
    assert _counts(bvh, [A, E], 2, 1) == ([3], [2], [3])
    assert _counts(bvh, [E, A], 2, 1) == ([3], [2], [3])
    assert _counts(bvh, [A, B, Cm, E], 4, 1) == ([1 + 2 + 1], [2 + 1], [3])
    # ragged last wave: three rays in waves of two
    assert _counts(bvh, [A, B, E], 2, 1) == ([3, 3], [2, 2], [2, 3])


def test_wave_model_hand_counts_pop_order():
    bvh = O.build_bvh(_four_triangles())
    # the traversal of the trace oracle: every popped node whose box passes is a step;
    # A: 0, 1, leaf 3.  E: 0, 1, leaf 3, 2, leaf 5.  C: 0, 1.  B: 0, 2, leaf 6.
    assert _counts(bvh, [A], 1, 0) == ([2], [1], [3])
    assert _counts(bvh, [E], 1, 0) == ([3], [2], [5])
    assert _counts(bvh, [Cm], 1, 0) == ([2], [0], [2])
    assert _counts(bvh, [A, E], 2, 0) == ([3], [2], [5])
    assert _counts(bvh, [A, B], 2, 0) == ([3], [2], [3])
    # any hit: A stops at its triangle, E never hits (its triangles lie in the ray's plane)
    assert _counts(bvh, [A, E], 2, 0, closest=False) == ([3], [2], [5])


def test_wave_model_single_triangle():
    tri = np.array([[0, 0, 1, 1, 0, 1, 0, 1, 1]], np.float32)
    bvh = O.build_bvh(tri)
    r = _ray((0.2, 0.2, 0.0), (0.0, 0.0, 1.0))
    for order in (0, 1):
        assert _counts(bvh, [r, r], 2, order) == ([0], [1], [1])


# ----------------------------------------------------------------------------- independent model

def _slab32(ray, box):
    """(hit, tnear) of the float32 slab test over [tmin, tmax] (minNum / maxNum, far x (1 + 3 ulp))."""
    f = np.float32
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        o = ray[0:3].astype(f)
        inv = (f(1.0) / ray[4:7].astype(f)).astype(f)
        t0 = ((box[0:3] - o) * inv).astype(f)
        t1 = ((box[3:6] - o) * inv).astype(f)
    tn = np.fmin(t0, t1)
    tf = (np.fmax(t0, t1) * f(1.0000003576278687)).astype(f)
    tnear = np.fmax(np.fmax(np.fmax(tn[0], tn[1]), tn[2]), ray[3])
    tfar = np.fmin(np.fmin(np.fmin(tf[0], tf[1]), tf[2]), ray[7])
    return bool(tnear <= tfar), tnear


def _tri32(tri, ray):
    """Moller-Trumbore in float32, operations in the order of the trace oracle; t or None."""
    f = np.float32
    with np.errstate(all="ignore"):
        v0, v1, v2 = tri[0:3], tri[3:6], tri[6:9]
        o, d = ray[0:3], ray[4:7]
        e1, e2 = (v1 - v0).astype(f), (v2 - v0).astype(f)
        p = np.array([d[1] * e2[2] - d[2] * e2[1], d[2] * e2[0] - d[0] * e2[2], d[0] * e2[1] - d[1] * e2[0]], f)
        det = f(f(e1[0] * p[0] + e1[1] * p[1]) + e1[2] * p[2])
        if det == 0:
            return None
        inv = f(f(1.0) / det)
        s = (o - v0).astype(f)
        u = f(f(f(s[0] * p[0] + s[1] * p[1]) + s[2] * p[2]) * inv)
        if not (u >= 0 and u <= 1):
            return None
        q = np.array([s[1] * e1[2] - s[2] * e1[1], s[2] * e1[0] - s[0] * e1[2], s[0] * e1[1] - s[1] * e1[0]], f)
        v = f(f(f(d[0] * q[0] + d[1] * q[1]) + d[2] * q[2]) * inv)
        if not (v >= 0 and f(u + v) <= 1):
            return None
        t = f(f(f(e2[0] * q[0] + e2[1] * q[1]) + e2[2] * q[2]) * inv)
        if not (ray[3] < t < ray[7]):
            return None
        return t


def _py_steps(bvh, ray, closest, order):
    """The model's step list of one ray, as [(node or None, {triangle leaf ids})]."""
    n_int = bvh.n - 1
    boxes, child, tris, lp = bvh.boxes, bvh.child, bvh.tris, bvh.leaf_prim
    best = [ray[7], None]                     # best t, best prim

    def leaf_hit(leaf_uid):
        prim = int(lp[leaf_uid - n_int])
        t = _tri32(tris[prim], ray)
        if t is None:
            return False
        if best[1] is None or t < best[0] or (t == best[0] and prim < best[1]):
            best[0], best[1] = t, prim
        return True

    steps = []
    if order == 0:
        stack = [0]
        while stack:
            u = stack.pop()
            if not _slab32(np.array([*ray[:7], best[0]], np.float32), boxes[u])[0]:
                continue
            if u >= n_int:
                steps.append((None, {u}))
                if leaf_hit(u) and not closest:
                    break
                continue
            steps.append((u, set()))
            c0, c1 = int(child[u, 0]), int(child[u, 1])
            seg = np.array([*ray[:7], best[0]], np.float32)
            h0, n0 = _slab32(seg, boxes[c0])
            h1, n1 = _slab32(seg, boxes[c1])
            if h0 and h1:
                stack += [c0, c1] if n1 < n0 else [c1, c0]
            elif h0:
                stack.append(c0)
            elif h1:
                stack.append(c1)
        return steps
    stack, u = [], 0
    while True:
        c0, c1 = int(child[u, 0]), int(child[u, 1])
        seg = np.array([*ray[:7], best[0] if closest else ray[7]], np.float32)
        h0, n0 = _slab32(seg, boxes[c0])
        h1, n1 = _slab32(seg, boxes[c1])
        leaves = {c for c, h in ((c0, h0), (c1, h1)) if h and c >= n_int}
        steps.append((u, leaves))
        hit = False
        for c in sorted(leaves):
            hit |= leaf_hit(c)
        if hit and not closest:
            break
        inner = [(c, nr) for c, h, nr in ((c0, h0, n0), (c1, h1, n1)) if h and c < n_int]
        if len(inner) == 2:
            near, far = (inner[1], inner[0]) if inner[1][1] < inner[0][1] else (inner[0], inner[1])
            stack.append(far[0])
            u = near[0]
        elif len(inner) == 1:
            u = inner[0][0]
        elif stack:
            u = stack.pop()
        else:
            break
    return steps


def _py_wave_counts(bvh, rays, perm, width, closest, order):
    order_idx = np.arange(rays.shape[0]) if perm is None else perm
    out_n, out_t = [], []
    for w0 in range(0, len(order_idx), width):
        lanes = [_py_steps(bvh, rays[r], closest, order) for r in order_idx[w0:w0 + width]]
        nodes = tris = 0
        for s in range(max(len(l) for l in lanes)):
            at = [l[s] for l in lanes if s < len(l)]
            nodes += len({node for node, _ in at if node is not None})
            tris += len(set().union(*(leaves for _, leaves in at)))
        out_n.append(nodes)
        out_t.append(tris)
    return out_n, out_t


@pytest.mark.parametrize("order", [0, 1])
@pytest.mark.parametrize("closest", [True, False])
def test_wave_model_matches_independent_count(order, closest):
    spec = W.tiny_scene()
    bvh = O.build_bvh(spec.tris)
    rays = random_rays(150, seed=31, tmax=np.inf if closest else 0.4)
    perm = np.random.default_rng(4).permutation(150).astype(np.uint32)
    for width, p in ((64, None), (32, perm)):
        n, t, _ = O.wave_fetches(bvh, rays, p, width, closest, order)
        pn, pt = _py_wave_counts(bvh, rays, p, width, closest, order)
        assert n.astype(int).tolist() == pn
        assert t.astype(int).tolist() == pt


def test_wave_model_properties():
    spec = W.tiny_scene()
    bvh = O.build_bvh(spec.tris)
    rays = random_rays(640, seed=32)
    _, nn, nt = O.trace(bvh, rays, counters=True)
    for order in (0, 1):
        n1, t1, s1 = O.wave_fetches(bvh, rays, None, 1, True, order)
        n64, t64, s64 = O.wave_fetches(bvh, rays, None, 64, True, order)
        # waves never fetch more than their rays alone, and at least their longest ray
        assert (n64 <= n1.reshape(-1, 64).sum(1)).all() and (t64 <= t1.reshape(-1, 64).sum(1)).all()
        assert (s64 == s1.reshape(-1, 64).max(1)).all()
        # lane order inside a wave does not change its count
        perm = np.concatenate([np.random.default_rng(w).permutation(64) + 64 * w for w in range(10)])
        pn, pt, _ = O.wave_fetches(bvh, rays, perm.astype(np.uint32), 64, True, order)
        assert (pn == n64).all() and (pt == t64).all()
        # a wave of copies of one ray costs that ray
        same = np.repeat(rays[:10], 64, axis=0)
        cn, ct, _ = O.wave_fetches(bvh, same, None, 64, True, order)
        assert (cn == n1[:10]).all() and (ct == t1[:10]).all()
    # order 0 with one ray per wave is the trace oracle's own per-ray count
    n1, t1, _ = O.wave_fetches(bvh, rays, None, 1, True, 0)
    assert (n1 == nn.astype(np.uint64) - nt).all() and (t1 == nt).all()
