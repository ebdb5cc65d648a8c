"""Pins for the CPU oracle: checks against what the paper and the mathematics fix,
independent of the oracle's own code (hand-computed values, the paper's printed
codes, a different construction algorithm, brute force, invariants)."""
import math
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
MISS = O.MISS


# ----------------------------------------------------------------------------- helpers

def _clz64(x: int) -> int:
    return 64 - x.bit_length()


def karras_tree(codes_sorted):
    """Karras (2012) parallel radix-tree construction, written out in Python.

    A different algorithm from the oracle's top-down split search: each internal
    node i finds its own range end by exponential + binary search and its split
    by binary search.  Returns child pairs as unified ids.
    """
    n = len(codes_sorted)
    keys = [(int(c) << 32) | j for j, c in enumerate(codes_sorted)]

    def delta(i, j):
        if j < 0 or j >= n:
            return -1
        return _clz64(keys[i] ^ keys[j])

    child = np.zeros((n - 1, 2), np.uint32)
    for i in range(n - 1):
        d = 1 if delta(i, i + 1) - delta(i, i - 1) > 0 else -1
        dmin = delta(i, i - d)
        lmax = 2
        while delta(i, i + lmax * d) > dmin:
            lmax *= 2
        l = 0
        t = lmax // 2
        while t >= 1:
            if delta(i, i + (l + t) * d) > dmin:
                l += t
            t //= 2
        j = i + l * d
        dnode = delta(i, j)
        s = 0
        div = 2
        while True:
            t = (l + div - 1) // div
            if delta(i, i + (s + t) * d) > dnode:
                s += t
            if t == 1:
                break
            div *= 2
        g = i + s * d + min(d, 0)
        left = (n - 1 + g) if min(i, j) == g else g
        right = (n - 1 + g + 1) if max(i, j) == g + 1 else g + 1
        child[i] = (left, right)
    return child


def tri_aabb(t):
    t = np.asarray(t, np.float32).reshape(3, 3)
    return np.concatenate([t.min(0), t.max(0)])


def leaves_under(bvh, node):
    out = []
    stack = [node]
    while stack:
        x = stack.pop()
        if bvh.is_leaf(x):
            out.append(x)
        else:
            stack.extend(int(c) for c in bvh.child[x])
    return out


def parents(bvh):
    par = {}
    for i in range(bvh.n - 1):
        for c in bvh.child[i]:
            par[int(c)] = i
    return par


def random_tris(n, seed, dup=False):
    idx = np.arange(n, dtype=np.uint64)
    v0 = np.stack([W.uniform01(seed, a, idx) for a in range(3)], -1)
    if dup:   # force many equal Morton codes
        v0 = np.round(v0 * 4) / 4
    e1 = (np.stack([W.uniform01(seed, 3 + a, idx) for a in range(3)], -1) - 0.5) * 0.05
    e2 = (np.stack([W.uniform01(seed, 6 + a, idx) for a in range(3)], -1) - 0.5) * 0.05
    return np.concatenate([v0, v0 + e1, v0 + e2], 1).astype(np.float32)


def random_rays(n, seed, lo=-0.2, hi=1.2, tmax=np.inf):
    idx = np.arange(n, dtype=np.uint64)
    o = lo + (hi - lo) * np.stack([W.uniform01(seed, 20 + a, idx) for a in range(3)], -1)
    d = np.stack([W.uniform01(seed, 23 + a, idx) for a in range(3)], -1) - 0.5
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = np.zeros((n, 8), np.float32)
    r[:, 0:3] = o
    r[:, 3] = 0.0
    r[:, 4:7] = d
    r[:, 7] = tmax
    return r


# ----------------------------------------------------------------------------- Morton

def test_morton3_closed_forms():
    assert O.morton3(0, 0, 1) == 1
    assert O.morton3(0, 1, 0) == 2
    assert O.morton3(1, 0, 0) == 4
    assert O.morton3(1023, 0, 0) == 0x24924924
    assert O.morton3(0, 1023, 0) == 0x12492492
    assert O.morton3(0, 0, 1023) == 0x09249249
    assert O.morton3(1023, 1023, 1023) == (1 << 30) - 1
    assert O.morton3(512, 0, 0) == 1 << 29


def test_morton_quantisation_cases():
    # scene box [0,1]^3 spanned by two big triangles; probes at known centres
    frame = np.array([[0, 0, 0, 1, 0, 0, 0, 1, 0], [1, 1, 1, 0, 1, 1, 1, 0, 1]], np.float32)
    probes = np.array([
        [0, 0, 0, 0, 0, 0, 0, 0, 0],                # centre at lo -> q = 0
        [1, 1, 1, 1, 1, 1, 1, 1, 1],                # centre at hi -> q = 1024 clamped to 1023
        [0.5, 0.5, 0.5] * 3,                        # centre 0.5 -> q = 512
        [0.25, 0.75, 0.125, 0.25, 0.75, 0.125, 0.25, 0.75, 0.125],
    ], np.float32)
    codes = O.morton_codes(np.concatenate([frame, probes]))[2:]
    assert codes[0] == 0
    assert codes[1] == (1 << 30) - 1
    assert codes[2] == O.morton3(512, 512, 512)
    assert codes[3] == O.morton3(256, 768, 128)


# ----------------------------------------------------------------------------- LBVH

@pytest.mark.parametrize("n,seed,dup", [(2, 1, False), (3, 2, False), (17, 3, False), (200, 4, False),
                                        (257, 5, True), (64, 6, True)])
def test_lbvh_equals_karras_construction(n, seed, dup):
    tris = random_tris(n, seed, dup)
    bvh = O.build_bvh(tris)
    assert np.array_equal(bvh.child, karras_tree(bvh.codes))


@pytest.mark.parametrize("n,seed,dup", [(1, 1, False), (2, 2, False), (100, 3, False), (300, 4, True)])
def test_lbvh_structure(n, seed, dup):
    tris = random_tris(n, seed, dup)
    bvh = O.build_bvh(tris)
    # leaves are the triangles in stable Morton order
    codes = O.morton_codes(tris)
    order = sorted(range(n), key=lambda i: (int(codes[i]), i))
    assert list(bvh.leaf_prim) == order
    assert np.array_equal(bvh.codes, codes[order])
    # leaf boxes are triangle AABBs
    for j in range(n):
        assert np.array_equal(bvh.boxes[n - 1 + j], tri_aabb(tris[bvh.leaf_prim[j]]))
    if n == 1:
        return
    # every node but the root has exactly one parent
    par = parents(bvh)
    assert sorted(par) == list(range(1, 2 * n - 1))
    # internal box = exact union; range contiguity; split at the highest differing bit
    keys = [(int(c) << 32) | j for j, c in enumerate(bvh.codes)]
    for i in range(n - 1):
        lv = sorted(x - (n - 1) for x in leaves_under(bvh, i))
        assert lv == list(range(lv[0], lv[-1] + 1))
        l, r = (int(c) for c in bvh.child[i])
        assert np.array_equal(bvh.boxes[i][:3], np.minimum(bvh.boxes[l][:3], bvh.boxes[r][:3]))
        assert np.array_equal(bvh.boxes[i][3:], np.maximum(bvh.boxes[l][3:], bvh.boxes[r][3:]))
        ll = sorted(x - (n - 1) for x in leaves_under(bvh, l))
        top = _clz64(keys[lv[0]] ^ keys[lv[-1]])
        bit = 63 - top
        assert all((keys[j] >> bit) & 1 == 0 for j in ll)
        assert all((keys[j] >> bit) & 1 == 1 for j in lv if j not in ll)
        # Karras numbering: an internal node's id is one end of its range
        assert i in (lv[0], lv[-1]) or i == 0


def test_lbvh_depth_bound():
    tris = random_tris(500, 9, dup=True)
    bvh = O.build_bvh(tris)
    depth = {0: 0}
    stack = [0]
    while stack:
        x = stack.pop()
        if not bvh.is_leaf(x):
            for c in bvh.child[x]:
                depth[int(c)] = depth[x] + 1
                stack.append(int(c))
    assert max(depth.values()) <= 63


# ----------------------------------------------------------------------------- HAD (Eq. 1)

def _four_triangles():
    a = 0.125
    out = []
    for (x, y) in [(0, 0), (0.875, 0), (0, 0.875), (0.875, 0.875)]:
        out.append([x, y, 0, x + a, y, 0, x, y + a, 0])
    return np.asarray(out, np.float32)


def test_had_hand_example():
    tris = _four_triangles()
    bvh = O.build_bvh(tris)
    assert list(bvh.leaf_prim) == [0, 2, 1, 3]
    assert bvh.child.tolist() == [[1, 2], [3, 4], [5, 6]]
    rows = [l.split() for l in open(os.path.join(GOLDEN, "had_four_triangles.txt")) if l[0] != "#"]
    for lam in (0.125, 0.5):
        h = O.had(bvh, lam)
        for lam_s, node, val in rows:
            if float(lam_s) == lam:
                assert h[int(node)] == float(val), (lam, node)


def test_had_scaling_and_monotonicity():
    tris = W.tiny_scene().tris
    bvh = O.build_bvh(tris)
    h = O.had(bvh)
    for k in (-3, 2):
        b2 = O.build_bvh(tris * np.float32(2.0 ** k))
        assert np.array_equal(b2.child, bvh.child)
        assert np.array_equal(b2.boxes, bvh.boxes * np.float32(2.0 ** k))
        h2 = O.had(b2)
        np.testing.assert_allclose(h2, h * 4.0 ** k, rtol=1e-14)
    for i in range(bvh.n - 1):
        for c in bvh.child[i]:
            assert h[i] > h[int(c)]
    # leaves: TC * SA with TC = 1
    n = bvh.n
    b = bvh.boxes[n - 1:].astype(np.float64)
    d = b[:, 3:] - b[:, :3]
    sa = 2.0 * ((d[:, 0] * d[:, 1] + d[:, 1] * d[:, 2]) + d[:, 2] * d[:, 0])
    assert np.array_equal(h[n - 1:], sa)


# ----------------------------------------------------------------------------- cut (Alg. 2)

def test_cut_hand_example():
    bvh = O.build_bvh(_four_triangles())
    h = O.had(bvh)
    assert O.select_cut(bvh, h, 1).tolist() == [0]
    assert O.select_cut(bvh, h, 2).tolist() == [1, 2]
    assert O.select_cut(bvh, h, 3).tolist() == [2, 3, 4]
    assert O.select_cut(bvh, h, 4).tolist() == [3, 4, 5, 6]
    assert O.select_cut(bvh, h, 5).tolist() == [3, 4, 5, 6]     # more than the leaves
    assert O.select_cut(bvh, h, 100).tolist() == [3, 4, 5, 6]


def test_cut_single_triangle():
    bvh = O.build_bvh(_four_triangles()[:1])
    h = O.had(bvh)
    assert O.select_cut(bvh, h, 1).tolist() == [0]
    assert O.select_cut(bvh, h, 8).tolist() == [0]


@pytest.mark.parametrize("cut_size", [1, 2, 7, 32, 64, 500, 3000])
def test_cut_invariants(cut_size):
    tris = W.tiny_scene().tris
    bvh = O.build_bvh(tris)
    h = O.had(bvh)
    cut = O.select_cut(bvh, h, cut_size)
    n = bvh.n
    assert len(cut) == min(cut_size, n)
    assert len(set(cut.tolist())) == len(cut)
    # a cut: every leaf lies under exactly one cut node
    cover = np.zeros(n, np.int64)
    for c in cut:
        for leaf in leaves_under(bvh, int(c)):
            cover[leaf - (n - 1)] += 1
    assert (cover == 1).all()
    # bit order: HAD descending, ties by id
    pairs = [(-h[c], int(c)) for c in cut]
    assert pairs == sorted(pairs)
    # max-HAD-first search: every expanded node outranks every internal cut node
    par = parents(bvh)
    anc = set()
    for c in cut:
        x = int(c)
        while x in par:
            x = par[x]
            anc.add(x)
    internal_cut = [int(c) for c in cut if not bvh.is_leaf(int(c))]
    if anc and internal_cut:
        assert min(h[a] for a in anc) >= max(h[c] for c in internal_cut)
    if cut_size == 2:
        assert sorted(cut.tolist()) == sorted(int(c) for c in bvh.child[0])


def test_cut_forces_leaf_in_unbalanced_tree():
    # the room walls are single-triangle leaves with large HAD: they must end up in the
    # cut as forced leaf nodes (Fig. Fig_BF (d)) while the search keeps going elsewhere
    tris = W.tiny_scene().tris
    bvh = O.build_bvh(tris)
    h = O.had(bvh)
    cut = O.select_cut(bvh, h, 64)
    leaf_prims = {int(bvh.leaf_prim[c - (bvh.n - 1)]) for c in cut if bvh.is_leaf(int(c))}
    assert set(range(12)) <= leaf_prims


def test_cut_scale_invariance():
    tris = W.tiny_scene().tris
    base = O.select_cut(O.build_bvh(tris), O.had(O.build_bvh(tris)), 64)
    for k in (-2, 3):
        b = O.build_bvh(tris * np.float32(2.0 ** k))
        assert np.array_equal(O.select_cut(b, O.had(b), 64), base)


# ----------------------------------------------------------------------------- HCC key (Alg. 1)

def _grid_boxes():
    """16 cells of a 4x4 grid, cell i = row-major (row 0 at the top), z in [-1, 1]."""
    boxes = []
    for i in range(16):
        r, c = divmod(i, 4)
        boxes.append([c, 3 - r, -1, c + 1, 4 - r, 1])
    return np.asarray(boxes, np.float32)


def _ray(o, d, tmax=np.inf, tmin=0.0):
    return np.array([o[0], o[1], 0.0, tmin, d[0], d[1], 0.0, tmax], np.float32)


SPACE_ANCHOR_RAYS = {
    "Ray1": _ray((0.9, 3.95), (1.0, -3.0), 0.8),
    "Ray2": _ray((0.92, 3.93), (1.0, -3.0), 0.8),
    "Ray3": _ray((2.3, 1.05), (-1.0, -0.35)),
    "Ray4": _ray((1.98, 0.3), (1.0, 2.2)),
}


def test_hcc_space_anchor_codes():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "space_anchor_codes.txt")) if l[0] != "#"]
    boxes = _grid_boxes()
    for name, code, cells in rows:
        key = int(O.encode_hcc(SPACE_ANCHOR_RAYS[name][None], boxes, 16)[0])
        assert key == int(code, 2), (name, format(key, "016b"), code)
        expect = sum(1 << (15 - int(c)) for c in cells.split(","))
        assert key == expect


def test_hcc_reversed_ray_changes_code():
    boxes = _grid_boxes()
    r3 = SPACE_ANCHOR_RAYS["Ray3"].copy()
    rev = r3.copy()
    rev[4:7] *= -1
    k3, kr = O.encode_hcc(np.stack([r3, rev]), boxes, 16)
    assert k3 != kr
    assert int(kr) == (1 << (15 - 10)) | (1 << (15 - 11))


def test_hcc_bit_count_rules():
    boxes = _grid_boxes()
    r = SPACE_ANCHOR_RAYS["Ray1"][None]
    # more cut nodes than key bits: only the first K nodes are encoded (MSB first)
    assert int(O.encode_hcc(r, boxes, 4)[0]) == 0b1100
    # fewer cut nodes than bits: low bits stay zero
    assert int(O.encode_hcc(r, boxes, 20)[0]) == 0xC440 << 4
    k64 = int(O.encode_hcc(r, boxes, 64)[0])
    assert k64 == 0xC440 << 48


def _np_slab(ray, box):
    """Independent float32 slab test in numpy (fmin/fmax ignore NaN like minNum/maxNum)."""
    f = np.float32
    o = ray[0:3].astype(f)
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        inv = (f(1.0) / ray[4:7].astype(f)).astype(f)
        t0 = ((box[0:3].astype(f) - o) * inv).astype(f)
        t1 = ((box[3:6].astype(f) - o) * inv).astype(f)
    tn = np.fmin(t0, t1)
    tf = (np.fmax(t0, t1) * f(1.0000003576278687)).astype(f)
    tnear = np.fmax(np.fmax(np.fmax(tn[0], tn[1]), tn[2]), f(ray[3]))
    tfar = np.fmin(np.fmin(np.fmin(tf[0], tf[1]), tf[2]), f(ray[7]))
    return bool(tnear <= tfar)


def test_hcc_bits_equal_no_cull_traversal():
    """Bit i set <=> a traversal that visits every node whose box the ray meets
    (no culling by hit distance) reaches cut node i (Section 4.2.1)."""
    scene = W.tiny_scene()
    bvh = O.build_bvh(scene.tris)
    cut = O.select_cut(bvh, O.had(bvh), 32)
    rays = random_rays(300, 7)
    rays[::3, 7] = 0.3                                  # some short segments
    keys = O.encode_hcc(rays, O.cut_boxes(bvh, cut), 32)
    cut_pos = {int(c): i for i, c in enumerate(cut)}
    for r, key in zip(rays, keys):
        reached = set()
        stack = [0]
        while stack:
            x = stack.pop()
            if not _np_slab(r, bvh.boxes[x]):
                continue
            if x in cut_pos:
                reached.add(cut_pos[x])
                continue
            if not bvh.is_leaf(x):
                stack.extend(int(c) for c in bvh.child[x])
        expect = sum(1 << (31 - i) for i in reached)
        assert int(key) == expect


def test_hcc_scale_invariance():
    scene = W.tiny_scene()
    bvh = O.build_bvh(scene.tris)
    cut = O.select_cut(bvh, O.had(bvh), 64)
    rays = random_rays(2000, 11)
    base = O.encode_hcc(rays, O.cut_boxes(bvh, cut), 64)
    for k in (-4, 5):
        s = np.float32(2.0 ** k)
        r2 = rays.copy()
        r2[:, 0:3] *= s
        r2[:, 3] *= s
        r2[:, 7] *= s
        b2 = O.build_bvh(scene.tris * s)
        c2 = O.select_cut(b2, O.had(b2), 64)
        assert np.array_equal(c2, cut)
        assert np.array_equal(O.encode_hcc(r2, O.cut_boxes(b2, c2), 64), base)


def test_slab_edge_cases():
    box = np.array([0, 0, 0, 1, 1, 1], np.float32)
    assert O.slab(np.array([0.5, 0.5, 0.5, 0, 1, 0, 0, np.inf], np.float32), box)   # inside, axis aligned
    # a ray lying in a face plane, parallel to it: 0 * inf = NaN on that axis and the
    # remaining operand is +-inf, so the interval is empty (the same as Moller-Trumbore's
    # det == 0 for a triangle in that plane)
    assert not O.slab(np.array([0.5, 0.5, 0.0, 0, 1, 0, 0, np.inf], np.float32), box)
    assert not O.slab(np.array([0.5, 0.5, 1.0, 0, 1, 0, 0, np.inf], np.float32), box)
    assert not O.slab(np.array([2, 0.5, 0.5, 0, 1, 0, 0, np.inf], np.float32), box)   # pointing away
    assert O.slab(np.array([2, 0.5, 0.5, 0, -1, 0, 0, np.inf], np.float32), box)
    assert not O.slab(np.array([2, 0.5, 0.5, 0, -1, 0, 0, 0.5], np.float32), box)     # segment too short
    assert not O.slab(np.array([0.5, 0.5, 0.5, 2, 1, 0, 0, 3], np.float32), box)       # starts beyond
    assert not O.slab(np.array([0.5, 2.0, 0.5, 0, 1, 0, 0, np.inf], np.float32), box)  # parallel, outside
    # the oracle's slab agrees with the independent numpy version on random cases
    rays = random_rays(500, 13, -1.0, 2.0)
    rays[::4, 4] = 0.0
    rays[1::4, 5] = -0.0
    for r in rays:
        assert O.slab(r, box) == _np_slab(r, box)


# ----------------------------------------------------------------------------- TwoPoint key

def _unit_scene_box_tris():
    return np.array([[0, 0, 0, 1, 0, 0, 0, 1, 0], [1, 1, 1, 0, 1, 1, 1, 0, 1]], np.float32)


def test_twopoint_hand_cases():
    lohi = O.scene_box(_unit_scene_box_tris())
    assert lohi.tolist() == [0, 0, 0, 1, 1, 1]
    r = np.array([[0, 0, 0, 0, 1, 0, 0, np.inf]], np.float32)    # origin at lo, +x
    # K = 12: two bits per dim; endpoint x = 0.25 -> q = 1 (binary 01): second level, dim 3
    assert int(O.encode_twopoint(r, lohi, 12)[0]) == 0b000000_000100
    # all six coordinates at the top of the box -> all ones
    top = np.array([[1, 1, 1, 0, 0, 0, 1, np.inf]], np.float32)
    top[0, 6] = 1.0
    for k in (16, 32, 64):
        assert int(O.encode_twopoint(top, lohi, k)[0]) == (1 << k) - 1 if k < 64 else 2 ** 64 - 1
    assert int(O.encode_twopoint(np.zeros((1, 8), np.float32) + [0, 0, 0, 0, -1, 0, 0, np.inf],
                                 lohi, 32)[0]) == 0
    # K = 32: dims get 6,6,5,5,5,5 bits; oz = 1 with a +x direction puts ones in dims 2
    # and 5 and the endpoint x = 0.25 -> q = 8 (01000) in dim 3
    r = np.array([[0, 0, 1, 0, 1, 0, 0, np.inf]], np.float32)
    assert int(O.encode_twopoint(r, lohi, 32)[0]) == 0x24D24924
    # the segment end clips the endpoint: tmax = 0.125 -> x = 0.125 -> q = 4 (00100)
    r[0, 7] = 0.125
    assert int(O.encode_twopoint(r, lohi, 32)[0]) == 0x24924924 | (1 << (31 - 3 - 2 * 6))


def test_twopoint_direction_length_invariance():
    lohi = O.scene_box(W.tiny_scene().tris)
    rays = random_rays(1000, 17)
    k1 = O.encode_twopoint(rays, lohi, 32)
    r2 = rays.copy()
    r2[:, 4:7] *= np.float32(4.0)          # exact scaling: normalised direction unchanged
    assert np.array_equal(O.encode_twopoint(r2, lohi, 32), k1)


# ----------------------------------------------------------------------------- sort

@pytest.mark.parametrize("n,bits,seed", [(0, 32, 1), (1, 32, 1), (1000, 4, 2), (5000, 32, 3), (3000, 64, 4),
                                         (777, 17, 5)])
def test_sort_is_stable_ascending(n, bits, seed):
    keys = W.u64_hash(seed, 0, np.arange(n, dtype=np.uint64)) >> np.uint64(64 - bits)
    perm = O.sort(keys)
    expect = sorted(range(n), key=lambda i: (int(keys[i]), i))
    assert perm.tolist() == expect


# ----------------------------------------------------------------------------- trace

def _np_mt64(tri, ray):
    """Moller-Trumbore in float64 for one triangle (independent of the C oracle)."""
    v0, v1, v2 = (tri[0:3].astype(np.float64), tri[3:6].astype(np.float64), tri[6:9].astype(np.float64))
    o, d = ray[0:3].astype(np.float64), ray[4:7].astype(np.float64)
    e1, e2 = v1 - v0, v2 - v0
    p = np.cross(d, e2)
    det = e1 @ p
    if det == 0:
        return None
    s = o - v0
    u = (s @ p) / det
    if u < 0 or u > 1:
        return None
    q = np.cross(s, e1)
    v = (d @ q) / det
    if v < 0 or u + v > 1:
        return None
    t = (e2 @ q) / det
    if not (ray[3] < t < ray[7]):
        return None
    return t


def test_trace_hand_cases():
    tri = np.array([[0, 0, 1, 1, 0, 1, 0, 1, 1]], np.float32)          # z = 1 plane
    tris = np.concatenate([tri, tri + np.float32([0, 0, 1] * 3)])     # and z = 2
    bvh = O.build_bvh(tris)
    rays = np.array([
        [0.25, 0.25, 0, 0, 0, 0, 1, np.inf],      # hits z=1 at t=1 (prim 0)
        [0.25, 0.25, 0, 0, 0, 0, 2, np.inf],      # unnormalised direction: t = 0.5
        [0.25, 0.25, 0, 0, 0, 0, 1, 0.5],         # segment ends before the hit
        [0.25, 0.25, 0, 1.5, 0, 0, 1, np.inf],    # starts past z=1: hits z=2 (prim 1)
        [0.75, 0.75, 0, 0, 0, 0, 1, np.inf],      # outside the triangle
        [0.25, 0.25, 3, 0, 0, 0, -1, np.inf],     # from above: first hit z=2 at t=1
    ], np.float32)
    h = O.trace(bvh, rays)
    assert h.t.tolist() == [1.0, 0.5, np.inf, 2.0, np.inf, 1.0]
    assert h.prim.tolist() == [0, 0, MISS, 1, MISS, 1]
    occ = O.trace(bvh, rays, closest=False)
    assert occ.tolist() == [1, 1, 0, 1, 0, 1]
    assert h.u[0] == 0.25 and h.v[0] == 0.25


def test_trace_matches_brute_force_tiny():
    scene = W.tiny_scene()
    bvh = O.build_bvh(scene.tris)
    rays = np.concatenate([W.pinhole_rays(scene, 32, 32), random_rays(2000, 19, 0.0, 1.0)])
    rays[1500:1700, 7] = 0.05
    h = O.trace(bvh, rays)
    bf = O.brute_force(scene.tris, rays)
    assert np.array_equal(h.t, bf.t)
    diff = np.nonzero(h.prim != bf.prim)[0]
    # a differing prim id is only allowed at an exact tie in t (rays through shared edges)
    for i in diff:
        assert h.t[i] == bf.t[i]
    assert diff.size <= 2
    occ = O.trace(bvh, rays, closest=False)
    assert np.array_equal(occ, O.brute_force(scene.tris, rays, closest=False))
    assert np.array_equal(occ, (bf.prim != MISS).astype(np.uint8))


def test_trace_agrees_with_float64_intersection():
    scene = W.tiny_scene(seed=4, n_random=300)
    bvh = O.build_bvh(scene.tris)
    rays = random_rays(400, 23, 0.0, 1.0)
    h = O.trace(bvh, rays)
    bad = 0
    for i, r in enumerate(rays):
        ts = [(_np_mt64(t, r), p) for p, t in enumerate(scene.tris)]
        ts = [(t, p) for t, p in ts if t is not None]
        if not ts:
            bad += h.prim[i] != MISS
            continue
        t64, p64 = min(ts)
        if h.prim[i] != p64:
            bad += 1
            continue
        assert abs(h.t[i] - t64) <= 1e-5 * abs(t64)
    assert bad <= 1


def test_trace_permutation_invariance():
    scene = W.tiny_scene()
    bvh = O.build_bvh(scene.tris)
    rays = random_rays(3000, 29, 0.0, 1.0)
    base = O.trace(bvh, rays)
    perm = np.random.default_rng(0).permutation(3000).astype(np.uint32)
    h2 = O.trace(bvh, rays, perm=perm, threads=3)
    assert np.array_equal(base.raw, h2.raw)
    occ = O.trace(bvh, rays, closest=False)
    assert np.array_equal(occ, O.trace(bvh, rays, perm=perm[::-1].copy(), closest=False))


def test_single_triangle_scene():
    tri = np.array([[0, 0, 1, 1, 0, 1, 0, 1, 1]], np.float32)
    bvh = O.build_bvh(tri)
    assert bvh.child.shape == (0, 2)
    assert bvh.boxes.shape == (1, 6)
    r = np.array([[0.2, 0.2, 0, 0, 0, 0, 1, np.inf], [2, 2, 0, 0, 0, 0, 1, np.inf]], np.float32)
    h = O.trace(bvh, r)
    assert h.prim.tolist() == [0, MISS]


# ----------------------------------------------------------------------------- metrics

def test_anc_definition():
    keys = np.array([1, 1, 2, 2, 3, 3, 3, 3], np.uint64)
    assert O.anc(keys, None, 4) == 1.5
    assert O.anc(keys, np.array([0, 2, 4, 6, 1, 3, 5, 7], np.uint32), 4) == 3.0
    assert O.anc(keys, None, 3) == pytest.approx((2 + 2 + 1) / 3)
