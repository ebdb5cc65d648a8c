"""Pins for the oracle's multi-level hierarchy cut code (Section 4.3, Alg. 3) and the
regular-grid control encoding (Section 5)."""
import numpy as np
import pytest

import os

import oracle as O
import workloads as W
from test_oracle import _four_triangles, leaves_under, random_rays

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_mlhcc_cut_hand_example():
    bvh = O.build_bvh(_four_triangles())
    h = O.had(bvh)
    top, low = O.select_mlhcc_cut(bvh, h, 2, 2)
    assert top.tolist() == [1, 2]
    assert low.tolist() == [[3, 4], [5, 6]]
    # only one top node wanted: the root (4 leaves >= 2)
    t1, l1 = O.select_mlhcc_cut(bvh, h, 1, 2)
    assert t1.tolist() == [0] and sorted(l1[0].tolist()) == [1, 2]
    # low level larger than any child: the root cannot be refined and is the only top node
    t3, l3 = O.select_mlhcc_cut(bvh, h, 4, 3)
    assert t3.tolist() == [0] and len(set(l3[0].tolist())) == 3
    # low level larger than the scene: no top node at all
    t5, _ = O.select_mlhcc_cut(bvh, h, 4, 5)
    assert t5.size == 0


def test_mlhcc_key_hand_example():
    bvh = O.build_bvh(_four_triangles())
    top, low = O.select_mlhcc_cut(bvh, O.had(bvh), 2, 2)
    tb = bvh.boxes[top]
    lb = bvh.boxes[low.reshape(-1)]
    rays = np.array([[0.05, 0.03, -1, 0, 0, 0, 1, np.inf],     # through T0: top node 1, low leaf 3
                     [0.9, 0.9, -1, 0, 0, 0, 1, np.inf],       # through T3: top node 2, low leaf 6
                     [0.5, 0.5, -1, 0, 0, 0, 1, np.inf],       # through nothing
                     [0.05, 0.5, -1, 0, 0, 0, 1, np.inf]],     # inside node 1's box, no leaf box
                    np.float32)
    keys = O.encode_mlhcc(rays, tb, lb, 2, 4)
    assert keys.tolist() == [0b1010, 0b0101, 0, 0b1000]


def _golden_rows(name):
    return [l.split() for l in open(os.path.join(GOLDEN, name)) if l[0] != "#"]


def test_mlhcc_caption_codes():
    """The codes printed for the MLHCC figure (Section 4.3), rebuilt from the cut nodes each ray
    passes.  The figure itself is not in the text, so its geometry is laid out here: eight top
    boxes side by side along x, each split into eight low boxes along x; a box is passed by a ray
    running along x when its y range holds the ray's y.  The low boxes of the top nodes the rays
    pass but that are not their representatives get other patterns, so a wrong choice of
    representative (the last node passed, say), swapped halves or a reversed bit order all change
    a code.  The caption names top node 3 as Ray1's representative while the text takes the
    first top node passed in HAD order (node 1 here); nodes 1 and 3 share a pattern, so the
    printed codes hold under either reading."""
    rows = _golden_rows("mlhcc_caption_codes.txt")
    assert len(rows) == 2
    bands = [(0.0, 1.0), (1.2, 2.0)]               # y band of Ray1, of Ray2
    nowhere = (5.0, 6.0)
    band_of = {}
    low_pattern = {t: "11111111" for t in range(8)}
    for r, (name, code, tops, lows) in enumerate(rows):
        met = [int(x) for x in tops.split(",")]
        for t in met:
            band_of[t] = bands[r]
        rep = met[0]
        low_pattern[rep] = "".join("1" if i in {int(x) for x in lows.split(",")} else "0" for i in range(8))
    low_pattern[3] = low_pattern[1]                # the caption's representative for Ray1
    low_pattern[4], low_pattern[5], low_pattern[7] = "10000001", "11110000", "11000000"
    tb, lb = [], []
    for t in range(8):
        y0, y1 = band_of.get(t, nowhere)
        tb.append([t, y0, 0, t + 1, y1, 1])
        for k in range(8):
            ly0, ly1 = (y0, y1) if low_pattern[t][k] == "1" and t in band_of else nowhere
            lb.append([t + k / 8, ly0, 0, t + (k + 1) / 8, ly1, 1])
    rays = np.array([[-1, 0.5, 0.5, 0, 1, 0, 0, np.inf],
                     [-1, 1.5, 0.5, 0, 1, 0, 0, np.inf]], np.float32)
    keys = O.encode_mlhcc(rays, np.asarray(tb, np.float32), np.asarray(lb, np.float32), 8, 16)
    assert [format(int(k), "016b") for k in keys] == [row[1] for row in rows]
    # the top half alone is the hierarchy cut code of the top boxes
    top_only = O.encode_hcc(rays, np.asarray(tb, np.float32), 8)
    assert [int(k) for k in top_only] == [int(row[1], 2) >> 8 for row in rows]

@pytest.mark.parametrize("top,low", [(8, 8), (16, 16), (4, 32), (30, 2)])
def test_mlhcc_cut_invariants(top, low):
    bvh = O.build_bvh(W.tiny_scene().tris)
    h = O.had(bvh)
    t, l = O.select_mlhcc_cut(bvh, h, top, low)
    assert 0 < t.size <= top
    assert [(-h[x], int(x)) for x in t] == sorted((-h[x], int(x)) for x in t)
    seen = set()
    for i, node in enumerate(t):
        under = set(leaves_under(bvh, int(node)))
        assert len(under) >= low                      # sufficient subtree
        assert not (under & seen)                     # top nodes are disjoint
        seen |= under
        row = [int(x) for x in l[i]]
        assert len(set(row)) == low
        assert [(-h[x], x) for x in row] == sorted((-h[x], x) for x in row)
        cover = []
        for x in row:
            cover += leaves_under(bvh, x)
        assert sorted(cover) == sorted(under)         # a cut of the top node's subtree


def test_mlhcc_key_consistent_with_hcc():
    bvh = O.build_bvh(W.tiny_scene().tris)
    h = O.had(bvh)
    top, low = 8, 8
    t, l = O.select_mlhcc_cut(bvh, h, top, low)
    tb = bvh.boxes[t]
    lb = bvh.boxes[l.reshape(-1)]
    rays = random_rays(1500, 31, 0.0, 1.0)
    rays[::4, 7] = 0.2
    keys = O.encode_mlhcc(rays, tb, lb, low, top + low).astype(np.uint64)
    top_bits = O.encode_hcc(rays, tb, top).astype(np.uint64)
    assert np.array_equal(keys >> np.uint64(low), top_bits)
    for r, k, tk in zip(rays, keys, top_bits):
        tk = int(tk)
        if tk == 0:
            assert int(k) & ((1 << low) - 1) == 0
            continue
        rep = top - tk.bit_length()                   # first top node met, in HAD order
        lo_bits = int(O.encode_hcc(r[None], bvh.boxes[l[rep]], low)[0])
        assert int(k) & ((1 << low) - 1) == lo_bits


def test_grid_boxes_tile_the_scene():
    lohi = O.scene_box(W.tiny_scene().tris)
    for k in (16, 24, 32, 48, 64):
        gx, gy, gz = O.grid_dims(k)
        assert gx * gy * gz == k and gx >= gy >= gz
        b = O.grid_boxes(lohi, gx, gy, gz).reshape(gz, gy, gx, 6)
        assert np.array_equal(b[..., 0, :3][..., 0], np.full((gz, gy), lohi[0]))
        assert np.all(b[:, :, -1, 3] == lohi[3]) and np.all(b[:, -1, :, 4] == lohi[4]) and np.all(b[-1, :, :, 5] == lohi[5])
        assert np.array_equal(b[:, :, 1:, 0], b[:, :, :-1, 3])      # neighbours share faces exactly
        assert np.array_equal(b[:, 1:, :, 1], b[:, :-1, :, 4])
        assert np.array_equal(b[1:, :, :, 2], b[:-1, :, :, 5])
        vol = np.prod(b[..., 3:].astype(np.float64) - b[..., :3], axis=-1).sum()
        assert vol == pytest.approx(np.prod(lohi[3:].astype(np.float64) - lohi[:3]), rel=1e-6)


def test_grid_key_single_cell_segments():
    lohi = np.array([0, 0, 0, 4, 4, 2], np.float32)
    boxes = O.grid_boxes(lohi, 4, 4, 2)
    rays = []
    for cell in range(32):
        x, y, z = cell % 4, (cell // 4) % 4, cell // 16
        rays.append([x + 0.3, y + 0.4, z + 0.45, 0, 0.2, 0.1, 0.05, 1.0])   # short segment inside the cell
    keys = O.encode_hcc(np.array(rays, np.float32), boxes, 32)
    assert keys.tolist() == [1 << (31 - c) for c in range(32)]


# ----------------------------------------------------------------------------- prefix path code

def _ppc_walk(bvh, ray, key_bits):
    """The forced-order walk written recursively: expanding a node tests child 0 then child 1;
    child 0's subtree is finished before child 1's."""
    from test_oracle import _np_slab
    seq = []

    def expand(node):
        met = []
        for c in bvh.child[node]:
            if len(seq) == key_bits:
                return
            h = _np_slab(ray, bvh.boxes[int(c)])
            seq.append(h)
            met.append((int(c), h))
        for c, h in met:
            if len(seq) == key_bits:
                return
            if h and not bvh.is_leaf(c):
                expand(c)

    if bvh.n == 1:
        seq.append(_np_slab(ray, bvh.boxes[0]))
    else:
        expand(0)
    return sum(1 << (key_bits - 1 - i) for i, h in enumerate(seq) if h)


def test_ppc_hand_example():
    bvh = O.build_bvh(_four_triangles())          # root -> (1, 2); 1 -> (T0, T2); 2 -> (T1, T3)
    rays = np.array([[0.05, 0.03, -1, 0, 0, 0, 1, np.inf],     # T0: 1 met, 2 not; then T0 met, T2 not
                     [0.9, 0.9, -1, 0, 0, 0, 1, np.inf],       # T3: 1 not, 2 met; then T1 not, T3 met
                     [0.5, 0.5, -1, 0, 0, 0, 1, np.inf],       # nothing
                     [0.05, 0.5, -1, 0, 0, 0, 1, np.inf]],     # node 1's box only
                    np.float32)
    assert O.encode_ppc(bvh, rays, 4).tolist() == [0b1010, 0b0101, 0, 0b1000]
    assert O.encode_ppc(bvh, rays, 6).tolist() == [0b101000, 0b010100, 0, 0b100000]
    assert O.encode_ppc(bvh, rays, 3).tolist() == [0b101, 0b010, 0, 0b100]   # walk cut after 3 tests
    one = O.build_bvh(_four_triangles()[:1])
    assert O.encode_ppc(one, rays[:3], 5).tolist() == [0b10000, 0, 0]



def test_ppc_caption_code():
    """The 4-bit prefix path code printed for the PPC figure (Section 4.1): tests true, true,
    false, false give 1100.  Scene: the four corner triangles of the unit square, tilted so that
    their boxes have depth; the root's children are the left column (triangles 0, 2) and the right
    column (1, 3).  A ray along x at mid height passes both columns' boxes but neither triangle of
    the left column, so the walk tests: left column (1), right column (1), then, expanding the left
    column, its two triangles (0, 0).  Testing the root as well, a breadth-first walk past four
    bits, or the bits reversed would each give another code."""
    (bits, code, seq), = _golden_rows("ppc_caption_code.txt")
    a = 0.125
    tris = np.asarray([[x, y, 0, x + a, y, a, x, y + a, a]
                       for (x, y) in [(0, 0), (0.875, 0), (0, 0.875), (0.875, 0.875)]], np.float32)
    bvh = O.build_bvh(tris)
    assert list(bvh.leaf_prim) == [0, 2, 1, 3] and bvh.child.tolist() == [[1, 2], [3, 4], [5, 6]]
    ray = np.array([[-1, 0.5, a / 2, 0, 1, 0, 0, np.inf]], np.float32)
    assert format(int(O.encode_ppc(bvh, ray, int(bits))[0]), "0%sb" % bits) == code
    assert [int(x) for x in seq.split(",")] == [int(c) for c in code]
    # the walk goes on into the right column, whose two triangles the ray also misses
    assert format(int(O.encode_ppc(bvh, ray, 6)[0]), "06b") == "110000"

@pytest.mark.parametrize("key_bits", [1, 7, 16, 32, 64])
def test_ppc_matches_recursive_walk(key_bits):
    bvh = O.build_bvh(W.tiny_scene().tris)
    rays = random_rays(400, 17, 0.0, 1.0)
    rays[::3, 7] = 0.15
    keys = O.encode_ppc(bvh, rays, key_bits)
    for r, k in zip(rays, keys):
        assert int(k) == _ppc_walk(bvh, r, key_bits)


def test_ppc_prefix_property_and_scale():
    bvh = O.build_bvh(W.tiny_scene().tris)
    rays = random_rays(600, 19, 0.0, 1.0)
    k64 = O.encode_ppc(bvh, rays, 64).astype(np.uint64)
    for kb in (8, 20, 33, 63):
        assert np.array_equal(k64 >> np.uint64(64 - kb), O.encode_ppc(bvh, rays, kb).astype(np.uint64))
    big = O.build_bvh(W.tiny_scene().tris * np.float32(4.0))
    r4 = rays.copy()
    r4[:, 0:3] *= 4.0
    assert np.array_equal(O.encode_ppc(big, r4, 64), k64)


# ----------------------------------------------------------------------------- shorter sorts

def test_sort_prefix_definition():
    rng = np.random.default_rng(3)
    keys = rng.integers(0, 1 << 20, 3000).astype(np.uint32)
    for skip in (0, 4, 8, 13, 20):
        perm = O.sort_prefix(keys, 20, skip)
        expect = sorted(range(keys.size), key=lambda i: (int(keys[i]) >> skip, i))
        assert perm.tolist() == expect


def test_sort_tiles_definition():
    rng = np.random.default_rng(4)
    keys = rng.integers(0, 50, 1000).astype(np.uint64)
    for tile in (1, 64, 100, 999, 1000, 4096):
        perm = O.sort_tiles(keys, tile)
        expect = []
        for t0 in range(0, 1000, tile):
            idx = range(t0, min(1000, t0 + tile))
            expect += sorted(idx, key=lambda i: (int(keys[i]), i))
        assert perm.tolist() == expect
