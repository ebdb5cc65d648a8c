"""Pins for the oracle's multi-level hierarchy cut code (Section 4.3, Alg. 3) and the
regular-grid control encoding (Section 5)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from test_oracle import _four_triangles, leaves_under, random_rays


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
