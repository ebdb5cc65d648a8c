"""Property-based pins for the CPU oracle (hypothesis): the same kinds of checks as the hand-made
pins, over scenes, rays and parameters that hypothesis draws (scene sizes from one triangle up,
many equal Morton codes, segments, cut and key sizes from 1 up, power-of-two scalings).

Each property is fixed by the mathematics or by the paper, not by the oracle's code: Python's
stable sort, a different BVH construction algorithm (Karras 2012), brute force over every
triangle, the definition of a cut (every leaf under exactly one cut node), exact invariance of
float32 arithmetic under scaling by powers of two, and the prefix structure of the prefix path
code (Section 4.1) and of the multi-level code's top half (Section 4.3)."""
import numpy as np
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle as O
from test_oracle import karras_tree, leaves_under, random_rays, random_tris

MISS = O.MISS
FAST = settings(max_examples=120, deadline=None, suppress_health_check=[HealthCheck.too_slow])

seeds = st.integers(min_value=0, max_value=2**31 - 1)


# ----------------------------------------------------------------------------- sorts

key_lists = st.one_of(
    st.lists(st.integers(min_value=0, max_value=2**64 - 1), max_size=300),
    st.lists(st.integers(min_value=0, max_value=7), max_size=300),          # many equal keys
)


@FAST
@given(keys=key_lists)
def test_prop_sort_is_pythons_stable_sort(keys):
    k = np.asarray(keys, np.uint64)
    assert O.sort(k).tolist() == sorted(range(len(keys)), key=lambda i: keys[i])


@FAST
@given(keys=st.lists(st.integers(min_value=0, max_value=2**32 - 1), max_size=300),
       skip=st.integers(min_value=0, max_value=32))
def test_prop_sort_prefix_ignores_the_low_bits(keys, skip):
    """Sections 6.5 / 6.6.1: the shortened sort orders by the key's top bits only, stably."""
    k = np.asarray(keys, np.uint32)
    assert O.sort_prefix(k, 32, skip).tolist() == sorted(range(len(keys)), key=lambda i: keys[i] >> skip)


@FAST
@given(keys=st.lists(st.integers(min_value=0, max_value=15), max_size=400),
       tile=st.sampled_from([1, 2, 3, 64, 256]))
def test_prop_tile_sort_sorts_each_tile_alone(keys, tile):
    k = np.asarray(keys, np.uint32)
    want = []
    for t0 in range(0, len(keys), tile):
        want += sorted(range(t0, min(t0 + tile, len(keys))), key=lambda i: keys[i])
    assert O.sort_tiles(k, tile).tolist() == want


# ----------------------------------------------------------------------------- LBVH

@FAST
@given(n=st.integers(min_value=2, max_value=300), seed=seeds, dup=st.booleans())
def test_prop_lbvh_equals_karras_construction(n, seed, dup):
    bvh = O.build_bvh(random_tris(n, seed, dup))
    assert np.array_equal(bvh.child, karras_tree(bvh.codes))


# ----------------------------------------------------------------------------- cut (Algorithm 2)

@FAST
@given(n=st.integers(min_value=1, max_value=200), seed=seeds, dup=st.booleans(),
       cut_size=st.integers(min_value=1, max_value=220))
def test_prop_cut_is_a_cut_in_had_order(n, seed, dup, cut_size):
    bvh = O.build_bvh(random_tris(n, seed, dup))
    h = O.had(bvh)
    cut = O.select_cut(bvh, h, cut_size)
    assert len(cut) == min(cut_size, n)
    cover = np.zeros(n, np.int64)
    for c in cut:
        for leaf in leaves_under(bvh, int(c)):
            cover[leaf - (n - 1)] += 1
    assert (cover == 1).all()
    pairs = [(-h[c], int(c)) for c in cut]
    assert pairs == sorted(pairs)


# ----------------------------------------------------------------------------- trace

@FAST
@given(n=st.integers(min_value=1, max_value=64), seed=seeds, dup=st.booleans(),
       short=st.booleans())
def test_prop_trace_equals_brute_force(n, seed, dup, short):
    tris = random_tris(n, seed, dup)
    rays = random_rays(96, seed ^ 0x5A5A, 0.0, 1.0, tmax=0.3 if short else np.inf)
    bvh = O.build_bvh(tris)
    h = O.trace(bvh, rays)
    bf = O.brute_force(tris, rays)
    assert np.array_equal(h.t, bf.t)
    for i in np.nonzero(h.prim != bf.prim)[0]:       # another triangle only at an exact tie in t
        assert h.prim[i] != MISS and bf.prim[i] != MISS
    occ = O.trace(bvh, rays, closest=False)
    assert np.array_equal(occ, (bf.prim != MISS).astype(np.uint8))


def _scaled(tris, rays, e):
    s = np.float32(2.0 ** e)
    r = rays.copy()
    r[:, 0:4] *= s                                    # origin and t_min
    r[:, 7] *= s                                      # t_max
    return tris * s, r


@FAST
@given(n=st.integers(min_value=1, max_value=120), seed=seeds, e=st.integers(min_value=-8, max_value=8),
       cut_size=st.integers(min_value=1, max_value=64))
def test_prop_power_of_two_scaling(n, seed, e, cut_size):
    """Scaling the scene and the ray origins by 2^e changes no Morton code, no HAD order, no slab
    or triangle decision: BVH, cut, HCC / PPC keys and hit triangles stay, hit distances scale."""
    tris = random_tris(n, seed)
    rays = random_rays(64, seed ^ 0x33, 0.0, 1.0)
    rays[::2, 7] = 0.4
    t2, r2 = _scaled(tris, rays, e)
    b1, b2 = O.build_bvh(tris), O.build_bvh(t2)
    assert np.array_equal(b1.child, b2.child) and np.array_equal(b1.leaf_prim, b2.leaf_prim)
    c1 = O.select_cut(b1, O.had(b1), cut_size)
    assert np.array_equal(c1, O.select_cut(b2, O.had(b2), cut_size))
    kb = min(64, len(c1))
    assert np.array_equal(O.encode_hcc(rays, O.cut_boxes(b1, c1), kb),
                          O.encode_hcc(r2, O.cut_boxes(b2, c1), kb))
    assert np.array_equal(O.encode_ppc(b1, rays, 32), O.encode_ppc(b2, r2, 32))
    h1, h2 = O.trace(b1, rays), O.trace(b2, r2)
    assert np.array_equal(h1.prim, h2.prim)
    hit = h1.prim != MISS
    assert np.array_equal(h1.t[hit] * np.float32(2.0 ** e), h2.t[hit])


# ----------------------------------------------------------------------------- key structure

@FAST
@given(n=st.integers(min_value=1, max_value=120), seed=seeds,
       kb=st.integers(min_value=1, max_value=64), k=st.integers(min_value=1, max_value=64))
def test_prop_ppc_prefix(n, seed, kb, k):
    """Section 4.1: the code is the first tests of one fixed walk, so a shorter code is the
    longer code's top bits."""
    k = min(k, kb)
    bvh = O.build_bvh(random_tris(n, seed))
    rays = random_rays(64, seed ^ 0x77, 0.0, 1.0)
    long = O.encode_ppc(bvh, rays, kb).astype(np.uint64)
    short = O.encode_ppc(bvh, rays, k).astype(np.uint64)
    assert np.array_equal(long >> np.uint64(kb - k), short)


@FAST
@given(n=st.integers(min_value=16, max_value=200), seed=seeds,
       top=st.integers(min_value=1, max_value=16), low=st.integers(min_value=1, max_value=8))
def test_prop_mlhcc_top_half_is_the_hcc_of_the_top_nodes(n, seed, top, low):
    """Section 4.3: the upper bits are the hierarchy cut code of the top-level nodes (ordered by
    HAD); the low bits are zero for a ray that passes no top node, and otherwise the code of the
    low-level boxes of the passed top node with the highest HAD, i.e. the first one passed."""
    bvh = O.build_bvh(random_tris(n, seed))
    t, l = O.select_mlhcc_cut(bvh, O.had(bvh), top, low)
    te = len(t)
    kb = te + low
    rays = random_rays(96, seed ^ 0x99, 0.0, 1.0)
    keys = O.encode_mlhcc(rays, bvh.boxes[t], bvh.boxes[l.reshape(-1)], low, kb).astype(np.uint64)
    hcc = O.encode_hcc(rays, bvh.boxes[t], te).astype(np.uint64)
    assert np.array_equal(keys >> np.uint64(low), hcc)
    low_bits = keys & np.uint64((1 << low) - 1)
    assert not low_bits[hcc == 0].any()
    for i in np.nonzero(hcc)[0]:
        per_top = [int(O.encode_hcc(rays[i:i + 1], bvh.boxes[l[j]], low)[0]) for j in range(te)
                   if (int(hcc[i]) >> (te - 1 - j)) & 1]
        assert int(low_bits[i]) == per_top[0]
