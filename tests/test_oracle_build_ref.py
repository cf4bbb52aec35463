"""Pins of the plain build-step definitions (linear BVH after Karras 2012):
Morton interleave, stable sort, the radix-tree split rule and the refit."""
import numpy as np
import pytest

import scenegen as sg
from oracle import build_ref as br


def test_interleave_single_bits():
    q = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [2, 0, 0], [2 ** 21 - 1] * 3], np.uint64)
    k = br.interleave(q)
    assert list(k[:4]) == [4, 2, 1, 32]
    assert int(k[4]) == 2 ** 63 - 1


def test_quantise_extremes():
    c = np.array([[0, 0, 0], [1, 2, 3], [0.5, 1, 1.5]], np.float32)
    q = br.quantise(c, c.min(0), c.max(0))
    assert (q[0] == 0).all()
    assert (q[1] == 2 ** 21 - 1).all()
    assert (q[2] == 2 ** 20).all()
    flat = np.array([[1, 5, 0], [2, 5, 0]], np.float32)   # a degenerate axis maps to 0
    q = br.quantise(flat, flat.min(0), flat.max(0))
    assert (q[:, 1] == 0).all() and (q[:, 2] == 0).all()


def test_compact_keys():
    """30-bit keys (10 bits per axis): hand values of the quantisation and the
    interleave, and the relation to the 63-bit keys: scaling by 2^21 is
    scaling by 2^10 times 2^11 exactly in float32, so each 10-bit coordinate
    is its 21-bit one shifted right by 11 and the 30-bit key is the 63-bit
    key's top 30 bits."""
    B = br.BITS_COMPACT
    q = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [2, 0, 0], [2 ** B - 1] * 3], np.uint64)
    k = br.interleave(q, B)
    assert list(k[:4]) == [4, 2, 1, 32]
    assert int(k[4]) == 2 ** 30 - 1
    c = np.array([[0, 0, 0], [1, 2, 3], [0.5, 1, 1.5], [0.25, 0.5, 0.75]], np.float32)
    qq = br.quantise(c, c.min(0), c.max(0), B)
    assert (qq[0] == 0).all() and (qq[1] == 1023).all() and (qq[2] == 512).all() and (qq[3] == 256).all()
    for seed, mesh in enumerate([sg.random_soup(3000, 61), sg.torus(40, 30, 1.0, 0.3, 0.05, 6.0, 62),
                                 sg.random_soup(500, 63, extent=1e-3, size=1e-4)]):
        k63 = br.morton_keys(mesh.verts, mesh.idx)
        k30 = br.morton_keys(mesh.verts, mesh.idx, B)
        assert k30.max() < 2 ** 30
        assert np.array_equal(k30, k63 >> np.uint64(33)), seed


def test_karras_figure_tree():
    """The 8-key example tree (5-bit keys 00001 00010 00100 00101 10011 11000
    11001 11110), split by hand at the highest differing bit."""
    keys = np.array([0b00001, 0b00010, 0b00100, 0b00101, 0b10011, 0b11000, 0b11001, 0b11110],
                    np.uint64)
    left, right, first, last = br.radix_tree(keys)
    L = lambda i: -(i + 1)  # noqa: E731
    expect = {0: (3, 4, 0, 7), 1: (L(0), L(1), 0, 1), 2: (L(2), L(3), 2, 3), 3: (1, 2, 0, 3),
              4: (L(4), 5, 4, 7), 5: (6, L(7), 5, 7), 6: (L(5), L(6), 5, 6)}
    for k, (l, r, f, la) in expect.items():
        assert (left[k], right[k], first[k], last[k]) == (l, r, f, la), k


def test_karras_duplicates_and_cover():
    rng = np.random.default_rng(0)
    keys = np.sort(rng.integers(0, 16, 200).astype(np.uint64))   # many duplicates
    left, right, first, last = br.radix_tree(keys)
    n = keys.shape[0]
    seen_leaf = np.zeros(n, int)
    seen_int = np.zeros(n - 1, int)
    for k in range(n - 1):
        assert first[k] == k or last[k] == k          # one end of the range is the node index
        for c in (left[k], right[k]):
            if c < 0:
                seen_leaf[-c - 1] += 1
            else:
                seen_int[c] += 1
        # children partition the parent's range
        lr = (first[left[k]], last[left[k]]) if left[k] >= 0 else (-left[k] - 1,) * 2
        rr = (first[right[k]], last[right[k]]) if right[k] >= 0 else (-right[k] - 1,) * 2
        assert lr[0] == first[k] and rr[1] == last[k] and lr[1] + 1 == rr[0]
    assert (seen_leaf == 1).all()
    assert seen_int[0] == 0 and (seen_int[1:] == 1).all()


def test_refit_contains_children():
    m = sg.random_soup(100, 3)
    keys = br.morton_keys(m.verts, m.idx)
    sk, order = br.sort_pairs(keys)
    assert (np.diff(sk.astype(np.float64)) >= 0).all()
    lo, hi = br.tri_boxes(m.verts, m.idx)
    lo, hi = lo[order], hi[order]
    left, right, first, last = br.radix_tree(sk)
    blo, bhi = br.refit(lo, hi, first, last)
    assert np.array_equal(blo[0], lo.min(0)) and np.array_equal(bhi[0], hi.max(0))
    for k in range(first.shape[0]):
        for c in (left[k], right[k]):
            clo, chi = (blo[c], bhi[c]) if c >= 0 else (lo[-c - 1], hi[-c - 1])
            assert (blo[k] <= clo).all() and (bhi[k] >= chi).all()


# ----------------------------------------------------------------- PLOC
def test_ploc_hand_case():
    """Four unit-section boxes along x at [0,1], [1,2], [4,5], [9,10]:
    union areas 2(2 dx + 1) give d(0,1) = 10, d(1,2) = 18, d(0,2) = 22,
    d(2,3) = 26.  Iteration 1 merges the mutual pair (0,1) into inner 2;
    iteration 2 pairs it with [4,5] (22 < 26) into inner 1; the root 0
    joins [9,10]."""
    lo = np.array([[0, 0, 0], [1, 0, 0], [4, 0, 0], [9, 0, 0]], np.float32)
    hi = lo + np.array([1, 1, 1], np.float32)
    left, right, blo, bhi, its = br.ploc(lo, hi, 3)
    assert left.tolist() == [1, 2, -1] and right.tolist() == [-4, -3, -2]
    assert its == 3
    assert blo[0].tolist() == [0, 0, 0] and bhi[0].tolist() == [10, 1, 1]
    assert bhi[1].tolist() == [5, 1, 1] and bhi[2].tolist() == [2, 1, 1]
    # radius 1 sees the same pairs here
    assert br.ploc(lo, hi, 1)[0].tolist() == [1, 2, -1]


def test_ploc_surface_area_float32():
    lo = np.array([[0.1, 0.2, 0.3]], np.float32)
    hi = np.array([[1.7, 2.9, 0.8]], np.float32)
    d = (hi - lo).astype(np.float32)
    expect = np.float32(2) * ((d[0, 0] * d[0, 1] + d[0, 1] * d[0, 2]) + d[0, 2] * d[0, 0])
    assert br.surface_area32(lo, hi)[0] == expect
    assert abs(float(br.surface_area32(lo, hi)[0]) - 2 * (1.6 * 2.7 + 2.7 * 0.5 + 0.5 * 1.6)) < 1e-5


@pytest.mark.parametrize("n,radius,seed", [(2, 1, 0), (3, 2, 1), (97, 4, 2), (600, 16, 3), (600, 1, 4)])
def test_ploc_structure(n, radius, seed):
    m = sg.random_soup(n, seed)
    lo, hi = br.tri_boxes(m.verts, m.idx)
    keys = br.morton_keys(m.verts, m.idx)
    _, order = br.sort_pairs(keys)
    slo, shi = lo[order], hi[order]
    left, right, blo, bhi, its = br.ploc(slo, shi, radius)
    # every leaf exactly once, every inner node except the root exactly once
    kids = np.concatenate([left, right])
    leaves = np.sort(-kids[kids < 0] - 1)
    assert np.array_equal(leaves, np.arange(n))
    inner = np.sort(kids[kids >= 0])
    assert np.array_equal(inner, np.arange(1, n - 1))
    # children are created before their parent: larger inner index
    assert all(c > k for k in range(n - 1) for c in (left[k], right[k]) if c >= 0)
    # inner box = exact union of the children's boxes
    def box(c):
        return (slo[-c - 1], shi[-c - 1]) if c < 0 else (blo[c], bhi[c])
    for k in range(n - 1):
        (a0, a1), (b0, b1) = box(left[k]), box(right[k])
        assert np.array_equal(blo[k], np.minimum(a0, b0)) and np.array_equal(bhi[k], np.maximum(a1, b1))
    # every iteration merges at least one pair (the globally closest neighbours)
    assert its <= n - 1
    # leaf order: a permutation under which every subtree is contiguous
    rank = br.leaf_order(left, right, n)
    assert np.array_equal(np.sort(rank), np.arange(n))
    def span(c):
        if c < 0:
            return rank[-c - 1], rank[-c - 1], 1
        l0, l1, ln = span(left[c])
        r0, r1, rn = span(right[c])
        assert l1 + 1 == r0                      # left subtree directly before the right one
        return l0, r1, ln + rn
    if n > 1:
        f, l, cnt = span(0)
        assert (f, l, cnt) == (0, n - 1, n)


def test_ploc_tighter_than_lbvh_on_a_mesh():
    """Not a theorem, a sanity pin on a smooth mesh: the summed inner-node
    area of the clustered tree is below the radix tree's."""
    mesh = sg.torus(40, 40, 1.0, 0.35, 0.0875, 6.0, 3001)
    lo, hi = br.tri_boxes(mesh.verts, mesh.idx)
    keys = br.morton_keys(mesh.verts, mesh.idx)
    skeys, order = br.sort_pairs(keys)
    slo, shi = lo[order], hi[order]
    left, right, first, last = br.radix_tree(skeys)
    klo, khi = br.refit(slo, shi, first, last)
    _, _, plo, phi, _ = br.ploc(slo, shi, 16)
    a_lbvh = br.surface_area32(klo, khi).astype(np.float64).sum()
    a_ploc = br.surface_area32(plo, phi).astype(np.float64).sum()
    assert a_ploc < 0.95 * a_lbvh
