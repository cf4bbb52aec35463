"""Pins of the plain build-step definitions (linear BVH after Karras 2012):
Morton interleave, stable sort, the radix-tree split rule and the refit."""
import numpy as np

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
