"""Treelet restructuring in the build oracle (Karras & Aila 2013), pinned by
exhaustive enumeration of every binary tree over a few leaves (the dynamic
program finds the least surface-area cost), a three-leaf case decided by
hand, and the structural invariants of the restructured hierarchy (a binary
tree over all leaves, unions as boxes, the same root box, a cost that never
rises from round to round)."""
import itertools

import numpy as np
import pytest

import scenegen as sg
from oracle import build_ref as br


def _area64(lo, hi):
    d = np.asarray(hi, np.float64) - np.asarray(lo, np.float64)
    return 2.0 * (d[0] * d[1] + d[1] * d[2] + d[2] * d[0])


def _all_trees(items):
    """Every binary tree over the leaf indices in `items` (nested pairs)."""
    if len(items) == 1:
        yield items[0]
        return
    first, rest = items[0], items[1:]
    for k in range(len(rest)):
        for chosen in itertools.combinations(rest, k):
            lset = (first,) + chosen
            rset = tuple(x for x in rest if x not in chosen)
            if not rset:
                continue
            for lt in _all_trees(lset):
                for rt in _all_trees(rset):
                    yield (lt, rt)


def _tree_cost(t, lo, hi):
    """FP64 sum of inner-node union areas; returns (cost, leaves)."""
    if not isinstance(t, tuple):
        return 0.0, [t]
    ca, la = _tree_cost(t[0], lo, hi)
    cb, lb = _tree_cost(t[1], lo, hi)
    ls = la + lb
    return ca + cb + _area64(lo[ls].min(axis=0), hi[ls].max(axis=0)), ls


def _dp_cost(split, full, lo, hi):
    def rec(S):
        if S & (S - 1) == 0:
            return 0.0
        bits = [k for k in range(lo.shape[0]) if (S >> k) & 1]
        a = _area64(lo[bits].min(axis=0), hi[bits].max(axis=0))
        return a + rec(int(split[S])) + rec(S ^ int(split[S]))
    return rec(full)


@pytest.mark.parametrize("m,seed", [(2, 1), (3, 2), (4, 3), (5, 4), (5, 5), (6, 6)])
def test_dynamic_program_finds_the_best_tree(m, seed):
    rng = np.random.default_rng(seed)
    c = rng.uniform(-5, 5, (m, 3))
    ext = rng.uniform(0.1, 2.0, (m, 3))
    lo, hi = (c - ext).astype(np.float32), (c + ext).astype(np.float32)
    cost, split, _, _ = br.optimal_treelet(lo, hi)
    full = (1 << m) - 1
    best = min(_tree_cost(t, lo, hi)[0] for t in _all_trees(tuple(range(m))))
    assert _dp_cost(split, full, lo, hi) <= best * (1 + 1e-6)
    assert abs(float(cost[full]) - best) <= 1e-5 * best


def test_three_leaves_by_hand():
    """Far leaf A and two neighbours B, C: the best tree pairs B with C, so
    the root splits {A} from {B, C} (split mask 0b001)."""
    lo = np.array([[0, 0, 0], [10, 10, 10], [10.5, 10.5, 10.5]], np.float32)
    hi = lo + np.float32(1.0)
    cost, split, slo, shi = br.optimal_treelet(lo, hi)
    assert split[0b111] == 0b001 and split[0b110] == 0b010
    # cost: the root's area (11.5^2 * 6) plus the pair's (1.5^2 * 6)
    assert cost[0b111] == np.float32(6 * 11.5 ** 2 + 6 * 1.5 ** 2)
    assert np.array_equal(slo[0b110], [10, 10, 10]) and np.array_equal(shi[0b110], [11.5, 11.5, 11.5])


def _lbvh(mesh):
    keys = br.morton_keys(mesh.verts, mesh.idx)
    ks, ids = br.sort_pairs(keys)
    left, right, first, last = br.radix_tree(ks)
    lo, hi = br.tri_boxes(mesh.verts, mesh.idx)
    lo_s, hi_s = lo[ids], hi[ids]
    blo, bhi = br.refit(lo_s, hi_s, first, last)
    return left, right, lo_s, hi_s, blo, bhi


def _check_tree(left, right, lo, hi, blo, bhi):
    n = lo.shape[0]
    seen = np.zeros(n, np.int64)
    inner_seen = np.zeros(n - 1, np.int64)
    stack = [0]
    while stack:
        c = stack.pop()
        if c < 0:
            seen[-c - 1] += 1
            continue
        inner_seen[c] += 1
        kids = [left[c], right[c]]
        klo = [lo[-k - 1] if k < 0 else blo[k] for k in kids]
        khi = [hi[-k - 1] if k < 0 else bhi[k] for k in kids]
        assert np.array_equal(blo[c], np.minimum(klo[0], klo[1])) and np.array_equal(bhi[c], np.maximum(khi[0], khi[1]))
        stack.extend(kids)
    assert (seen == 1).all() and (inner_seen == 1).all()


@pytest.mark.parametrize("name", ["soup", "torus", "dupes"])
def test_restructured_hierarchy_invariants(name):
    mesh = {"soup": lambda: sg.random_soup(800, 21),
            "torus": lambda: sg.torus(24, 20, 1.0, 0.35, 0.08, 6.0, 3001),
            "dupes": lambda: sg.triangles_mesh(np.repeat(np.array([[[0, 0, 0], [1, 0, 0], [0, 1, 0]]]), 60, axis=0))}[name]()
    left, right, lo, hi, blo, bhi = _lbvh(mesh)
    L0, R0, B0, H0 = br.treelet_optimise(left, right, lo, hi, blo, bhi, rounds=0)
    assert np.array_equal(L0, left) and np.array_equal(R0, right) and np.array_equal(B0, blo)
    costs = [br.sah_cost(left, right, lo, hi, blo, bhi)]
    state = (left, right, blo, bhi)
    for r in range(2):
        state = br.treelet_optimise(state[0], state[1], lo, hi, state[2], state[3], rounds=1)
        _check_tree(state[0], state[1], lo, hi, state[2], state[3])
        assert np.array_equal(state[2][0], blo[0]) and np.array_equal(state[3][0], bhi[0])
        costs.append(br.sah_cost(state[0], state[1], lo, hi, state[2], state[3]))
    assert costs[1] <= costs[0] * (1 + 1e-6) and costs[2] <= costs[1] * (1 + 1e-6)
    if name != "dupes":
        assert costs[2] < 0.95 * costs[0]
    # two rounds at once are the two single rounds in a row
    both = br.treelet_optimise(left, right, lo, hi, blo, bhi, rounds=2)
    for a, b in zip(both, state):
        assert np.array_equal(a, b)
