"""Plain definitions of the hierarchy-build steps -- TEST INFRASTRUCTURE ONLY.

These are the steps of a linear BVH build (Morton-code LBVH, Karras 2012,
"Maximizing Parallelism in the Construction of BVHs, Octrees, and k-d
Trees"), written as their definitions in NumPy so that the GPU's build
kernels can be compared step by step.  The paper only says the bottom level
is built from the models' vertex data and the top level from instances and
their matrices (section 1); how the structure is built is this project's
choice, so these definitions are its specification:

  centroid  c = 0.5 * (lo + hi) of each triangle's box, float32
  bounds    lo_c, hi_c = exact min / max of the centroids
  quantise  q_k = min(floor((c_k - lo_k) * s_k), 2^B - 1) with
            s_k = 2^B / (hi_k - lo_k) (0 when hi_k == lo_k), every step
            float32 and rounded to nearest (no fused multiply-add); B = 21
            bits per axis, or B = 10 for the compact option
  key       3B-bit interleave (63 or 30 bits): bit 3i+2 <- x bit i,
            3i+1 <- y bit i, 3i <- z bit i
  sort      stable ascending by key
  hierarchy for the sorted keys, the unique binary radix tree: a range
            [first, last] splits after the last index whose key shares more
            leading bits with key[first] than key[last] does; duplicate keys
            are made distinct by appending the index (Karras's tie-break)
  refit     node box = exact min / max of its leaves' triangle boxes
"""
from __future__ import annotations

import numpy as np

BITS = 21          # bits per axis of the default keys
BITS_COMPACT = 10  # the compact option (30-bit keys)


def tri_boxes(verts: np.ndarray, idx: np.ndarray):
    v = verts.astype(np.float32)[idx.astype(np.int64)]     # [T,3,3]
    return v.min(axis=1), v.max(axis=1)


def centroids(verts, idx) -> np.ndarray:
    lo, hi = tri_boxes(verts, idx)
    return (np.float32(0.5) * (lo + hi)).astype(np.float32)


def quantise(c: np.ndarray, lo: np.ndarray, hi: np.ndarray, bits: int = BITS) -> np.ndarray:
    c = c.astype(np.float32)
    ext = (hi.astype(np.float32) - lo.astype(np.float32)).astype(np.float32)
    with np.errstate(divide="ignore"):
        s = np.where(ext > 0, np.float32(2 ** bits) / np.where(ext > 0, ext, np.float32(1)),
                     np.float32(0)).astype(np.float32)
    x = ((c - lo.astype(np.float32)).astype(np.float32) * s).astype(np.float32)
    q = np.floor(x).astype(np.int64)
    return np.clip(q, 0, 2 ** bits - 1).astype(np.uint64)


def interleave(q: np.ndarray, bits: int = BITS) -> np.ndarray:
    """Bit-by-bit interleave of three `bits`-bit integers (x highest)."""
    key = np.zeros(q.shape[0], np.uint64)
    for i in range(bits):
        for axis, shift in ((0, 2), (1, 1), (2, 0)):
            bit = (q[:, axis] >> np.uint64(i)) & np.uint64(1)
            key |= bit << np.uint64(3 * i + shift)
    return key


def morton_keys(verts, idx, bits: int = BITS) -> np.ndarray:
    c = centroids(verts, idx)
    return interleave(quantise(c, c.min(axis=0), c.max(axis=0), bits), bits)


def morton_keys_for_centroids(c: np.ndarray) -> np.ndarray:
    c = c.astype(np.float32)
    return interleave(quantise(c, c.min(axis=0), c.max(axis=0)))


def sort_pairs(keys: np.ndarray):
    order = np.argsort(keys, kind="stable")
    return keys[order], order.astype(np.uint32)


def _clz64(x: int) -> int:
    return 64 - int(x).bit_length()


def _delta(keys, i: int, j: int) -> int:
    """Common-prefix length of the index-augmented keys i and j."""
    ki, kj = int(keys[i]), int(keys[j])
    if ki != kj:
        return _clz64(ki ^ kj)
    return 64 + (32 - int(i ^ j).bit_length())


def radix_tree(keys: np.ndarray):
    """Karras's numbering: internal node k covers a range with one end at k;
    children encoded as +index (internal) or -(index+1) (leaf).
    Returns left[n-1], right[n-1], first[n-1], last[n-1] (int64)."""
    n = keys.shape[0]
    left = np.zeros(max(n - 1, 0), np.int64)
    right = np.zeros(max(n - 1, 0), np.int64)
    first = np.zeros(max(n - 1, 0), np.int64)
    last = np.zeros(max(n - 1, 0), np.int64)
    if n < 2:
        return left, right, first, last
    stack = [(0, 0, n - 1)]
    while stack:
        node, f, l = stack.pop()
        first[node], last[node] = f, l
        common = _delta(keys, f, l)
        # largest s in [f, l) whose prefix with f is longer than `common`
        lo, hi = f, l - 1
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if _delta(keys, f, mid) > common:
                lo = mid
            else:
                hi = mid - 1
        s = lo
        if s == f:
            left[node] = -(s + 1)
        else:
            left[node] = s
            stack.append((s, f, s))
        if s + 1 == l:
            right[node] = -(s + 1 + 1)
        else:
            right[node] = s + 1
            stack.append((s + 1, s + 1, l))
    return left, right, first, last


def refit(lo_sorted: np.ndarray, hi_sorted: np.ndarray, first, last):
    """Box of each internal node = min/max over its range of leaf boxes."""
    n_int = first.shape[0]
    blo = np.empty((n_int, 3), np.float32)
    bhi = np.empty((n_int, 3), np.float32)
    for k in range(n_int):
        blo[k] = lo_sorted[first[k]:last[k] + 1].min(axis=0)
        bhi[k] = hi_sorted[first[k]:last[k] + 1].max(axis=0)
    return blo, bhi


# ----------------------------------------------------------------------------
# Locally-ordered clustering (PLOC; Meister & Bittner 2018, "Parallel
# Locally-Ordered Clustering for Bounding Volume Hierarchy Construction")
# ----------------------------------------------------------------------------
def surface_area32(lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """2 (dx dy + dy dz + dz dx) of boxes, float32, left to right, no FMA."""
    d = (hi.astype(np.float32) - lo.astype(np.float32)).astype(np.float32)
    a = (d[..., 0] * d[..., 1]).astype(np.float32)
    b = (d[..., 1] * d[..., 2]).astype(np.float32)
    c = (d[..., 2] * d[..., 0]).astype(np.float32)
    return (np.float32(2.0) * ((a + b).astype(np.float32) + c).astype(np.float32)).astype(np.float32)


def ploc(lo_sorted: np.ndarray, hi_sorted: np.ndarray, radius: int):
    """Agglomerative clustering over the Morton-sorted leaves, as defined for
    this build:

      clusters  start as the leaves in sorted order (leaf p encoded -(p+1))
      distance  d(i, j) = float32 surface area of the union of the boxes
      nearest   n(i) = argmin over j in [i-radius, i+radius], j != i, of
                (d(i, j), j): ties go to the smaller index
      merge     i < n(i) and n(n(i)) == i: a new inner node with children
                (cluster i, cluster n(i)) takes position i, n(i) is dropped;
                the remaining clusters keep their order
      numbering the k-th merge (iterations in order, positions ascending
                within one) gets inner index n-2-k, so the root is 0

    Returns left, right (int64[n-1], Karras-style encoding), the inner boxes
    (lo, hi float32[n-1,3]) and the number of iterations."""
    n = lo_sorted.shape[0]
    left = np.zeros(max(n - 1, 0), np.int64)
    right = np.zeros(max(n - 1, 0), np.int64)
    blo = np.zeros((max(n - 1, 0), 3), np.float32)
    bhi = np.zeros((max(n - 1, 0), 3), np.float32)
    cid = -(np.arange(n, dtype=np.int64) + 1)
    clo = lo_sorted.astype(np.float32).copy()
    chi = hi_sorted.astype(np.float32).copy()
    next_id = n - 2
    its = 0
    while cid.shape[0] > 1:
        its += 1
        m = cid.shape[0]
        best_d = np.full(m, np.inf, np.float32)
        best_j = np.full(m, m, np.int64)
        for j_off in range(-radius, radius + 1):
            if j_off == 0:
                continue
            j = np.arange(m) + j_off
            ok = (j >= 0) & (j < m)
            jj = np.where(ok, j, 0)
            d = surface_area32(np.minimum(clo, clo[jj]), np.maximum(chi, chi[jj]))
            d = np.where(ok, d, np.float32(np.inf))
            better = ok & ((d < best_d) | ((d == best_d) & (jj < best_j)))
            best_d = np.where(better, d, best_d)
            best_j = np.where(better, jj, best_j)
        i = np.arange(m)
        mutual = best_j[best_j] == i
        merge = mutual & (i < best_j)
        a = i[merge]
        b = best_j[merge]
        ids = next_id - np.arange(a.shape[0])
        next_id -= a.shape[0]
        left[ids] = cid[a]
        right[ids] = cid[b]
        blo[ids] = np.minimum(clo[a], clo[b])
        bhi[ids] = np.maximum(chi[a], chi[b])
        cid[a] = ids
        clo[a] = blo[ids]
        chi[a] = bhi[ids]
        keep = np.ones(m, bool)
        keep[b] = False
        cid, clo, chi = cid[keep], clo[keep], chi[keep]
    return left, right, blo, bhi, its


def leaf_order(left: np.ndarray, right: np.ndarray, n: int) -> np.ndarray:
    """Rank of each leaf in the left-to-right order of the tree (the order
    the triangles are stored in, so that every subtree is a contiguous
    range)."""
    rank = np.zeros(n, np.int64)
    if n == 1:
        return rank
    k = 0
    stack = [0]
    while stack:
        c = stack.pop()
        if c < 0:
            rank[-c - 1] = k
            k += 1
        else:
            stack.append(right[c])
            stack.append(left[c])
    return rank


# Treelet restructuring (Karras & Aila 2013, "Fast Parallel Construction of
# High-Quality Bounding Volume Hierarchies")
# ----------------------------------------------------------------------------
def _subtree_leaves(left, right, n):
    """Leaf count below every inner node."""
    cnt = np.zeros(max(n - 1, 0), np.int64)

    def count(c):
        return 1 if c < 0 else cnt[c]

    for node in _post_order(left, right, n):
        cnt[node] = count(left[node]) + count(right[node])
    return cnt


def _post_order(left, right, n):
    """Inner nodes, every node after the inner nodes below it (children
    left before right)."""
    if n < 2:
        return []
    out, stack = [], [(0, False)]
    while stack:
        c, seen = stack.pop()
        if seen:
            out.append(c)
            continue
        stack.append((c, True))
        for k in (right[c], left[c]):
            if k >= 0:
                stack.append((k, False))
    return out


def optimal_treelet(lo: np.ndarray, hi: np.ndarray):
    """The binary tree over m <= 7 leaf boxes with the least sum of float32
    surface areas of its inner nodes (the surface-area cost the leaves do
    not change), by dynamic programming over the subsets S of the leaves:
    cost(S) = 0 for one leaf, else area(S) + min over the splits (P, S \\ P)
    of cost(P) + cost(S \\ P), P holding the lowest leaf of S and enumerated
    in increasing bit order, the first minimum kept; every sum float32.
    Returns cost, split (per subset bit mask) and the union boxes."""
    m = lo.shape[0]
    full = (1 << m) - 1
    slo = np.zeros((full + 1, 3), np.float32)
    shi = np.zeros((full + 1, 3), np.float32)
    area = np.zeros(full + 1, np.float32)
    for S in range(1, full + 1):
        bits = [k for k in range(m) if (S >> k) & 1]
        slo[S] = np.min(lo[bits], axis=0)
        shi[S] = np.max(hi[bits], axis=0)
        area[S] = surface_area32(slo[S], shi[S])
    cost = np.zeros(full + 1, np.float32)
    split = np.zeros(full + 1, np.int64)
    for S in sorted(range(1, full + 1), key=lambda s: (bin(s).count("1"), s)):
        if S & (S - 1) == 0:
            continue
        low = S & -S
        rest = S ^ low
        best, bp = np.float32(np.inf), 0
        Q = 0
        while True:
            P = low | Q
            if P != S:
                v = np.float32(cost[P] + cost[S ^ P])
                if v < best:
                    best, bp = v, P
            if Q == rest:
                break
            Q = (Q - rest) & rest
        cost[S] = np.float32(area[S] + best)
        split[S] = bp
    return cost, split, slo, shi


def treelet_optimise(left, right, leaf_lo, leaf_hi, int_lo, int_hi, rounds: int = 3, size: int = 7):
    """Rounds of treelet restructuring over a binary hierarchy (Karras-style
    encoding, leaves -(i+1)), as defined for this build:

      order     each round visits the inner nodes with at least three
                leaves below them, every node after the inner nodes below
                it (as the tree stood when the round began)
      treelet   starts as the node's two children; while it has fewer than
                `size` leaves, its inner leaf of largest float32 surface
                area (first in the list on ties) is replaced in place by its
                left child, its right child appended
      topology  optimal_treelet over the treelet's leaves
      rebuild   the node keeps its index; the treelet's other inner nodes
                take the replaced nodes' indices in increasing order, in
                pre-order of the new topology (left subtree first); inner
                boxes are the unions of their leaves' boxes

    Returns left, right, inner lo, inner hi (new arrays)."""
    left = np.array(left, np.int64)
    right = np.array(right, np.int64)
    blo = np.array(int_lo, np.float32)
    bhi = np.array(int_hi, np.float32)
    n = leaf_lo.shape[0]

    def box(c):
        return (leaf_lo[-c - 1], leaf_hi[-c - 1]) if c < 0 else (blo[c], bhi[c])

    for _ in range(rounds):
        cnt = _subtree_leaves(left, right, n)
        for node in _post_order(left, right, n):
            if cnt[node] < 3:
                continue
            leaves = [int(left[node]), int(right[node])]
            removed = []
            while len(leaves) < size:
                best_k, best_a = -1, np.float32(-np.inf)
                for k, c in enumerate(leaves):
                    if c >= 0:
                        a = surface_area32(blo[c], bhi[c])
                        if a > best_a:
                            best_k, best_a = k, a
                if best_k < 0:
                    break
                c = leaves[best_k]
                removed.append(c)
                leaves[best_k] = int(left[c])
                leaves.append(int(right[c]))
            m = len(leaves)
            lo = np.array([box(c)[0] for c in leaves], np.float32)
            hi = np.array([box(c)[1] for c in leaves], np.float32)
            _, split, slo, shi = optimal_treelet(lo, hi)
            ids = sorted(removed)
            nxt = 0
            full = (1 << m) - 1
            stack = [(full ^ int(split[full]), node, 1), (int(split[full]), node, 0)]
            while stack:
                T, parent, side = stack.pop()
                if T & (T - 1) == 0:
                    child = leaves[T.bit_length() - 1]
                else:
                    child = ids[nxt]
                    nxt += 1
                    blo[child], bhi[child] = slo[T], shi[T]
                    stack.append((T ^ int(split[T]), child, 1))
                    stack.append((int(split[T]), child, 0))
                if side == 0:
                    left[parent] = child
                else:
                    right[parent] = child
    return left, right, blo, bhi


def sah_cost(left, right, leaf_lo, leaf_hi, int_lo, int_hi) -> float:
    """Sum of inner-node surface areas over the root's (FP64)."""
    d = (int_hi.astype(np.float64) - int_lo.astype(np.float64))
    a = 2.0 * (d[:, 0] * d[:, 1] + d[:, 1] * d[:, 2] + d[:, 2] * d[:, 0])
    return float(a.sum() / a[0])
