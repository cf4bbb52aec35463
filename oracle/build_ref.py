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
  quantise  q_k = min(floor((c_k - lo_k) * s_k), 2^21 - 1) with
            s_k = 2^21 / (hi_k - lo_k) (0 when hi_k == lo_k), every step
            float32 and rounded to nearest (no fused multiply-add)
  key       63-bit interleave: bit 3i+2 <- x bit i, 3i+1 <- y bit i,
            3i <- z bit i
  sort      stable ascending by key
  hierarchy for the sorted keys, the unique binary radix tree: a range
            [first, last] splits after the last index whose key shares more
            leading bits with key[first] than key[last] does; duplicate keys
            are made distinct by appending the index (Karras's tie-break)
  refit     node box = exact min / max of its leaves' triangle boxes
"""
from __future__ import annotations

import numpy as np

BITS = 21
Q = np.float32(2 ** BITS)


def tri_boxes(verts: np.ndarray, idx: np.ndarray):
    v = verts.astype(np.float32)[idx.astype(np.int64)]     # [T,3,3]
    return v.min(axis=1), v.max(axis=1)


def centroids(verts, idx) -> np.ndarray:
    lo, hi = tri_boxes(verts, idx)
    return (np.float32(0.5) * (lo + hi)).astype(np.float32)


def quantise(c: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    c = c.astype(np.float32)
    ext = (hi.astype(np.float32) - lo.astype(np.float32)).astype(np.float32)
    with np.errstate(divide="ignore"):
        s = np.where(ext > 0, Q / np.where(ext > 0, ext, np.float32(1)), np.float32(0)).astype(np.float32)
    x = ((c - lo.astype(np.float32)).astype(np.float32) * s).astype(np.float32)
    q = np.floor(x).astype(np.int64)
    return np.clip(q, 0, 2 ** BITS - 1).astype(np.uint64)


def interleave(q: np.ndarray) -> np.ndarray:
    """Bit-by-bit interleave of three 21-bit integers (x highest)."""
    key = np.zeros(q.shape[0], np.uint64)
    for i in range(BITS):
        for axis, shift in ((0, 2), (1, 1), (2, 0)):
            bit = (q[:, axis] >> np.uint64(i)) & np.uint64(1)
            key |= bit << np.uint64(3 * i + shift)
    return key


def morton_keys(verts, idx) -> np.ndarray:
    c = centroids(verts, idx)
    return interleave(quantise(c, c.min(axis=0), c.max(axis=0)))


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
