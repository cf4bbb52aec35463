"""Host-side structural checks of the hierarchy buffers (layout of include/rg.h):
every link in range, a tree (no node reached twice), every primitive in
exactly one leaf, and every box containing what lies below it."""
import numpy as np

LEAF = 0x80000000
EMPTY = 0xFFFFFFFF


def _nodes(buf: np.ndarray, off: int, n_nodes: int, W: int):
    raw = buf[off: off + n_nodes * 32 * W].view(np.float32).reshape(n_nodes, 8 * W)
    lo = np.stack([raw[:, 0:W], raw[:, W:2 * W], raw[:, 2 * W:3 * W]], -1)       # [n, W, 3]
    hi = np.stack([raw[:, 3 * W:4 * W], raw[:, 4 * W:5 * W], raw[:, 5 * W:6 * W]], -1)
    child = raw[:, 6 * W:7 * W].view(np.uint32)
    return lo, hi, child


def walk(lo, hi, child, n_prims: int, leaf_boxes, max_leaf: int):
    """Walks from the root; returns (depth, visits per primitive)."""
    n_nodes = child.shape[0]
    seen_node = np.zeros(n_nodes, np.int64)
    seen_prim = np.zeros(n_prims, np.int64)
    max_depth = 0
    stack = [(0, 1)]
    while stack:
        node, d = stack.pop()
        assert 0 <= node < n_nodes, f"node index {node} out of range"
        seen_node[node] += 1
        assert seen_node[node] == 1, f"node {node} reached twice"
        max_depth = max(max_depth, d)
        n_used = 0
        for k in range(child.shape[1]):
            c = int(child[node, k])
            if c == EMPTY:
                assert np.all(lo[node, k] == np.inf) and np.all(hi[node, k] == -np.inf)
                continue
            n_used += 1
            if c & LEAF:
                first, cnt = c & 0x0FFFFFFF, ((c >> 28) & 7) + 1
                assert cnt <= max_leaf
                assert first + cnt <= n_prims, "leaf range out of bounds"
                seen_prim[first: first + cnt] += 1
                blo = leaf_boxes[0][first: first + cnt].min(axis=0)
                bhi = leaf_boxes[1][first: first + cnt].max(axis=0)
                assert np.all(lo[node, k] <= blo) and np.all(hi[node, k] >= bhi), "leaf box too small"
            else:
                assert 0 <= c < n_nodes
                cl, ch = lo[c], hi[c]
                m = child[c] != EMPTY
                assert np.all(lo[node, k] <= cl[m].min(axis=0)) and np.all(hi[node, k] >= ch[m].max(axis=0))
                stack.append((c, d + 1))
        assert n_used >= 1
    assert (seen_node == 1).all(), "unreachable nodes"
    return max_depth, seen_prim


LEVELS_CAP = 255   # RG_LEVELS_CAP


def _check_levels_and_parents(buf: np.ndarray, desc, child: np.ndarray):
    """Nodes are numbered level by level: the level table's entry l is the
    first node at depth l (root 0) and entry `depth` the node count; each
    node's parent link names the node and child slot that point to it."""
    n_nodes, depth = desc.n_nodes, desc.depth
    parents = buf[desc.parents_off: desc.parents_off + 4 * n_nodes].view(np.uint32)
    assert parents[0] == EMPTY, "the root has no parent"
    node_depth = np.full(n_nodes, -1, np.int64)
    node_depth[0] = 0
    for node in range(n_nodes):       # parents precede their children
        assert node_depth[node] >= 0, f"node {node} numbered before its parent"
        for k in range(child.shape[1]):
            c = int(child[node, k])
            if c == EMPTY or c & LEAF:
                continue
            assert c > node
            node_depth[c] = node_depth[node] + 1
            assert parents[c] == (node << 3) | k, f"parent link of node {c}"
    assert node_depth.max() + 1 == depth
    if depth <= LEVELS_CAP:
        levels = buf[desc.levels_off: desc.levels_off + 4 * (depth + 1)].view(np.uint32).astype(np.int64)
        assert levels[0] == 0 and levels[depth] == n_nodes
        assert np.array_equal(np.searchsorted(levels, np.arange(n_nodes), side="right") - 1, node_depth), \
            "level table"


def check_blas(buf: np.ndarray, desc, refitted: bool = False) -> dict:
    W = desc.width
    lo, hi, child = _nodes(buf, desc.nodes_off, desc.n_nodes, W)
    n = desc.n_tris
    tri = buf[desc.tris_off: desc.tris_off + 40 * n].view(np.float32).reshape(n, 10)
    v = tri[:, :9].reshape(n, 3, 3)
    depth, seen = walk(lo, hi, child, n, (v.min(axis=1), v.max(axis=1)), desc.leaf_max)
    assert (seen == 1).all(), "each triangle must sit in exactly one leaf"
    assert depth == desc.depth
    prim = tri[:, 9].view(np.uint32)
    assert np.array_equal(np.sort(prim), np.arange(n, dtype=np.uint32)), "leaf order is a permutation"
    slots = buf[desc.slots_off: desc.slots_off + 4 * n].view(np.uint32)
    assert np.array_equal(slots[prim], np.arange(n, dtype=np.uint32)), "slots invert the leaf order"
    # the root box in the header (kept current by refits) is the union of the
    # triangles, and so is the descriptor's unless the level was refitted
    root = buf[32:56].view(np.float32)
    assert np.array_equal(root[:3], v.reshape(-1, 3).min(axis=0))
    assert np.array_equal(root[3:], v.reshape(-1, 3).max(axis=0))
    assert buf[56:60].view(np.uint32)[0] == 0, "status of the last refit"
    _check_levels_and_parents(buf, desc, child)
    if not refitted:
        assert np.array_equal(np.array(desc.lo, np.float32), root[:3])
        assert np.array_equal(np.array(desc.hi, np.float32), root[3:])
    hdr = buf[0:32].view(np.uint64)
    return dict(depth=depth, n_nodes=desc.n_nodes, prim=prim, verts=v, tri_mats=buf[
        desc.mats_off: desc.mats_off + 2 * n].view(np.uint16), header=hdr)


def check_tlas(buf: np.ndarray, desc, blas_descs, xform, roots=None, inst_flags=None) -> dict:
    W = desc.width
    lo, hi, child = _nodes(buf, desc.nodes_off, desc.n_nodes, W)
    n = desc.n_inst
    rec = buf[desc.inst_off: desc.inst_off + 112 * n]
    recf = rec.view(np.float32).reshape(n, 28)
    recu = rec.view(np.uint32).reshape(n, 28)
    inst = recu[:, 19]
    assert np.array_equal(np.sort(inst), np.arange(n, dtype=np.uint32))
    rec_of = buf[desc.rec_off: desc.rec_off + 4 * n].view(np.uint32)
    assert np.array_equal(rec_of[inst], np.arange(n, dtype=np.uint32))
    # instance world boxes from the leaf boxes in the nodes: gather per record
    boxes_lo = np.full((n, 3), np.inf, np.float32)
    boxes_hi = np.full((n, 3), -np.inf, np.float32)
    for node in range(desc.n_nodes):
        for k in range(W):
            c = int(child[node, k])
            if c != EMPTY and (c & LEAF):
                first = c & 0x0FFFFFFF
                assert ((c >> 28) & 7) == 0, "one instance per leaf"
                boxes_lo[first] = lo[node, k]
                boxes_hi[first] = hi[node, k]
    depth, seen = walk(lo, hi, child, n, (boxes_lo, boxes_hi), 1)
    assert (seen == 1).all() and depth == desc.depth
    X = np.asarray(xform, np.float64).reshape(-1, 3, 4)
    for r in range(n):
        i = inst[r]
        # the record's inverse is the inverse of the instance's linear part
        inv = recf[r, 0:9].reshape(3, 3).astype(np.float64)
        assert np.allclose(inv @ X[i, :, :3], np.eye(3), atol=1e-5)
        assert np.array_equal(recf[r, 9:12], X[i, :, 3].astype(np.float32))
    # each record carries its bottom level's root box (the current one, from
    # roots, after refits; else the descriptor's)
    if roots is None:
        roots = [(b.lo, b.hi) for b in blas_descs]
    by_nodes = {int(b.buf) + int(b.nodes_off): rb for b, rb in zip(blas_descs, roots)}
    rec_nodes = rec.view(np.uint64).reshape(n, 14)[:, 6]
    for r in range(n):
        rlo, rhi = by_nodes[int(rec_nodes[r])]
        assert np.array_equal(recf[r, 20:23], np.array(rlo, np.float32))
        assert np.array_equal(recf[r, 23:26], np.array(rhi, np.float32))
    # the instance flags word (visibility mask, cull flags); all visible by default
    want = np.full(n, 0xFF, np.uint32) if inst_flags is None else np.asarray(inst_flags, np.uint32)
    assert np.array_equal(recu[:, 26], want[inst])
    return dict(depth=depth, inst=inst, boxes=(boxes_lo, boxes_hi))
