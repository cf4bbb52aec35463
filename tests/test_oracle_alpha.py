"""Opacity masks (alpha-tested triangles: the accept / ignore decision of an
any-hit stage per point of a triangle) in the FP64 oracle, pinned by the
subdivision worked out by hand at levels 1 and 2, by the micro-triangles
partitioning the triangle into equal areas at every level, and by the
identities of empty and full masks."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from tests.helpers import ray, scene_from_meshes

# one triangle with u = x and v = y: (0,0,0), (1,0,0), (0,1,0) scaled by 4
TRI = [[(0, 0, 0), (4, 0, 0), (0, 4, 0)]]


def _down(points):
    return np.stack([ray((4 * x, 4 * y, 3.0), (0.0, 0.0, -1.0)) for x, y in points])


def _scene(mask, level, tris=TRI):
    sc = scene_from_meshes([sg.triangles_mesh(tris)])
    return oracle.Scene(sc, alpha=[(np.asarray(mask, np.uint64), level)])


def test_level_one_by_hand():
    """n = 2: micro-triangle 0 is x, y <= 1/2 below x + y = 1/2; 1 the
    inverted one above it in the same square; 2 the corner at x >= 1/2;
    3 the corner at y >= 1/2."""
    pts = [(0.1, 0.1), (0.4, 0.4), (0.7, 0.1), (0.1, 0.7)]
    for mask in range(16):
        res = _scene([mask], 1).trace(_down(pts))
        assert (res["amb"] == 0).all()
        assert list(res["hit"]) == [(mask >> k) & 1 for k in range(4)], mask


def test_level_two_by_hand():
    """n = 4, rows of 7, 5, 3, 1 micro-triangles: (x, y) -> index."""
    cases = {(0.05, 0.05): 0, (0.2, 0.2): 1, (0.3, 0.05): 2, (0.45, 0.2): 3, (0.55, 0.1): 4, (0.7, 0.2): 5,
             (0.8, 0.1): 6, (0.05, 0.3): 7, (0.2, 0.45): 8, (0.3, 0.3): 9, (0.45, 0.45): 10, (0.55, 0.3): 11,
             (0.05, 0.55): 12, (0.2, 0.7): 13, (0.3, 0.55): 14, (0.1, 0.8): 15}
    pts = list(cases)
    for k in range(16):
        res = _scene([1 << k], 2).trace(_down(pts))
        assert (res["amb"] == 0).all()
        assert [p for p, h in zip(pts, res["hit"]) if h] == [p for p in pts if cases[p] == k], k


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_micro_triangles_partition_the_triangle(level):
    """Rays through a fine grid of points inside the triangle: with one bit
    set, each point is accepted under exactly one bit (a partition), and each
    micro-triangle takes 1 / 4^level of the points up to the grid's edge
    effects."""
    g = (np.arange(160) + 0.5) / 160
    X, Y = np.meshgrid(g, g)
    inside = X + Y < 1.0 - 1e-3
    pts = list(zip(X[inside], Y[inside]))
    rays = _down(pts)
    n = 4 ** level
    hits = np.zeros((n, len(pts)), np.uint8)
    ok = np.ones(len(pts), bool)
    for k in range(n):
        res = _scene([1 << k], level).trace(rays)
        hits[k] = res["hit"]
        ok &= res["amb"] == 0
    assert ok.mean() > 0.9
    assert (hits[:, ok].sum(axis=0) == 1).all()
    share = hits[:, ok].sum(axis=1) / ok.sum()
    assert np.allclose(share, 1.0 / n, rtol=0.08)


def test_empty_and_full_masks():
    sc = sg.config_small()
    rays = sg.random_rays(3000, 5, extent=1.5)
    base = oracle.Scene(sc).trace(rays)
    full = oracle.Scene(sc, alpha=[(np.full(sc.blas[0].n_tris, ~np.uint64(0)), 3)]).trace(rays)
    for k in ("hit", "inst", "prim", "t", "u", "v", "amb"):
        assert np.array_equal(base[k], full[k]), k
    empty = oracle.Scene(sc, alpha=[(np.zeros(sc.blas[0].n_tris, np.uint64), 2)]).trace(rays, any_hit=True)
    assert empty["hit"].sum() == 0 and empty["amb"].sum() == 0


@pytest.mark.parametrize("seed", [7])
def test_complementary_masks_split_the_hits(seed):
    """The closest hit without masks lies on one micro-triangle: under a mask
    M it is kept when that micro-triangle's bit is set, and under ~M
    otherwise; the any hit without masks is the OR of the any hits under M
    and ~M where nothing is ambiguous."""
    rng = np.random.default_rng(seed)
    mesh = sg.random_soup(400, seed, 1.0, 0.5)
    sc = scene_from_meshes([mesh])
    M = rng.integers(0, 2 ** 63, mesh.n_tris, dtype=np.int64).astype(np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, mesh.n_tris).astype(np.uint64)
    rays = sg.random_rays(4000, seed + 1, extent=1.5)
    a = oracle.Scene(sc).trace(rays)
    m1 = oracle.Scene(sc, alpha=[(M, 3)]).trace(rays)
    m2 = oracle.Scene(sc, alpha=[(~M, 3)]).trace(rays)
    ok = (a["amb"] == 0) & (m1["amb"] == 0) & (m2["amb"] == 0) & (a["hit"] == 1)
    assert ok.sum() > 500
    kept1 = ok & (m1["hit"] == 1) & (m1["prim"] == a["prim"]) & (m1["t"] == a["t"])
    kept2 = ok & (m2["hit"] == 1) & (m2["prim"] == a["prim"]) & (m2["t"] == a["t"])
    assert np.array_equal(kept1 | kept2, ok) and not (kept1 & kept2).any()
    o = [oracle.Scene(sc, alpha=al).trace(rays, any_hit=True) for al in (None, [(M, 3)], [(~M, 3)])]
    ok = (o[0]["amb"] == 0) & (o[1]["amb"] == 0) & (o[2]["amb"] == 0)
    assert np.array_equal(o[0]["hit"][ok], (o[1]["hit"] | o[2]["hit"])[ok])
