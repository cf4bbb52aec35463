"""Pins of the FP64 oracle's ray-triangle outcome (closest hit / miss per ray,
paper section 1) against exact rational arithmetic and hand-derived cases."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import scenegen as sg
from oracle import exact
from tests.helpers import ray, tri_scene

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "triangle_hand_cases.json")


def _load():
    with open(GOLDEN) as f:
        return json.load(f)


def _tmax(s):
    return np.inf if s == "inf" else float(Fraction(s))


@pytest.mark.parametrize("case", _load()["cases"], ids=lambda c: c["name"])
def test_hand_case_exact(case):
    g = _load()
    a, b, c = g["triangle"]
    r = exact.intersect(case["o"], case["d"], a, b, c, 0, _tmax(case["tmax"]))
    if not case["hit"]:
        assert r is None
        return
    assert r == (Fraction(case["t"]), Fraction(case["u"]), Fraction(case["v"]))


@pytest.mark.parametrize("case", _load()["cases"], ids=lambda c: c["name"])
def test_hand_case_oracle(case):
    g = _load()
    sc = tri_scene([g["triangle"]])
    res = oracle.Scene(sc).trace(ray(case["o"], case["d"], 0.0, _tmax(case["tmax"]))[None])
    assert bool(res["hit"][0]) == case["hit"]
    if case["hit"]:
        assert res["t"][0] == pytest.approx(float(Fraction(case["t"])), abs=1e-12)
        assert res["u"][0] == pytest.approx(float(Fraction(case["u"])), abs=1e-12)
        assert res["v"][0] == pytest.approx(float(Fraction(case["v"])), abs=1e-12)
        assert res["inst"][0] == 0 and res["prim"][0] == 0
    else:
        assert res["inst"][0] == oracle.MISS and res["prim"][0] == oracle.MISS
        assert np.isinf(res["t"][0])


@pytest.mark.parametrize("case", _load()["ground"]["cases"], ids=lambda c: c["name"])
def test_ground_plane(case):
    g = _load()["ground"]
    sc = tri_scene([g["P0"], g["P1"]])
    res = oracle.Scene(sc).trace(ray(case["o"], case["d"])[None])
    assert res["hit"][0] == 1
    assert res["prim"][0] == case["prim"]
    assert res["t"][0] == pytest.approx(float(Fraction(case["t"])), abs=1e-12)
    # closed form t = (-1 - o_y) / d_y
    assert res["t"][0] == pytest.approx((-1.0 - case["o"][1]) / case["d"][1], abs=1e-12)
    if "u" in case:
        assert res["u"][0] == pytest.approx(float(Fraction(case["u"])), abs=1e-12)
        assert res["v"][0] == pytest.approx(float(Fraction(case["v"])), abs=1e-12)
    if "tie" in case:
        ties = {int(res["ties"][0, k, 1]) for k in range(res["nties"][0])}
        assert ties == set(case["tie"])
        assert res["amb"][0] == 1  # a shared edge lies inside every error band
    # the exact solver agrees on the hit primitive
    tris = [(0, 0, *g["P0"]), (0, 1, *g["P1"])]
    best = exact.closest(case["o"], case["d"], tris)
    assert best[2] == case["prim"] and best[0] == Fraction(case["t"])


def _f32(x):
    return np.asarray(x, np.float32)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_random_soup_vs_exact(seed):
    """Brute force on tiny inputs: FP64 oracle == exact rationals."""
    mesh = sg.random_soup(24, seed, extent=1.0, size=0.5)
    V32 = mesh.verts.astype(np.float64)
    cen = V32[mesh.idx].mean(axis=1)
    rays = np.concatenate([sg.random_rays(80, seed + 100, extent=1.5),
                           sg.rays_through_points(np.repeat(cen, 3, axis=0), seed + 200, 3.0)])
    # a few rays with a finite tmax
    rays[::7, 7] = 1.3
    sc = sg.Scene("soup", [mesh], sg.identity_xform(1), np.zeros(1, np.uint32),
                  np.zeros(1, np.uint32), sg.materials([(0, (1, 1, 1), 1.5)]),
                  sg.Camera((0, 0, 5), (0, 0, 0), (0, 1, 0), 60), sg.Light((0, 5, 0)), 1, 1, 1)
    res = oracle.Scene(sc).trace(rays)
    V = mesh.verts.astype(np.float64)
    tris = [(0, j, V[i0], V[i1], V[i2]) for j, (i0, i1, i2) in enumerate(mesh.idx)]
    n_hit = 0
    for r in range(rays.shape[0]):
        o, d = rays[r, 0:3], rays[r, 3:6]
        best = exact.closest(o, d, tris, rays[r, 6], rays[r, 7])
        if best is None:
            assert res["hit"][r] == 0
            continue
        n_hit += 1
        assert res["hit"][r] == 1
        assert res["prim"][r] == best[2]
        assert abs(res["t"][r] - float(best[0])) <= 1e-12 * max(1.0, float(best[0]))
        assert abs(res["u"][r] - float(best[3])) <= 1e-9
        assert abs(res["v"][r] - float(best[4])) <= 1e-9
    assert n_hit > 60


def test_icosphere_closed_forms():
    """Rays towards the centre: through a vertex (t = 4 from 5 v) and through a
    face's circumcentre (t = 5 - n.v0), which lies inside every (acute) face."""
    mesh = sg.icosphere(2)
    sc = sg.Scene("ico", [mesh], sg.identity_xform(1), np.zeros(1, np.uint32), np.zeros(1, np.uint32),
                  sg.materials([(0, (1, 1, 1), 1.5)]), sg.Camera((0, 0, 5), (0, 0, 0), (0, 1, 0), 60),
                  sg.Light((0, 5, 0)), 1, 1, 1)
    orc = oracle.Scene(sc)
    V = mesh.verts.astype(np.float64)
    # vertex rays
    vi = np.arange(0, V.shape[0], 7)
    vh = V[vi] / np.linalg.norm(V[vi], axis=1, keepdims=True)
    rays = np.zeros((vi.shape[0], 8), np.float32)
    rays[:, 0:3] = 5.0 * vh
    rays[:, 3:6] = -vh
    rays[:, 7] = np.inf
    res = orc.trace(rays)
    assert res["hit"].all()
    r_eff = np.linalg.norm(V[vi], axis=1)
    assert np.allclose(res["t"], 5.0 - r_eff, atol=2e-6)
    for k, v in enumerate(vi):
        assert v in mesh.idx[res["prim"][k]], "a vertex ray must hit a triangle incident to it"
    # face-centre rays
    F = mesh.idx.astype(np.int64)
    fi = np.arange(0, F.shape[0], 5)
    a, b, c = V[F[fi, 0]], V[F[fi, 1]], V[F[fi, 2]]
    n = np.cross(b - a, c - a)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    rays = np.zeros((fi.shape[0], 8), np.float32)
    rays[:, 0:3] = 5.0 * n
    rays[:, 3:6] = -n
    rays[:, 7] = np.inf
    res = orc.trace(rays)
    assert (res["prim"] == fi).all()
    expect = 5.0 - np.einsum("ij,ij->i", n, a)
    assert np.allclose(res["t"], expect, rtol=2e-6)


def test_nonzero_tmin_and_miss_sentinel():
    g = _load()
    sc = tri_scene([g["triangle"]])
    orc = oracle.Scene(sc)
    r = np.stack([ray((0.25, 0.25, 1), (0, 0, -1), 1.5, np.inf),   # hit before tmin -> miss
                  ray((0.25, 0.25, 1), (0, 0, -1), 1.0, 1.0)])     # degenerate interval at t
    res = orc.trace(r)
    assert res["hit"][0] == 0 and res["inst"][0] == oracle.MISS
    assert res["hit"][1] == 1 and res["t"][1] == 1.0
