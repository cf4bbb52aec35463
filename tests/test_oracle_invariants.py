"""Invariants of the two-level scene (paper section 1: instances with
transformation matrices over mesh vertex data; closest hit, any hit, miss),
checked on the FP64 oracle."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from tests.helpers import ray, scene_from_meshes

UNIT = [(0, 0, 0), (1, 0, 0), (0, 1, 0)]


def _xf(R, t):
    X = np.zeros((1, 3, 4), np.float32)
    X[0, :, :3] = R
    X[0, :, 3] = t
    return X


@pytest.mark.parametrize("name,R,t,o,d", [
    ("rot90z", [[0, -1, 0], [1, 0, 0], [0, 0, 1]], [0, 0, 0], (-0.25, 0.25, 1), (0, 0, -1)),
    ("translate", np.eye(3), [5, 0, 0], (5.25, 0.25, 1), (0, 0, -1)),
    ("scale2", 2 * np.eye(3), [0, 0, 0], (0.5, 0.5, 2), (0, 0, -2)),
])
def test_instance_hand_cases(name, R, t, o, d):
    """Rotating, translating or scaling the instance together with the ray
    keeps t = 1 and u = v = 1/4 of the canonical case."""
    sc = scene_from_meshes([sg.triangles_mesh([UNIT])], xforms=_xf(R, t))
    res = oracle.Scene(sc).trace(ray(o, d)[None])
    assert res["hit"][0] == 1
    assert res["t"][0] == pytest.approx(1.0, abs=1e-12)
    assert res["u"][0] == pytest.approx(0.25, abs=1e-12)
    assert res["v"][0] == pytest.approx(0.25, abs=1e-12)


def _apply(G, gt, rays):
    out = rays.copy()
    out[:, 0:3] = rays[:, 0:3] @ G.T + gt
    out[:, 3:6] = rays[:, 3:6] @ G.T
    return out.astype(np.float32)


def _compose(G, gt, X):
    Y = np.empty_like(X)
    Y[:, :, :3] = np.einsum("ij,njk->nik", G, X[:, :, :3])
    Y[:, :, 3] = X[:, :, 3] @ G.T + gt
    return Y.astype(np.float32)


def _soup_scene(seed):
    meshes = [sg.random_soup(30, seed, 1.0, 0.4), sg.icosphere(1)]
    rng = np.random.default_rng(seed)
    X = np.zeros((4, 3, 4), np.float32)
    for i in range(4):
        X[i, :, :3] = np.eye(3) * [1, 2, 0.5, 1][i]
        X[i, :, 3] = rng.integers(-2, 3, 3)
    return scene_from_meshes(meshes, xforms=X, blas_id=[0, 1, 0, 1])


def test_rigid_motion_exact():
    """A motion that is exact in float32 (axis permutation with signs, a power
    of two scale, an integer translation) applied to every instance and to
    the rays leaves t, ids, u, v unchanged to 1e-12."""
    sc = _soup_scene(5)
    rays = sg.random_rays(300, 6, extent=3.0)
    rays[:, :6] = np.round(rays[:, :6] * 4096.0) / 4096.0   # so that integer shifts stay exact
    base = oracle.Scene(sc).trace(rays)
    G = np.array([[0, 0, 2], [-2, 0, 0], [0, 2, 0]], np.float64)
    gt = np.array([3.0, -1.0, 4.0])
    sc2 = scene_from_meshes(sc.blas, xforms=_compose(G, gt, sc.xform), blas_id=sc.blas_id)
    moved = oracle.Scene(sc2).trace(_apply(G, gt, rays))
    assert base["hit"].sum() > 30
    assert (base["hit"] == moved["hit"]).all()
    h = base["hit"] == 1
    assert (base["inst"][h] == moved["inst"][h]).all()
    assert (base["prim"][h] == moved["prim"][h]).all()
    assert np.allclose(base["t"][h], moved["t"][h], rtol=1e-12)
    assert np.allclose(base["u"][h], moved["u"][h], atol=1e-12)
    assert np.allclose(base["v"][h], moved["v"][h], atol=1e-12)


def test_rigid_motion_random_rotation():
    """A random rotation + translation (rounded to float32) changes results
    only within the float32 rounding of the moved inputs."""
    sc = _soup_scene(7)
    rays = sg.random_rays(300, 8, extent=3.0)
    base = oracle.Scene(sc).trace(rays)
    G = sg.quat_to_matrix(sg.uniform_quaternion(np.random.default_rng(3), 1))[0]
    gt = np.array([10.0, -3.0, 2.5])
    sc2 = scene_from_meshes(sc.blas, xforms=_compose(G, gt, sc.xform), blas_id=sc.blas_id)
    moved = oracle.Scene(sc2).trace(_apply(G, gt, rays))
    ok = (base["amb"] == 0) & (moved["amb"] == 0)
    assert ok.mean() > 0.9
    assert (base["hit"][ok] == moved["hit"][ok]).all()
    h = ok & (base["hit"] == 1)
    assert (base["prim"][h] == moved["prim"][h]).all()
    # the moved origin carries a float32 rounding of about 1e-6 in absolute terms
    assert np.allclose(base["t"][h], moved["t"][h], rtol=1e-5, atol=1e-5)


def test_closest_vs_any():
    """closest t <= every any-hit t, and occluded == a closest hit exists."""
    sc = _soup_scene(9)
    rays = sg.random_rays(400, 10, extent=3.0)
    rays[::3, 7] = 0.7
    orc = oracle.Scene(sc)
    c = orc.trace(rays)
    a = orc.trace(rays, any_hit=True)
    assert (c["hit"] == a["hit"]).all()
    assert c["hit"].sum() > 30


def test_permutation_invariance():
    """Permuting triangles or instances relabels ids but keeps t, u, v."""
    sc = _soup_scene(13)
    rays = sg.random_rays(300, 14, extent=3.0)
    base = oracle.Scene(sc).trace(rays)
    # permute instances
    perm = np.array([2, 0, 3, 1])
    sc_i = scene_from_meshes(sc.blas, xforms=sc.xform[perm], blas_id=sc.blas_id[perm])
    pi = oracle.Scene(sc_i).trace(rays)
    # permute the soup's triangles
    m0 = sc.blas[0]
    tperm = np.random.default_rng(1).permutation(m0.n_tris)
    m0p = sg.Mesh(m0.verts, m0.idx[tperm])
    sc_t = scene_from_meshes([m0p, sc.blas[1]], xforms=sc.xform, blas_id=sc.blas_id)
    pt = oracle.Scene(sc_t).trace(rays)
    ok = base["amb"] == 0
    h = ok & (base["hit"] == 1)
    for other in (pi, pt):
        assert (other["hit"][ok] == base["hit"][ok]).all()
        assert np.allclose(other["t"][h], base["t"][h], rtol=1e-12)
    assert (perm[pi["inst"][h]] == base["inst"][h]).all()
    soup = h.copy()
    soup[h] = sc.blas_id[base["inst"][h]] == 0
    assert (tperm[pt["prim"][soup]] == base["prim"][soup]).all()


def test_sphere_reject_is_exact():
    """The bounding-sphere reject only skips instances that cannot be hit."""
    sc = sg.config_two_level(width=64, height=36)
    orc = oracle.Scene(sc)
    px = sg.sample_pixels(64, 36, 48, 1)
    cam_rays = oracle.camera_rays(sc.camera, 64, 36, px)
    rays = np.zeros((px.shape[0], 8), np.float32)
    rays[:, :6] = cam_rays
    rays[:, 7] = np.inf
    a = orc.trace(rays)
    orc.set_sphere_reject(True)
    b = orc.trace(rays)
    assert b["tests"] < a["tests"]
    for k in ("hit", "inst", "prim", "amb", "t", "u", "v"):
        assert np.array_equal(a[k], b[k]), k
