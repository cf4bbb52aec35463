"""Closed-form pins of the oracle's camera, shading recursion and ambient
occlusion.  The paper names ray generation (section 1), shadow casting,
reflection and refraction (section 2.1) and a recursion cap (section 1,
footnote); the constants and formulas pinned here are this project's
readings of those names, each reduced to a case with a hand-computed value."""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg
from tests.helpers import quad, scene_from_meshes

SKY_H = (0.75, 0.85, 1.0)   # sky for any horizontal direction: a = 1/2


def _cam(eye=(0.0, 0.0, 5.0), target=(0.0, 0.0, 0.0), vfov=60.0):
    return sg.Camera(eye, target, (0.0, 1.0, 0.0), vfov)


def _render_center(meshes, mats, inst_mat, max_depth=1, light=(0.0, 0.0, 10.0), camera=None,
                   mode=0, blas_id=None, xforms=None):
    sc = scene_from_meshes(meshes, mats=mats, inst_mat=inst_mat, camera=camera or _cam(),
                           light=sg.Light(light), width=1, height=1, max_depth=max_depth, mode=mode,
                           blas_id=blas_id, xforms=xforms)
    return oracle.Scene(sc).render(np.array([0]))


def test_camera_centre_pixel_is_forward():
    for W, H in ((1, 1), (5, 3), (7, 9)):
        px = np.array([(H // 2) * W + W // 2])
        r = oracle.camera_rays(_cam(eye=(1.0, 2.0, 3.0), target=(4.0, -2.0, 3.0)), W, H, px)
        f = np.array([3.0, -4.0, 0.0]) / 5.0
        assert np.allclose(r[0, 3:6], f, atol=1e-15)
        assert np.allclose(r[0, 0:3], (1.0, 2.0, 3.0))


def test_camera_vertical_fov():
    """Top-centre pixel of an odd-width image: elevation atan((1-1/H) tan(vfov/2));
    right-centre pixel: azimuth atan((1-1/W) tan(vfov/2) W/H); y = 0 is the top row."""
    W, H, vfov = 9, 5, 60.0
    th = math.tan(math.radians(vfov / 2))
    r = oracle.camera_rays(_cam(), W, H, np.array([W // 2, (H // 2) * W + W - 1]))
    d_top, d_right = r[0, 3:6], r[1, 3:6]
    assert d_top[1] > 0
    assert math.atan2(d_top[1], -d_top[2]) == pytest.approx(math.atan((1 - 1 / H) * th), abs=1e-14)
    assert d_right[0] > 0
    assert math.atan2(d_right[0], -d_right[2]) == pytest.approx(math.atan((1 - 1 / W) * th * W / H),
                                                                abs=1e-14)


@pytest.mark.parametrize("target,expect", [
    ((0.0, 0.0, -1.0), SKY_H), ((0.0, 0.0, 10.0), SKY_H),
    ((0.0, 10.0, 5.0), (0.5, 0.7, 1.0)), ((0.0, -10.0, 5.0), (1.0, 1.0, 1.0)),
])
def test_sky(target, expect):
    up = (1.0, 0.0, 0.0) if target[0] == 0 and target[2] == 5.0 else (0.0, 1.0, 0.0)
    cam = sg.Camera((0.0, 0.0, 5.0), target, up, 60.0)
    far = sg.triangles_mesh([[(100, 100, 100), (101, 100, 100), (100, 101, 100)]])
    out = _render_center([far], sg.materials([(0, (1, 1, 1), 1.5)]), [0], camera=cam)
    assert np.allclose(out["rgb"][0], expect, atol=1e-12)


def test_diffuse_unshadowed_and_shadowed():
    """rho (k_a + I cos V) with rho = 0.8, k_a = 0.1, light along the normal:
    0.88 lit, 0.08 in shadow."""
    mats = sg.materials([(sg.DIFFUSE, (0.8, 0.8, 0.8), 1.5)])
    lit = _render_center([sg.triangles_mesh(quad(0.0))], mats, [0])
    assert np.allclose(lit["rgb"][0], 0.88, atol=1e-12)
    blocker = sg.triangles_mesh(quad(7.0, half=0.5))   # behind the camera, in front of the light
    dark = _render_center([sg.triangles_mesh(quad(0.0)), blocker], mats, [0, 0])
    assert np.allclose(dark["rgb"][0], 0.08, atol=1e-12)


def test_diffuse_cosine():
    """Light at 60 degrees from the normal: 0.8 (0.1 + cos 60) = 0.48."""
    mats = sg.materials([(sg.DIFFUSE, (0.8, 0.8, 0.8), 1.5)])
    lp = (10.0 * math.sin(math.radians(60)), 0.0, 10.0 * math.cos(math.radians(60)))
    out = _render_center([sg.triangles_mesh(quad(0.0, half=20))], mats, [0], light=lp)
    assert np.allclose(out["rgb"][0], 0.8 * (0.1 + 0.5), atol=1e-7)


def test_mirror_reflects_sky():
    mats = sg.materials([(sg.MIRROR, (0.9, 0.9, 0.9), 1.5)])
    out = _render_center([sg.triangles_mesh(quad(0.0))], mats, [0], max_depth=1)
    assert np.allclose(out["rgb"][0], (0.675, 0.765, 0.9), atol=1e-12)
    capped = _render_center([sg.triangles_mesh(quad(0.0))], mats, [0], max_depth=0)
    assert np.allclose(capped["rgb"][0], 0.0, atol=0)


@pytest.mark.parametrize("D,factor", [(0, 0.0), (1, 0.04), (2, 0.04 + 0.96 ** 2),
                                      (3, 0.04 + 0.96 ** 2 + 0.96 * 0.04 * 0.96)])
def test_glass_slab_normal_incidence(D, factor):
    """Slab between z=-1 and z=0 (outward normals), seen head-on.  Schlick at
    normal incidence gives F = 0.04 at both faces; the cap decides which paths
    count: D=1 -> 0.04 sky, D=2 -> (0.04 + 0.96^2) sky, D=3 adds the path
    that reflects once off the back face and leaves through the front
    (0.96 * 0.04 * 0.96); a glass hit at depth D contributes nothing."""
    mats = sg.materials([(sg.GLASS, (1.0, 1.0, 1.0), 1.5)])
    slab = sg.triangles_mesh(quad(0.0) + quad(-1.0, normal_sign=-1.0))
    out = _render_center([slab], mats, [0], max_depth=D)
    assert np.allclose(out["rgb"][0], np.array(SKY_H) * factor, atol=1e-12)


def test_glass_total_internal_reflection():
    """Inside glass at 60 degrees (> 41.8 critical): F = 1, all light reflects."""
    mats = sg.materials([(sg.GLASS, (1, 1, 1), 1.5), (sg.DIFFUSE, (0.5, 0.5, 0.5), 1.5)])
    ang = math.radians(60)
    eye = (0.0, 0.0, 0.0)
    tgt = (math.sin(ang), 0.0, math.cos(ang))       # looking towards +z face at 60 deg
    cam = sg.Camera(eye, tgt, (0.0, 1.0, 0.0), 60.0)
    face = sg.triangles_mesh(quad(1.0, half=50.0))  # normal +z: the ray exits through it
    out = _render_center([face], mats, [0], max_depth=1, camera=cam)
    # reflected ray goes down (-z) to the sky with d_y = 0
    assert np.allclose(out["rgb"][0], SKY_H, atol=1e-12)


def test_ao_uniforms_match_splitmix64_reference():
    """SplitMix64 seeded with 1234567 outputs 6457827717110365317,
    3203168211198807973 first (the generator's published reference output);
    with key 0 the uniforms are their top 24 bits times 2^-24."""
    u1, u2 = oracle.ao_uniforms(1234567, 0)
    assert u1 == (6457827717110365317 >> 40) / 2.0 ** 24
    assert u2 == (3203168211198807973 >> 40) / 2.0 ** 24


def test_ao_direction_distribution():
    """Cosine-weighted hemisphere: unit length, inside the hemisphere, and
    E[cos] = 2/3 (Malley's method)."""
    rng = np.random.default_rng(0)
    ns = rng.normal(size=(6, 3))
    ns /= np.linalg.norm(ns, axis=1, keepdims=True)
    ns = np.vstack([ns, [[0, 0, 1], [0, 0, -1], [1, 0, 0]]])
    for n in ns:
        cs = []
        for k in range(4000):
            u1, u2 = oracle.ao_uniforms(77, k)
            d = oracle.ao_direction(n, u1, u2)
            assert abs(np.linalg.norm(d) - 1.0) < 1e-12
            cs.append(d @ n)
        cs = np.array(cs)
        assert cs.min() >= 0.0
        assert abs(cs.mean() - 2.0 / 3.0) < 0.02


def test_ao_open_plane_and_closed_box():
    plane = sg.triangles_mesh(quad(0.0, half=50.0))
    cam = _cam(eye=(0.0, 0.0, 5.0))
    out = _render_center([plane], None, [0], camera=cam, mode=1)
    assert np.allclose(out["rgb"][0], 1.0)
    # inside a closed cube of half-size 1: every ray hits within 5
    V, F = _cube_mesh()
    cube = sg.Mesh(V, F)
    inside = _cam(eye=(0.0, 0.0, 0.5), target=(0.0, 0.0, -1.0))
    out = _render_center([cube], None, [0], camera=inside, mode=1)
    assert np.allclose(out["rgb"][0], 0.0)
    # no geometry at all in front: miss pixel = 1
    out = _render_center([sg.triangles_mesh([[(0, 100, 0), (1, 100, 0), (0, 101, 0)]])], None, [0],
                         camera=cam, mode=1)
    assert np.allclose(out["rgb"][0], 1.0)


def _cube_mesh():
    V = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], np.float64)
    faces = []
    for axis in range(3):
        for sgn in (-1, 1):
            ids = [i for i in range(8) if V[i, axis] == sgn]
            # order the 4 corners around the face
            c = V[ids].mean(axis=0)
            u = (axis + 1) % 3
            w = (axis + 2) % 3
            ang = [math.atan2(V[i, w] - c[w], V[i, u] - c[u]) for i in ids]
            ids = [i for _, i in sorted(zip(ang, ids))]
            faces += [(ids[0], ids[1], ids[2]), (ids[0], ids[2], ids[3])]
    F = np.array(faces)
    cen = (V[F[:, 0]] + V[F[:, 1]] + V[F[:, 2]]) / 3
    F = sg._orient_outward(V, F, cen)
    return V.astype(np.float32), F.astype(np.uint32)


def test_small_config_frame_properties():
    """Full small-configuration frame: finite, non-negative, deterministic,
    few ambiguous pixels, and mirror pixels show the reflected ground."""
    sc = sg.config_small()
    orc = oracle.Scene(sc)
    a = orc.render()
    b = orc.render(threads=3)
    assert np.array_equal(a["rgb"], b["rgb"]) and np.array_equal(a["amb"], b["amb"])
    assert np.isfinite(a["rgb"]).all() and (a["rgb"] >= 0).all()
    assert a["amb"].mean() < 0.005
    assert a["nrays"].min() >= 1 and a["nrays"].max() <= 4


def test_normal_uses_inverse_transpose():
    """A sheared instance maps the plane z=0 to z=x, whose normal is
    (-1,0,1)/sqrt2 (the inverse-transpose image of +z, not M(+z) = +z).
    Camera and light along that normal: 0.8 (0.1 + 1) = 0.88."""
    X = np.zeros((1, 3, 4), np.float32)
    X[0, :, :3] = [[1, 0, 0], [0, 1, 0], [1, 0, 1]]
    n = np.array([-1.0, 0.0, 1.0]) / math.sqrt(2.0)
    cam = sg.Camera(tuple(5 * n), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0)
    mats = sg.materials([(sg.DIFFUSE, (0.8, 0.8, 0.8), 1.5)])
    out = _render_center([sg.triangles_mesh(quad(0.0, half=5))], mats, [0], camera=cam,
                         light=tuple(10 * n), xforms=X)
    assert np.allclose(out["rgb"][0], 0.88, atol=1e-6)


@pytest.mark.parametrize("mirror", [False, True])
def test_glass_oblique_entry_and_winding_flip(mirror):
    """A single glass face z=0 (normal +z) hit from above at 45 degrees in the
    yz-plane.  Snell: sin t = sin 45 / 1.5; Schlick: F = 0.04 + 0.96 (1-cos45)^5.
    Both children reach the sky (D=1).  Mirroring the instance (x -> -x,
    det < 0) reverses the world-space winding, but the normal transforms with
    the inverse transpose, which keeps the object's outward side outward, so
    the result is the same; a winding-based world normal would read the hit as
    an exit (total internal reflection)."""
    X = sg.identity_xform(1)
    if mirror:
        X[0, 0, 0] = -1.0
    s = math.sqrt(0.5)
    cam = sg.Camera((0.0, 5 * s, 5 * s), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0)
    mats = sg.materials([(sg.GLASS, (1, 1, 1), 1.5)])
    out = _render_center([sg.triangles_mesh(quad(0.0, half=5))], mats, [0], camera=cam,
                         max_depth=1, xforms=X)

    def sky(dy):
        a = 0.5 * (dy + 1)
        return (1 - a) * np.ones(3) + a * np.array([0.5, 0.7, 1.0])

    F = 0.04 + 0.96 * (1 - s) ** 5
    sin_t = s / 1.5
    expect = F * sky(-s) + (1 - F) * sky(-sin_t)
    assert np.allclose(out["rgb"][0], expect, atol=1e-12)
