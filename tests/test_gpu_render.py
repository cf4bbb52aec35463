"""GPU frame rendering (a7, a11-a13): closed-form scenes, the small
configuration's full frame, a reduced two-level frame and an ambient-
occlusion frame against the FP64 oracle; determinism of the fixed-point sums."""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg
from tests import parity
from tests.helpers import quad, scene_from_meshes

pytestmark = pytest.mark.gpu

SKY_H = np.array([0.75, 0.85, 1.0])


def _render(scene, width=None, height=None, max_depth=None, mode=None, seed=None):
    import paper_2001_09792_amd as rg
    W = width or scene.width
    H = height or scene.height
    D = scene.max_depth if max_depth is None else max_depth
    M = scene.mode if mode is None else mode
    tl = rg.upload_scene(scene)
    r = rg.Renderer(W, H, D, M)
    img, st = r.render(tl, scene.materials, scene.camera, scene.light, scene.seed if seed is None else seed,
                       stats=True)
    return img.cpu().numpy().reshape(-1, 3).copy(), st


def _one(meshes, mats, max_depth=1, light=(0.0, 0.0, 10.0), camera=None, mode=0, xforms=None):
    cam = camera or sg.Camera((0.0, 0.0, 5.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0)
    sc = scene_from_meshes(meshes, mats=mats, inst_mat=[0] * (len(meshes) if xforms is None else len(xforms)),
                           camera=cam, light=sg.Light(light), width=1, height=1, max_depth=max_depth,
                           mode=mode, xforms=xforms)
    img, _ = _render(sc)
    return img[0]


def test_closed_form_pixels():
    diff = sg.materials([(sg.DIFFUSE, (0.8, 0.8, 0.8), 1.5)])
    assert np.allclose(_one([sg.triangles_mesh(quad(0.0))], diff), 0.88, atol=1e-6)
    blk = [sg.triangles_mesh(quad(0.0)), sg.triangles_mesh(quad(7.0, half=0.5))]
    assert np.allclose(_one(blk, diff), 0.08, atol=1e-6)
    mir = sg.materials([(sg.MIRROR, (0.9, 0.9, 0.9), 1.5)])
    assert np.allclose(_one([sg.triangles_mesh(quad(0.0))], mir), [0.675, 0.765, 0.9], atol=1e-6)
    assert np.allclose(_one([sg.triangles_mesh(quad(0.0))], mir, max_depth=0), 0.0, atol=0)
    glass = sg.materials([(sg.GLASS, (1, 1, 1), 1.5)])
    slab = sg.triangles_mesh(quad(0.0) + quad(-1.0, normal_sign=-1.0))
    for D, f in ((1, 0.04), (2, 0.04 + 0.96 ** 2), (3, 0.04 + 0.96 ** 2 + 0.96 * 0.04 * 0.96)):
        assert np.allclose(_one([slab], glass, max_depth=D), SKY_H * f, atol=1e-6), D
    far = sg.triangles_mesh([[(100, 100, 100), (101, 100, 100), (100, 101, 100)]])
    assert np.allclose(_one([far], diff), SKY_H, atol=1e-6)


def test_closed_form_ao():
    plane = sg.triangles_mesh(quad(0.0, half=50.0))
    assert np.allclose(_one([plane], None, mode=1), 1.0)
    V = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], np.float32)
    faces = [(0, 1, 3), (0, 3, 2), (4, 6, 7), (4, 7, 5), (0, 4, 5), (0, 5, 1), (2, 3, 7), (2, 7, 6),
             (0, 2, 6), (0, 6, 4), (1, 5, 7), (1, 7, 3)]
    cube = sg.Mesh(V, np.array(faces, np.uint32))
    cam = sg.Camera((0.0, 0.0, 0.5), (0.0, 0.0, -1.0), (0.0, 1.0, 0.0), 60.0)
    assert np.allclose(_one([cube], None, camera=cam, mode=1), 0.0)


def test_small_config_full_frame():
    sc = sg.config_small()
    print("[render] small configuration 256x256 D=1", flush=True)
    img, st = _render(sc)
    assert st["rays_traced"] >= sc.width * sc.height
    ref = oracle.Scene(sc).render()
    res = parity.check_image(img, ref, 0.002, "small frame")
    print(res, flush=True)
    img2, _ = _render(sc)
    assert np.array_equal(img, img2), "fixed-point sums make frames bitwise reproducible"


@pytest.mark.parametrize("D", [1, 4])
def test_two_level_frame_sampled(D):
    W, H = 160, 90
    sc = sg.config_two_level(width=W, height=H, max_depth=D)
    print(f"[render] two-level {W}x{H} D={D}", flush=True)
    img, st = _render(sc)
    px = sg.sample_pixels(W, H, 1500, 11)
    ref = oracle.Scene(sc, sphere_reject=True).render(px)
    res = parity.check_image(img[px], ref, 0.025, f"two-level D={D}")
    print(res, st, flush=True)


def test_ao_frame_sampled():
    W, H = 160, 90
    sc = sg.config_incoherent(segments=24, width=W, height=H)
    print(f"[render] ambient occlusion {W}x{H}", flush=True)
    img, st = _render(sc)
    assert np.all((img == 1.0) | (np.abs(img * 8 - np.round(img * 8)) < 1e-6))
    px = sg.sample_pixels(W, H, 1500, 12)
    ref = oracle.Scene(sc, sphere_reject=True).render(px)
    res = parity.check_image(img[px], ref, 0.008, "ao")
    print(res, st, flush=True)


def test_oblique_glass_matches_snell_schlick():
    s = math.sqrt(0.5)
    cam = sg.Camera((0.0, 5 * s, 5 * s), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0)
    glass = sg.materials([(sg.GLASS, (1, 1, 1), 1.5)])
    for mirror in (False, True):
        X = sg.identity_xform(1)
        if mirror:
            X[0, 0, 0] = -1.0
        got = _one([sg.triangles_mesh(quad(0.0, half=5))], glass, camera=cam, xforms=X)

        def sky(dy):
            a = 0.5 * (dy + 1)
            return (1 - a) * np.ones(3) + a * np.array([0.5, 0.7, 1.0])

        F = 0.04 + 0.96 * (1 - s) ** 5
        expect = F * sky(-s) + (1 - F) * sky(-s / 1.5)
        assert np.allclose(got, expect, atol=1e-5), mirror


def test_frame_launch_parameters_do_not_change_images():
    """The frame family's launch parameters reorder work only: bitwise the same image."""
    import paper_2001_09792_amd as rg
    sc = sg.config_two_level(width=160, height=90, max_depth=3)
    tl = rg.upload_scene(sc, 4, 2)
    saved = rg.trace_tuning(scope="frame")
    try:
        ref = None
        for cfg in (dict(refill=8, waves_per_cu=16, lds_depth=16, leaf_batch=1, inst_batch=1),
                    dict(refill=32, waves_per_cu=8, lds_depth=8, leaf_batch=16, inst_batch=8),
                    dict(refill=1, waves_per_cu=24, lds_depth=32, leaf_batch=64, inst_batch=64)):
            rg.trace_tuning(scope="frame", **cfg)
            img = rg.render(tl, sc.materials, sc.camera, sc.light, 160, 90, 3).cpu().numpy()
            if ref is None:
                ref = img
            assert np.array_equal(img.view(np.uint32), ref.view(np.uint32)), cfg
    finally:
        rg.trace_tuning(scope="frame", **saved)
