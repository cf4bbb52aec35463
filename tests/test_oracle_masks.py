"""Ray visibility masks and face culling in the FP64 oracle (the accept /
ignore semantics an any-hit stage applies, in the form of RTX / Vulkan
instance masks and cull flags), pinned by closed forms on hand scenes and by
invariants that hold for any scene: culling splits the hits into the two
facings, and masks select instances."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from tests.helpers import quad, ray, scene_from_meshes, tri_scene

BACK, FRONT = oracle.RAY_CULL_BACK, oracle.RAY_CULL_FRONT


def _t(res, k=0):
    return float(res["t"][k]) if res["hit"][k] else np.inf


def test_single_quad_facing():
    """A quad at z = 0 wound counter-clockwise seen from +z (normal +z): a ray
    coming down from +z travels against the normal (front face), one coming
    up from below along it (back face)."""
    sc = tri_scene(quad(0.0, normal_sign=1.0))
    o = oracle.Scene(sc)
    down = ray((0.3, 0.2, 5.0), (0.0, 0.0, -1.0))
    up = ray((0.3, 0.2, -5.0), (0.0, 0.0, 1.0))
    rays = np.stack([down, up])
    assert [_t(o.trace(rays), k) for k in (0, 1)] == [5.0, 5.0]
    assert [_t(o.trace(rays, cull=BACK), k) for k in (0, 1)] == [5.0, np.inf]
    assert [_t(o.trace(rays, cull=FRONT), k) for k in (0, 1)] == [np.inf, 5.0]
    assert [_t(o.trace(rays, cull=BACK | FRONT), k) for k in (0, 1)] == [np.inf, np.inf]
    # any hit follows the same rule
    assert list(o.trace(rays, any_hit=True, cull=BACK)["hit"]) == [1, 0]


def test_stacked_quads_closed_forms():
    """Quads at z = 0 (normal +z) and z = -1 (normal -z) in one mesh: a ray
    down from z = 5 meets the first as a front face at t = 5 and the second as
    a back face at t = 6."""
    sc = tri_scene(quad(0.0, normal_sign=1.0) + quad(-1.0, normal_sign=-1.0))
    o = oracle.Scene(sc)
    r = ray((0.1, -0.4, 5.0), (0.0, 0.0, -1.0))[None]
    assert _t(o.trace(r)) == 5.0
    assert _t(o.trace(r, cull=BACK)) == 5.0
    assert _t(o.trace(r, cull=FRONT)) == 6.0
    assert o.trace(r, cull=FRONT)["prim"][0] in (2, 3)


def _two_instances(flags=None, xf2=None):
    X = sg.identity_xform(2)
    X[1, 2, 3] = -1.0  # the second copy one unit lower
    if xf2 is not None:
        X[1] = xf2
    sc = scene_from_meshes([sg.triangles_mesh(quad(0.0, normal_sign=1.0))], xforms=X, blas_id=[0, 0])
    return sc, oracle.Scene(sc, inst_flags=flags)


def test_instance_masks():
    sc, o = _two_instances(flags=np.array([0x01, 0x02], np.uint32))
    r = np.stack([ray((0.2, 0.1, 5.0), (0.0, 0.0, -1.0))] * 4)
    assert _t(o.trace(r[:1], mask=0x01)) == 5.0
    assert _t(o.trace(r[:1], mask=0x02)) == 6.0 and o.trace(r[:1], mask=0x02)["inst"][0] == 1
    assert _t(o.trace(r[:1], mask=0x04)) == np.inf
    assert _t(o.trace(r[:1], mask=0x03)) == 5.0
    # per-ray masks override the call's
    res = o.trace(r, ray_mask=np.array([0x01, 0x02, 0x04, 0xFF], np.uint8))
    assert [_t(res, k) for k in range(4)] == [5.0, 6.0, np.inf, 5.0]
    # an instance whose mask is 0 is seen by no ray
    sc, o0 = _two_instances(flags=np.array([0x00, 0xFF], np.uint32))
    assert _t(o0.trace(r[:1])) == 6.0


def test_instance_flip_and_cull_disable():
    down = ray((0.2, 0.1, 5.0), (0.0, 0.0, -1.0))[None]
    # flipped facing: the down ray now meets a back face
    sc, o = _two_instances(flags=np.array([0xFF | oracle.INST_FLIP_FACING, 0x00], np.uint32))
    assert _t(o.trace(down, cull=BACK)) == np.inf and _t(o.trace(down, cull=FRONT)) == 5.0
    # culling disabled for the first instance: both flags leave its hit
    sc, o = _two_instances(flags=np.array([0xFF | oracle.INST_CULL_DISABLE, 0xFF], np.uint32))
    assert _t(o.trace(down, cull=FRONT)) == 5.0
    assert _t(o.trace(down, cull=BACK | FRONT)) == 5.0


def test_mirrored_instance_facing_is_object_space():
    """An instance mirrored in x (det < 0) flips the winding seen in world
    space; facing is decided in object space, so the down ray still meets a
    front face."""
    X = np.zeros((3, 4), np.float32)
    X[0, 0], X[1, 1], X[2, 2] = -1.0, 1.0, 1.0
    sc = scene_from_meshes([sg.triangles_mesh(quad(0.0, normal_sign=1.0))], xforms=X[None], blas_id=[0])
    o = oracle.Scene(sc)
    down = ray((0.2, 0.1, 5.0), (0.0, 0.0, -1.0))[None]
    assert _t(o.trace(down, cull=BACK)) == 5.0
    assert _t(o.trace(down, cull=FRONT)) == np.inf


def _random_scene(seed):
    meshes = [sg.random_soup(300, seed, 1.0, 0.3), sg.icosphere(1), sg.torus(12, 10, 1.0, 0.3)]
    rng = np.random.default_rng(seed)
    xf = sg.random_instances(rng, 12, extent=2.5)
    return scene_from_meshes(meshes, xforms=xf, blas_id=np.arange(12) % 3), rng


@pytest.mark.parametrize("seed", [3, 4])
def test_culling_splits_the_hits(seed):
    """For every ray not flagged ambiguous: the closest hit without culling is
    the nearer of the closest hits with back faces culled and with front faces
    culled, and it is the same triangle."""
    sc, rng = _random_scene(seed)
    o = oracle.Scene(sc)
    rays = sg.random_rays(1500, seed + 10, extent=4.0)
    a, b, f = o.trace(rays), o.trace(rays, cull=BACK), o.trace(rays, cull=FRONT)
    ok = (a["amb"] == 0) & (b["amb"] == 0) & (f["amb"] == 0)
    assert ok.mean() > 0.95
    ta = np.where(a["hit"] == 1, a["t"], np.inf)
    tb = np.where(b["hit"] == 1, b["t"], np.inf)
    tf = np.where(f["hit"] == 1, f["t"], np.inf)
    assert np.array_equal(ta[ok], np.minimum(tb, tf)[ok])
    for res, t in ((b, tb), (f, tf)):
        same = ok & (t == ta) & np.isfinite(ta)
        assert np.array_equal(res["inst"][same], a["inst"][same]) and np.array_equal(res["prim"][same],
                                                                                      a["prim"][same])
    # both facings occur
    assert np.isfinite(tb[ok]).sum() > 50 and np.isfinite(tf[ok]).sum() > 50
    # culling both facings sees nothing
    assert o.trace(rays, cull=BACK | FRONT)["hit"].sum() == 0


@pytest.mark.parametrize("seed", [5])
def test_masks_select_instances(seed):
    """Any hit under a union of mask bits is the OR of the any hits under the
    bits alone; the closest hit under a mask equals the closest hit of the
    scene restricted to the instances that share a bit with it."""
    sc, rng = _random_scene(seed)
    flags = rng.choice([0x01, 0x02, 0x04, 0x03], size=12).astype(np.uint32)
    o = oracle.Scene(sc, inst_flags=flags)
    rays = sg.random_rays(1200, seed + 20, extent=4.0)
    occ = {m: o.trace(rays, any_hit=True, mask=m) for m in (0x01, 0x02, 0x04, 0x07)}
    ok = np.all([occ[m]["amb"] == 0 for m in occ], axis=0)
    union = occ[0x01]["hit"] | occ[0x02]["hit"] | occ[0x04]["hit"]
    assert np.array_equal(occ[0x07]["hit"][ok], union[ok])
    keep = np.nonzero(flags & 0x02)[0]
    sub = scene_from_meshes(sc.blas, xforms=sc.xform[keep], blas_id=sc.blas_id[keep])
    rs, rm = oracle.Scene(sub).trace(rays), o.trace(rays, mask=0x02)
    ok = (rs["amb"] == 0) & (rm["amb"] == 0)
    assert np.array_equal(rs["hit"][ok], rm["hit"][ok])
    h = ok & (rm["hit"] == 1)
    assert np.array_equal(rs["t"][h], rm["t"][h])
    assert np.array_equal(keep[rs["inst"][h]], rm["inst"][h])
