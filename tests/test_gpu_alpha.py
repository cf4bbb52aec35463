"""Opacity masks on the GPU (alpha-tested triangles: the accept / ignore
decision of an any-hit stage per point of a triangle): the subdivisions
worked out by hand, parity with the FP64 oracle on random scenes for every
level and with the other ray options, full masks equal to no masks bit for
bit, removal, and the rendered frame against the oracle's."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from tests import bvh_check, parity
from tests.helpers import ray, scene_from_meshes

pytestmark = pytest.mark.gpu


def _rg():
    import paper_2001_09792_amd as rg
    return rg


def _masks(m):
    import torch
    return torch.from_numpy(np.ascontiguousarray(m, np.uint64).view(np.int64)).cuda()


def _tlas(sc, alpha, width=4, leaf=4, builder="lbvh", flags=None):
    """Top level over the scene's meshes with opacity masks per mesh
    (alpha[b] = (mask per triangle, level) or None)."""
    rg = _rg()
    tl = rg.upload_scene(sc, width, leaf, builder=builder)
    for b, a in zip(tl.blas, alpha):
        if a is not None:
            rg.set_alpha(b, _masks(a[0]), a[1])
    tl2 = rg.build_tlas(tl.blas, sc.xform, sc.blas_id, sc.inst_mat, width, builder=builder, inst_flags=flags)
    want_flags = (np.full(sc.xform.shape[0], 0xFF, np.uint32) if flags is None else np.asarray(flags, np.uint32)) | \
        np.array([(1 << 16) if alpha[b] is not None else 0 for b in sc.blas_id], np.uint32)
    bvh_check.check_tlas(tl2.buf.cpu().numpy(), tl2.desc, [b.desc for b in tl2.blas], sc.xform, inst_flags=want_flags)
    return tl2


TRI = [[(0, 0, 0), (4, 0, 0), (0, 4, 0)]]


def _down(points):
    return np.stack([ray((4 * x, 4 * y, 3.0), (0.0, 0.0, -1.0)) for x, y in points])


@pytest.mark.parametrize("width", [2, 4, 8])
def test_levels_one_and_two_by_hand(width):
    rg = _rg()
    sc = scene_from_meshes([sg.triangles_mesh(TRI)])
    pts1 = [(0.1, 0.1), (0.4, 0.4), (0.7, 0.1), (0.1, 0.7)]
    print(f"[alpha] hand cases W{width}", flush=True)
    for mask in (0b0101, 0b1010, 0b0001, 0b1111, 0):
        tl = _tlas(sc, [([mask], 1)], width)
        h = parity.hits_to_numpy(rg.trace_closest(tl, rg.rays_to_device(_down(pts1))))
        assert list(h["inst"].astype(np.uint32) != 0xFFFFFFFF) == [bool((mask >> k) & 1) for k in range(4)]
        occ = rg.trace_any(tl, rg.rays_to_device(_down(pts1))).cpu().numpy()
        assert list(occ) == [(mask >> k) & 1 for k in range(4)]
    cases = {(0.05, 0.05): 0, (0.2, 0.2): 1, (0.3, 0.05): 2, (0.45, 0.2): 3, (0.55, 0.1): 4, (0.7, 0.2): 5,
             (0.8, 0.1): 6, (0.05, 0.3): 7, (0.2, 0.45): 8, (0.3, 0.3): 9, (0.45, 0.45): 10, (0.55, 0.3): 11,
             (0.05, 0.55): 12, (0.2, 0.7): 13, (0.3, 0.55): 14, (0.1, 0.8): 15}
    pts = list(cases)
    for k in (0, 3, 9, 15):
        tl = _tlas(sc, [([1 << k], 2)], width)
        occ = rg.trace_any(tl, rg.rays_to_device(_down(pts))).cpu().numpy()
        assert [p for p, o in zip(pts, occ) if o] == [p for p in pts if cases[p] == k], k


def _scene(seed):
    rng = np.random.default_rng(seed)
    meshes = [sg.random_soup(700, seed, 1.0, 0.5), sg.icosphere(2), sg.torus(20, 14, 1.0, 0.35), sg.random_soup(300, 9)]
    xf = sg.random_instances(rng, 12, extent=2.5)
    sc = scene_from_meshes(meshes, xforms=xf, blas_id=np.arange(12) % 4)
    masks = [rng.integers(0, 2 ** 63, m.n_tris, dtype=np.int64).astype(np.uint64) * np.uint64(2) +
             rng.integers(0, 2, m.n_tris).astype(np.uint64) for m in meshes]
    return sc, masks, rng


@pytest.mark.parametrize("builder,width,leaf", [("lbvh", 4, 4), ("ploc", 8, 3), ("lbvh", 2, 1), ("treelet", 4, 1)])
def test_parity_with_the_oracle(builder, width, leaf):
    """Levels 0, 1, 2, 3 on four meshes (one without masks in the second
    case), alone and with culling and per-ray masks."""
    import torch
    rg = _rg()
    sc, masks, rng = _scene(31)
    rays = np.concatenate([sg.random_rays(2500, 41, extent=4.0),
                           sg.rays_through_points(rng.uniform(-2.5, 2.5, (2500, 3)), 42, 6.0)])
    rd = rg.rays_to_device(rays)
    for case, levels in enumerate(([0, 1, 2, 3], [3, None, 2, 1])):
        alpha = [None if l is None else (masks[b], l) for b, l in enumerate(levels)]
        tl = _tlas(sc, alpha, width, leaf, builder)
        orc = oracle.Scene(sc, alpha=alpha)
        rm_np = rng.choice([0x01, 0xFF], size=rays.shape[0]).astype(np.uint8)
        for cull, per_ray in ((0, False), (rg.RAY_CULL_BACK, False), (0, True)):
            label = f"{builder} W{width} L{leaf} levels={levels} cull={cull} per_ray={per_ray}"
            print(f"[alpha parity] {label}", flush=True)
            kw = dict(cull=cull, ray_mask=torch.from_numpy(rm_np).cuda() if per_ray else None)
            h = parity.hits_to_numpy(rg.trace_closest(tl, rd, **kw))
            occ = rg.trace_any(tl, rd, **kw).cpu().numpy()
            okw = dict(cull=cull, ray_mask=rm_np if per_ray else None)
            res = parity.check_closest(h, orc.trace(rays, **okw), 0.002, label)
            parity.check_any(occ, orc.trace(rays, any_hit=True, **okw), 0.002, label)
            assert np.array_equal(occ != 0, h["inst"].astype(np.uint32) != 0xFFFFFFFF)
            print(f"  {res}", flush=True)


def test_full_masks_equal_no_masks_and_removal_restores():
    """All micro-triangles opaque: bitwise the hits without masks (through the
    option variant of the traversal); masks removed and the top level rebuilt:
    the plain traversal again."""
    rg = _rg()
    sc, masks, _ = _scene(32)
    rays = rg.rays_to_device(sg.random_rays(20000, 43, extent=4.0))
    plain = rg.upload_scene(sc)
    full = _tlas(sc, [(np.full(m.shape, ~np.uint64(0)), 3) for m in masks])
    assert full.desc.has_inst_flags == 1 and plain.desc.has_inst_flags == 0
    a = parity.hits_to_numpy(rg.trace_closest(plain, rays))
    b = parity.hits_to_numpy(rg.trace_closest(full, rays))
    for k in a:
        assert np.array_equal(a[k].view(np.uint32), b[k].view(np.uint32)), k
    assert np.array_equal(rg.trace_any(plain, rays).cpu().numpy(), rg.trace_any(full, rays).cpu().numpy())
    for bl in full.blas:
        rg.set_alpha(bl, None)
        assert bl.desc.has_alpha == 0
    again = rg.build_tlas(full.blas, sc.xform, sc.blas_id, sc.inst_mat, 4)
    assert again.desc.has_inst_flags == 0
    c = parity.hits_to_numpy(rg.trace_closest(again, rays))
    for k in a:
        assert np.array_equal(a[k].view(np.uint32), c[k].view(np.uint32)), k


def test_render_with_opacity_masks_matches_oracle():
    """A two-level frame whose meshes carry level-3 masks (every other
    micro-triangle of some triangles see-through): sampled pixels against the
    oracle's frame; shadow and bounce rays pass through the same holes."""
    rg = _rg()
    sc = sg.config_two_level(width=160, height=90, max_depth=3)
    rng = np.random.default_rng(50)
    alpha = []
    for m in sc.blas:
        mk = np.full(m.n_tris, ~np.uint64(0))
        holes = rng.random(m.n_tris) < 0.5
        mk[holes] = np.uint64(0x5555555555555555)
        alpha.append((mk, 3))
    print("[alpha render]", flush=True)
    tl = _tlas(sc, alpha, 4, 1)
    img = rg.render(tl, sc.materials, sc.camera, sc.light, sc.width, sc.height, sc.max_depth).cpu().numpy()
    px = sg.sample_pixels(sc.width, sc.height, 800, 51)
    ref = oracle.Scene(sc, sphere_reject=True, alpha=alpha).render(px)
    print(parity.check_image(img.reshape(-1, 3)[px], ref, 0.045, "alpha render"), flush=True)
    plain = rg.render(rg.upload_scene(sc, 4, 1), sc.materials, sc.camera, sc.light, sc.width, sc.height,
                      sc.max_depth).cpu().numpy()
    assert not np.array_equal(img, plain)


def test_masks_survive_a_refit():
    """The masks belong to the triangles (input order), not to the hierarchy:
    after a refit to moved vertices the top level rebuilt over the bottom
    level still ignores the transparent micro-triangles of the moved mesh."""
    rg = _rg()
    mesh = sg.torus(48, 40, 1.0, 0.35, 0.08, 6.0, 3004)
    moved = sg.Mesh(sg.animate_mesh(mesh, 0.3, amp=0.06, seed=9), mesh.idx)
    rng = np.random.default_rng(60)
    masks = rng.integers(0, 2 ** 63, mesh.n_tris, dtype=np.int64).astype(np.uint64)
    import torch
    v0 = torch.from_numpy(mesh.verts).cuda()
    idx = torch.from_numpy(mesh.idx.view(np.int32)).cuda()
    b = rg.build_blas(v0, idx, None, 4, 1, builder="treelet")
    rg.set_alpha(b, _masks(masks), 2)
    rg.refit_blas(b, torch.from_numpy(moved.verts).cuda(), idx)
    tl = rg.build_tlas([b], sg.identity_xform(1), [0], [0], 4)
    assert tl.desc.has_inst_flags == 1
    cen = moved.verts[moved.idx].mean(axis=1)
    rays = np.concatenate([sg.random_rays(3000, 61, extent=1.8),
                           sg.rays_through_points(cen[rng.integers(0, cen.shape[0], 3000)], 62, 3.0)])
    rd = rg.rays_to_device(rays)
    orc = oracle.Scene(scene_from_meshes([moved]), alpha=[(masks, 2)])
    print("[alpha refit]", flush=True)
    res = parity.check_closest(parity.hits_to_numpy(rg.trace_closest(tl, rd)), orc.trace(rays), 0.003, "alpha refit")
    parity.check_any(rg.trace_any(tl, rd).cpu().numpy(), orc.trace(rays, any_hit=True), 0.003, "alpha refit any")
    print(f"  {res}", flush=True)


def test_bad_masks_are_rejected():
    import torch
    rg = _rg()
    sc, masks, _ = _scene(33)
    tl = rg.upload_scene(sc)
    b = tl.blas[0]
    with pytest.raises(rg.RgError):
        rg.set_alpha(b, _masks(masks[0]), 4)
    with pytest.raises(ValueError):
        rg.set_alpha(b, _masks(masks[0][:10]), 3)
    with pytest.raises(ValueError):
        rg.set_alpha(b, torch.zeros(b.n_tris, dtype=torch.int32, device="cuda"), 3)
    torch.cuda.synchronize()
