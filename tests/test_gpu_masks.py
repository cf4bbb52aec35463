"""Ray visibility masks and face culling on the GPU (the accept / ignore
decisions of an any-hit stage, as instance masks and cull flags): the closed
forms of the hand scenes, parity with the FP64 oracle on random scenes under
every flag combination, the default options equal to the plain calls bit for
bit, and hidden instances leaving the rendered frame as if they were absent."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from tests import bvh_check, parity
from tests.helpers import quad, ray, scene_from_meshes, tri_scene

pytestmark = pytest.mark.gpu


def _rg():
    import paper_2001_09792_amd as rg
    return rg


def _closest(tl, rays, **kw):
    rg = _rg()
    return parity.hits_to_numpy(rg.trace_closest(tl, rg.rays_to_device(rays), **kw))


def _t(h, k=0):
    return float(h["t"][k])


def _upload(sc, flags=None, width=4, leaf=4, builder="lbvh"):
    rg = _rg()
    tl = rg.upload_scene(sc, width, leaf, builder=builder, inst_flags=flags)
    bvh_check.check_tlas(tl.buf.cpu().numpy(), tl.desc, [b.desc for b in tl.blas], sc.xform, inst_flags=flags)
    return tl


def test_single_quad_facing():
    rg = _rg()
    tl = _upload(tri_scene(quad(0.0, normal_sign=1.0)))
    rays = np.stack([ray((0.3, 0.2, 5.0), (0.0, 0.0, -1.0)), ray((0.3, 0.2, -5.0), (0.0, 0.0, 1.0))])
    print("[masks] single quad", flush=True)
    for cull, want in ((0, [5.0, 5.0]), (rg.RAY_CULL_BACK, [5.0, np.inf]), (rg.RAY_CULL_FRONT, [np.inf, 5.0]),
                       (rg.RAY_CULL_BACK | rg.RAY_CULL_FRONT, [np.inf, np.inf])):
        h = _closest(tl, rays, cull=cull)
        assert [_t(h, k) for k in (0, 1)] == pytest.approx(want, rel=1e-6), cull
        occ = rg.trace_any(tl, rg.rays_to_device(rays), cull=cull).cpu().numpy()
        assert list(occ) == [int(np.isfinite(w)) for w in want]


def test_stacked_quads():
    rg = _rg()
    tl = _upload(tri_scene(quad(0.0, normal_sign=1.0) + quad(-1.0, normal_sign=-1.0)))
    r = ray((0.1, -0.4, 5.0), (0.0, 0.0, -1.0))[None]
    assert _t(_closest(tl, r)) == pytest.approx(5.0, rel=1e-6)
    assert _t(_closest(tl, r, cull=rg.RAY_CULL_BACK)) == pytest.approx(5.0, rel=1e-6)
    h = _closest(tl, r, cull=rg.RAY_CULL_FRONT)
    assert _t(h) == pytest.approx(6.0, rel=1e-6) and int(h["prim"][0]) in (2, 3)


def _two_instances(xf2=None):
    X = sg.identity_xform(2)
    X[1, 2, 3] = -1.0
    if xf2 is not None:
        X[1] = xf2
    return scene_from_meshes([sg.triangles_mesh(quad(0.0, normal_sign=1.0))], xforms=X, blas_id=[0, 0])


@pytest.mark.parametrize("width", [2, 4, 8])
def test_instance_masks(width):
    import torch
    rg = _rg()
    tl = _upload(_two_instances(), np.array([0x01, 0x02], np.uint32), width)
    r = np.stack([ray((0.2, 0.1, 5.0), (0.0, 0.0, -1.0))] * 4)
    print(f"[masks] instance masks W{width}", flush=True)
    assert _t(_closest(tl, r[:1], mask=0x01)) == pytest.approx(5.0, rel=1e-6)
    h = _closest(tl, r[:1], mask=0x02)
    assert _t(h) == pytest.approx(6.0, rel=1e-6) and int(h["inst"][0]) == 1
    assert np.isinf(_t(_closest(tl, r[:1], mask=0x04)))
    assert _t(_closest(tl, r[:1], mask=0x03)) == pytest.approx(5.0, rel=1e-6)
    rm = torch.tensor([0x01, 0x02, 0x04, 0xFF], dtype=torch.uint8, device="cuda")
    h = _closest(tl, r, ray_mask=rm)
    assert [_t(h, k) for k in range(4)] == pytest.approx([5.0, 6.0, np.inf, 5.0], rel=1e-6)
    occ = rg.trace_any(tl, rg.rays_to_device(r), ray_mask=rm).cpu().numpy()
    assert list(occ) == [1, 1, 0, 1]
    tl0 = _upload(_two_instances(), np.array([0x00, 0xFF], np.uint32), width)
    assert _t(_closest(tl0, r[:1])) == pytest.approx(6.0, rel=1e-6)


def test_instance_flip_and_cull_disable():
    rg = _rg()
    down = ray((0.2, 0.1, 5.0), (0.0, 0.0, -1.0))[None]
    tl = _upload(_two_instances(), np.array([0xFF | rg.INST_FLIP_FACING, 0x00], np.uint32))
    assert np.isinf(_t(_closest(tl, down, cull=rg.RAY_CULL_BACK)))
    assert _t(_closest(tl, down, cull=rg.RAY_CULL_FRONT)) == pytest.approx(5.0, rel=1e-6)
    tl = _upload(_two_instances(), np.array([0xFF | rg.INST_CULL_DISABLE, 0xFF], np.uint32))
    assert _t(_closest(tl, down, cull=rg.RAY_CULL_FRONT)) == pytest.approx(5.0, rel=1e-6)
    assert _t(_closest(tl, down, cull=rg.RAY_CULL_BACK | rg.RAY_CULL_FRONT)) == pytest.approx(5.0, rel=1e-6)


def test_mirrored_instance_facing_is_object_space():
    rg = _rg()
    X = np.zeros((1, 3, 4), np.float32)
    X[0, 0, 0], X[0, 1, 1], X[0, 2, 2] = -1.0, 1.0, 1.0
    tl = _upload(scene_from_meshes([sg.triangles_mesh(quad(0.0, normal_sign=1.0))], xforms=X, blas_id=[0]))
    down = ray((0.2, 0.1, 5.0), (0.0, 0.0, -1.0))[None]
    assert _t(_closest(tl, down, cull=rg.RAY_CULL_BACK)) == pytest.approx(5.0, rel=1e-6)
    assert np.isinf(_t(_closest(tl, down, cull=rg.RAY_CULL_FRONT)))


def _random_scene(seed, n_inst=12):
    meshes = [sg.random_soup(600, seed, 1.0, 0.3), sg.icosphere(2), sg.torus(16, 12, 1.0, 0.3)]
    rng = np.random.default_rng(seed)
    xf = sg.random_instances(rng, n_inst, extent=2.5)
    # some mirrored instances: facing must still be decided in object space
    xf[::5, 0, :3] *= -1.0
    return scene_from_meshes(meshes, xforms=xf, blas_id=np.arange(n_inst) % 3), rng


@pytest.mark.parametrize("builder,width,leaf", [("lbvh", 2, 1), ("lbvh", 4, 4), ("ploc", 8, 3), ("lbvh", 8, 1)])
def test_parity_with_the_oracle_under_every_option(builder, width, leaf):
    """Every combination of the cull flags with instance masks, flip and
    cull-disable flags, a call mask and per-ray masks, against the oracle:
    closest hit within the tolerance, any hit exactly."""
    import torch
    rg = _rg()
    sc, rng = _random_scene(21)
    flags = rng.choice([0x01, 0x02, 0x03, 0x04, 0xFF], size=12).astype(np.uint32)
    flags[rng.random(12) < 0.3] |= rg.INST_FLIP_FACING
    flags[rng.random(12) < 0.3] |= rg.INST_CULL_DISABLE
    tl = _upload(sc, flags, width, leaf, builder)
    orc = oracle.Scene(sc, inst_flags=flags)
    rays = np.concatenate([sg.random_rays(2500, 31, extent=4.0),
                           sg.rays_through_points(rng.uniform(-2.5, 2.5, (2500, 3)), 32, 6.0)])
    rm_np = rng.choice([0x01, 0x02, 0x04, 0x06, 0xFF], size=rays.shape[0]).astype(np.uint8)
    rm = torch.from_numpy(rm_np).cuda()
    rd = rg.rays_to_device(rays)
    for cull in (0, rg.RAY_CULL_BACK, rg.RAY_CULL_FRONT, rg.RAY_CULL_BACK | rg.RAY_CULL_FRONT):
        for mask, per_ray in ((0xFF, False), (0x02, False), (0xFF, True)):
            label = f"{builder} W{width} L{leaf} cull={cull} mask={mask:#x} per_ray={per_ray}"
            print(f"[masks parity] {label}", flush=True)
            kw = dict(cull=cull, mask=mask, ray_mask=rm if per_ray else None)
            h = parity.hits_to_numpy(rg.trace_closest(tl, rd, **kw))
            occ = rg.trace_any(tl, rd, **kw).cpu().numpy()
            okw = dict(cull=cull, mask=mask, ray_mask=rm_np if per_ray else None)
            oc = orc.trace(rays, **okw)
            oa = orc.trace(rays, any_hit=True, **okw)
            sc_ = parity.check_closest(h, oc, 0.002, label)
            parity.check_any(occ, oa, 0.002, label)
            assert np.array_equal(occ != 0, h["inst"].astype(np.uint32) != 0xFFFFFFFF)
            if cull == rg.RAY_CULL_BACK | rg.RAY_CULL_FRONT:
                # culled everywhere except in the cull-disabled instances
                keep = h["inst"].astype(np.uint32) != 0xFFFFFFFF
                assert np.all(flags[h["inst"][keep].astype(np.int64)] & rg.INST_CULL_DISABLE)
            print(f"  {sc_}", flush=True)


def test_default_options_equal_the_plain_calls():
    """All-visible per-ray masks and no culling through the option calls, and
    all-visible instance flags in the top level, give the plain calls' hits
    bit for bit."""
    import torch
    rg = _rg()
    sc, _ = _random_scene(22)
    tl = _upload(sc)
    tlf = _upload(sc, np.full(12, 0xFF, np.uint32))
    rays = rg.rays_to_device(sg.random_rays(20000, 33, extent=4.0))
    ones = torch.full((rays.shape[1],), 0xFF, dtype=torch.uint8, device="cuda")
    plain = parity.hits_to_numpy(rg.trace_closest(tl, rays))
    for t, kw in ((tl, dict(ray_mask=ones)), (tlf, {}), (tlf, dict(mask=0xFF, ray_mask=ones))):
        h = parity.hits_to_numpy(rg.trace_closest(t, rays, **kw))
        for k in plain:
            assert np.array_equal(plain[k].view(np.uint32), h[k].view(np.uint32)), k
        assert np.array_equal(rg.trace_any(tl, rays).cpu().numpy(), rg.trace_any(t, rays, **kw).cpu().numpy())


def test_hidden_instances_leave_the_frame_as_if_absent():
    """A two-level frame with some instances masked 0 (seen by no ray, shadow
    and bounce rays included): the rendered pixels match the oracle's frame of
    the scene with those flags, and the GPU's frame of the scene without the
    hidden instances."""
    rg = _rg()
    sc = sg.config_two_level(width=160, height=90, max_depth=3)
    n = sc.xform.shape[0]
    rng = np.random.default_rng(40)
    hide = rng.random(n) < 0.3
    flags = np.where(hide, 0x00, 0xFF).astype(np.uint32)
    print(f"[masks render] hiding {int(hide.sum())} of {n} instances", flush=True)
    tl = _upload(sc, flags, 4, 1)
    img = rg.render(tl, sc.materials, sc.camera, sc.light, sc.width, sc.height, sc.max_depth).cpu().numpy()
    keep = np.nonzero(~hide)[0]
    sub = sg.Scene(sc.name, sc.blas, sc.xform[keep], sc.blas_id[keep], sc.inst_mat[keep], sc.materials, sc.camera,
                   sc.light, sc.width, sc.height, sc.max_depth, sc.mode, sc.seed)
    tl_sub = _upload(sub, None, 4, 1)
    img_sub = rg.render(tl_sub, sc.materials, sc.camera, sc.light, sc.width, sc.height, sc.max_depth).cpu().numpy()
    diff = np.abs(img.astype(np.float64) - img_sub).max()
    print(f"  hidden vs absent: max |diff| {diff:.3g}, bitwise {np.array_equal(img, img_sub)}", flush=True)
    assert diff <= 1e-5
    px = sg.sample_pixels(sc.width, sc.height, 800, 41)
    ref = oracle.Scene(sc, sphere_reject=True, inst_flags=flags).render(px, width=sc.width, height=sc.height,
                                                                          max_depth=sc.max_depth)
    print(parity.check_image(img.reshape(-1, 3)[px], ref, 0.01, "masked render"), flush=True)


def _flagged_frames():
    """Three small two-level frames: one with hidden instances, one with all
    instances visible through explicit flags, one without flags."""
    rg = _rg()
    out = []
    for k, mode in enumerate(("hidden", "all", "none")):
        sc = sg.config_two_level(seed=60 + k, width=48 + 16 * k, height=40, max_depth=2 + k)
        n = sc.xform.shape[0]
        if mode == "hidden":
            flags = np.where(np.arange(n) % 3 == 0, 0x00, 0xFF).astype(np.uint32)
        elif mode == "all":
            flags = np.full(n, 0xFF, np.uint32)
        else:
            flags = None
        tl = rg.upload_scene(sc, inst_flags=flags)
        assert tl.desc.has_inst_flags == (1 if mode == "hidden" else 0)
        out.append((tl, sc.materials, sc.camera, sc.light, sc.width, sc.height, sc.max_depth))
    return out


def test_batch_and_engine_frames_with_instance_flags_equal_frames_alone():
    """Frames whose top levels carry instance flags, batched or served with
    frames whose top levels do not: each image equals its frame alone."""
    import torch
    rg = _rg()
    frames = _flagged_frames()
    print("[masks batch/engine]", flush=True)
    alone = [rg.Renderer(W, H, D).render(tl, m, c, l).cpu().numpy().copy() for tl, m, c, l, W, H, D in frames]
    imgs = [i.cpu().numpy() for i in rg.Batch(frames).render()]
    for k in range(len(frames)):
        assert np.array_equal(imgs[k], alone[k]), f"batch frame {k}"
    eng = rg.Engine(1 << 22, 1 << 20, max_jobs=8)
    out = {}
    for k, (tl, m, c, l, W, H, D) in enumerate(frames):
        out[k] = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
        assert eng.admit(tl, rg.materials_array(m), c, l, W, H, D, out[k], k)
        eng.step()
    done = []
    while eng.step():
        done += eng.poll()
    while len(done) < len(frames):
        done += eng.poll(wait=True)
    for k in range(len(frames)):
        assert np.array_equal(out[k].cpu().numpy(), alone[k]), f"engine frame {k}"
    eng.close()
    # the hidden instances are absent from the frame
    tl, m, c, l, W, H, D = frames[0]
    assert not np.array_equal(alone[0], rg.Renderer(W, H, D).render(rg.upload_scene(
        sg.config_two_level(seed=60, width=W, height=H, max_depth=D)), m, c, l).cpu().numpy())


def test_bad_options_are_rejected():
    import torch
    rg = _rg()
    sc, _ = _random_scene(23)
    tl = _upload(sc)
    rays = rg.rays_to_device(sg.random_rays(100, 34))
    with pytest.raises(rg.RgError):
        rg.trace_closest(tl, rays, cull=4)
    with pytest.raises(rg.RgError):
        rg.trace_any(tl, rays, mask=0x100)
    with pytest.raises(ValueError):
        rg.trace_closest(tl, rays, ray_mask=torch.zeros(100, dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError):
        rg.trace_closest(tl, rays, ray_mask=torch.zeros(50, dtype=torch.uint8, device="cuda"))
    with pytest.raises(rg.RgError):
        rg.upload_scene(sc, inst_flags=np.full(12, 1 << 12, np.uint32))
    torch.cuda.synchronize()
