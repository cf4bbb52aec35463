"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times: the incoherent workload's scene (10,035,200 unique triangles, 1,024
instances) on its hierarchy shape and default launch parameters, traced in
launches of the benchmark's sizes (2,073,600 camera rays, about 10.3 million
AO rays) whose rays are oracle-generated camera and AO rays of sampled pixels,
repeated to fill the launch; the same AO launch with the ray options on
(culling, instance masks, opacity masks); and the two-level 1080p depth-4
frame on its shape, sampled pixels against the oracle's."""
import numpy as np
import pytest

import bench
import oracle
import scenegen as sg
from tests import parity

pytestmark = pytest.mark.gpu


def _tiled(rays, n):
    """n rays cycling through `rays` (f32 [k, 8])."""
    return rays[np.arange(n) % rays.shape[0]]


def _check_tiles(h, k, label):
    """Every copy of a ray gets the first copy's result bit for bit."""
    n = h["t"].shape[0]
    for key, v in h.items():
        v = v.view(np.uint32) if v.dtype == np.float32 else v
        first = v[:k]
        reps = n // k
        assert np.array_equal(v[: reps * k].reshape(reps, k), np.broadcast_to(first, (reps, k))), (label, key)
        assert np.array_equal(v[reps * k:], first[: n - reps * k]), (label, key)


def test_incoherent_workload_at_full_size():
    import torch
    import paper_2001_09792_amd as rg
    width, leaf, builder = bench.SHAPES["incoherent"]
    scene = sg.config_incoherent()
    W, H = scene.width, scene.height
    print(f"[full size] incoherent: {scene.unique_tris()} unique tris, W{width} L{leaf} {builder}, "
          f"launch parameters {rg.trace_tuning(scope='trace')}", flush=True)
    tl = rg.upload_scene(scene, width=width, leaf_max=leaf, builder=builder)
    orc = oracle.Scene(scene, sphere_reject=True)
    px = sg.sample_pixels(W, H, 256, 71)
    cam = np.zeros((px.shape[0], 8), np.float32)
    cam[:, :6] = oracle.camera_rays(scene.camera, W, H, px)
    cam[:, 7] = np.inf
    ao = orc.ao_rays(cam, scene.seed)
    hit = ao["hit"] == 1
    aor = np.zeros((int(hit.sum()) * 8, 8), np.float32)
    aor[:, :6] = ao["rays"][hit].reshape(-1, 6)
    aor[:, 7] = 5.0
    n_ao = 10_315_840     # the benchmark's AO launch: 8 rays for each of its 1,289,480 primary hits
    for label, rays, n in (("camera", cam, W * H), ("ao", aor, n_ao)):
        print(f"[full size] {label}: {rays.shape[0]} distinct rays in a launch of {n}", flush=True)
        d = rg.rays_to_device(_tiled(rays, n))
        h = parity.hits_to_numpy(rg.trace_closest(tl, d))
        _check_tiles(h, rays.shape[0], label)
        first = {k: v[: rays.shape[0]] for k, v in h.items()}
        res = parity.check_closest(first, orc.trace(rays), 0.006, f"full-size {label}")
        occ = rg.trace_any(tl, d).cpu().numpy()
        assert np.array_equal(occ[: rays.shape[0]], occ[rays.shape[0]: 2 * rays.shape[0]])
        parity.check_any(occ[: rays.shape[0]], orc.trace(rays, any_hit=True), 0.006, f"full-size {label} any")
        print(f"  {res}", flush=True)
        del d
        torch.cuda.empty_cache()


def test_options_workload_at_full_size():
    """The options workload's launch: about 10.3 million AO rays traced with
    back faces culled and ray mask 0x02 over the incoherent scene whose top
    level flags half of the instances out of that mask and whose even meshes
    carry level-3 opacity masks."""
    import torch
    import paper_2001_09792_amd as rg
    width, leaf, builder = bench.SHAPES["options"]
    scene = sg.config_incoherent()
    flags, alpha = sg.option_inputs(scene)
    print(f"[full size] options: W{width} L{leaf} {builder}, {sum(a is not None for a in alpha)} alpha-tested "
          f"meshes, launch parameters {rg.trace_tuning(scope='trace')}", flush=True)
    tl = rg.upload_scene(scene, width=width, leaf_max=leaf, builder=builder)
    for b, a in zip(tl.blas, alpha):
        if a is not None:
            rg.set_alpha(b, torch.from_numpy(a[0].view(np.int64)).cuda(), a[1])
    opt = rg.build_tlas(tl.blas, scene.xform, scene.blas_id, scene.inst_mat, width, builder=builder,
                        inst_flags=flags)
    assert opt.desc.has_inst_flags == 1
    W, H = scene.width, scene.height
    px = sg.sample_pixels(W, H, 256, 73)
    cam = np.zeros((px.shape[0], 8), np.float32)
    cam[:, :6] = oracle.camera_rays(scene.camera, W, H, px)
    cam[:, 7] = np.inf
    ao = oracle.Scene(scene, sphere_reject=True).ao_rays(cam, scene.seed)
    hit = ao["hit"] == 1
    aor = np.zeros((int(hit.sum()) * 8, 8), np.float32)
    aor[:, :6] = ao["rays"][hit].reshape(-1, 6)
    aor[:, 7] = 5.0
    orc = oracle.Scene(scene, sphere_reject=True, inst_flags=flags, alpha=alpha)
    k = aor.shape[0]
    n_ao = 10_315_840
    print(f"[full size] options ao: {k} distinct rays in a launch of {n_ao}", flush=True)
    d = rg.rays_to_device(_tiled(aor, n_ao))
    h = parity.hits_to_numpy(rg.trace_closest(opt, d, mask=0x02, cull=rg.RAY_CULL_BACK))
    _check_tiles(h, k, "options ao")
    first = {key: v[:k] for key, v in h.items()}
    ref = orc.trace(aor, mask=0x02, cull=oracle.RAY_CULL_BACK)
    res = parity.check_closest(first, ref, 0.008, "full-size options ao")
    # the options change the answer: the plain oracle finds hits they remove
    plain_hit = oracle.Scene(scene, sphere_reject=True).trace(aor)["hit"] == 1
    assert (plain_hit & (ref["hit"] == 0)).sum() > 0.05 * plain_hit.sum()
    occ = rg.trace_any(opt, d, mask=0x02, cull=rg.RAY_CULL_BACK).cpu().numpy()
    assert np.array_equal(occ[:k], occ[k: 2 * k])
    parity.check_any(occ[:k], orc.trace(aor, any_hit=True, mask=0x02, cull=oracle.RAY_CULL_BACK), 0.008,
                     "full-size options any")
    print(f"  {res}", flush=True)


def test_two_level_frame_at_full_size():
    import paper_2001_09792_amd as rg
    width, leaf, builder = bench.SHAPES["two_level"]
    sc = sg.config_two_level()
    print(f"[full size] two-level {sc.width}x{sc.height} D={sc.max_depth}, W{width} L{leaf} {builder}, "
          f"launch parameters {rg.trace_tuning(scope='frame')}", flush=True)
    tl = rg.upload_scene(sc, width=width, leaf_max=leaf, builder=builder)
    img = rg.Renderer(sc.width, sc.height, sc.max_depth).render(tl, sc.materials, sc.camera, sc.light, sc.seed)
    img = img.cpu().numpy().reshape(-1, 3)
    px = sg.sample_pixels(sc.width, sc.height, 400, 72)
    ref = oracle.Scene(sc, sphere_reject=True).render(px)
    print(parity.check_image(img[px], ref, 0.01, "full-size two-level"), flush=True)
