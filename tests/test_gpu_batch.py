"""Batched rendering (a14): frames of many scenes of uneven size advanced
together, one launch per pass.  Each frame must be bitwise the frame
rendered alone, and match the oracle on sampled pixels."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from tests import parity

pytestmark = pytest.mark.gpu


def _frames(scenes):
    import paper_2001_09792_amd as rg
    out = []
    for sc in scenes:
        tl = rg.upload_scene(sc)
        out.append((tl, sc.materials, sc.camera, sc.light, sc.width, sc.height, sc.max_depth))
    return out


def test_batch_equals_frames_alone():
    import torch
    import paper_2001_09792_amd as rg
    scenes = sg.config_batched(seed=41, n_scenes=12, tri_range=(1e3, 2e4), max_inst=24, pix_range=(16 ** 2, 96 ** 2))
    scenes[3].max_depth = 0       # frames may have different depth caps
    scenes[5].max_depth = 3
    print("[batch] 12 scenes", [(s.unique_tris(), s.n_inst, s.width, s.max_depth) for s in scenes], flush=True)
    frames = _frames(scenes)
    b = rg.Batch(frames, seed=0)
    imgs, st = b.render(stats=True)
    imgs = [i.cpu().numpy().copy() for i in imgs]
    total_rays = 0
    for k, (tl, mats, cam, light, W, H, D) in enumerate(frames):
        alone, s1 = rg.Renderer(W, H, D).render(tl, mats, cam, light, stats=True)
        assert np.array_equal(alone.cpu().numpy(), imgs[k]), f"frame {k} differs from its batch image"
        total_rays += s1["rays_traced"]
    assert st["rays_traced"] == total_rays
    again = [i.cpu().numpy() for i in b.render()]
    assert all(np.array_equal(x, y) for x, y in zip(imgs, again))
    torch.cuda.synchronize()


@pytest.mark.parametrize("k", [0, 2, 7])
def test_batch_frames_match_oracle(k):
    import paper_2001_09792_amd as rg
    scenes = sg.config_batched(seed=42, n_scenes=8, tri_range=(1e3, 1e4), max_inst=16, pix_range=(24 ** 2, 64 ** 2))
    frames = _frames(scenes)
    imgs = [i.cpu().numpy().reshape(-1, 3).copy() for i in rg.Batch(frames).render()]
    sc = scenes[k]
    px = sg.sample_pixels(sc.width, sc.height, 400, 7 + k)
    ref = oracle.Scene(sc, sphere_reject=True).render(px)
    res = parity.check_image(imgs[k][px], ref, 0.008, f"batch frame {k}")
    print(res, flush=True)


def test_batch_rejects_mixed_widths():
    import paper_2001_09792_amd as rg
    scenes = sg.config_batched(seed=43, n_scenes=2, tri_range=(1e3, 2e3), max_inst=4, pix_range=(16 ** 2, 32 ** 2))
    tl4 = rg.upload_scene(scenes[0], width=4)
    tl8 = rg.upload_scene(scenes[1], width=8)
    f = [(tl4, scenes[0].materials, scenes[0].camera, scenes[0].light, 16, 16, 1),
         (tl8, scenes[1].materials, scenes[1].camera, scenes[1].light, 16, 16, 1)]
    with pytest.raises(rg.RgError):
        rg.Batch(f)


def test_batch_graph_replays_match_eager():
    """A batch captured into a HIP graph: every replay, with eager work and
    synchronisations between replays, gives the eager images bitwise."""
    import torch
    import paper_2001_09792_amd as rg
    scenes = sg.config_batched(seed=43, n_scenes=8, tri_range=(1e3, 1e4), max_inst=12, pix_range=(16 ** 2, 64 ** 2))
    frames = _frames(scenes)
    b = rg.Batch(frames, seed=0)
    eager = [i.clone() for i in b.render()]
    torch.cuda.synchronize()
    print("[batch] capturing 8 frames", flush=True)
    g = b.capture()
    for rep in range(4):
        for img in b.images:
            img.fill_(-1.0)          # the replay must rewrite every pixel
        g.replay()
        torch.cuda.synchronize()
        for k, (img, ref) in enumerate(zip(b.images, eager)):
            assert torch.equal(img, ref), f"replay {rep}, frame {k}"
        # eager work on the same buffers between replays
        b.render()
        torch.cuda.synchronize()
    del g


def test_full_size_batched_workload():
    """The batched benchmark's own input (256 scenes: triangles log-uniform
    in 1e3..2e6, 1..128 instances, 64^2..1024^2 pixels, depth 2) in one
    batch on its hierarchy shape: 16 frames spread over the batch are bitwise
    the frames rendered alone, and 4 of them match the oracle on sampled
    pixels."""
    import torch
    import paper_2001_09792_amd as rg
    scenes = sg.config_batched()
    assert len(scenes) == 256
    print(f"[batch] 256 scenes, {sum(s.unique_tris() for s in scenes)} unique tris, "
          f"{sum(s.width * s.height for s in scenes)} pixels", flush=True)
    frames = []
    for sc in scenes:
        tl = rg.upload_scene(sc, width=4, leaf_max=1, builder="lbvh")
        frames.append((tl, sc.materials, sc.camera, sc.light, sc.width, sc.height, sc.max_depth))
    b = rg.Batch(frames)
    imgs = b.render()
    torch.cuda.synchronize()
    rng = np.random.default_rng(256)
    pick = np.sort(rng.choice(256, 16, replace=False))
    for k in pick:
        tl, mats, cam, light, W, H, D = frames[k]
        alone = rg.Renderer(W, H, D).render(tl, mats, cam, light)
        assert torch.equal(alone, imgs[k]), f"frame {k} ({W}x{H}) differs from its batch image"
    print(f"[batch] frames {pick.tolist()} bitwise equal to rendering alone", flush=True)
    for k in pick[::4]:
        sc = scenes[k]
        px = sg.sample_pixels(sc.width, sc.height, 64, 1000 + int(k))
        ref = oracle.Scene(sc, sphere_reject=True).render(px)
        res = parity.check_image(imgs[k].cpu().numpy().reshape(-1, 3)[px], ref, 0.05, f"batch frame {k}")
        print(f"[batch] frame {k} ({sc.unique_tris()} tris, {sc.n_inst} instances): {res}", flush=True)
