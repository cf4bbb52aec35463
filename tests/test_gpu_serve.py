"""Serving on the GPU (a15): frames rendered by the continuous-batching engine
while others are in flight are bitwise the frames rendered alone (64-bit
fixed-point sums), whatever the overlap; the engine's frames match the FP64
oracle; admission refuses what does not fit and queues what does not fit
yet."""
import math

import numpy as np
import pytest

import oracle
import scenegen as sg
from tests import parity

pytestmark = pytest.mark.gpu

SIZES = ((64, 64), (96, 64), (128, 96), (160, 120))


@pytest.fixture(scope="module")
def pool():
    """Four resident scenes: the small configuration, a two-level scene and
    two scenes sharing one set of displaced tori (shared bottom levels)."""
    import paper_2001_09792_amd as rg
    from paper_2001_09792_amd import serve
    scenes = [sg.config_small(), sg.config_two_level(seed=5000)]
    shared = sg.c3_meshes(24)
    scenes += [sg.serving_c3_scene(5100, shared), sg.serving_c3_scene(5101, shared)]
    c3_blas = []

    def load(k):
        sc = scenes[k]
        if k >= 2:
            if not c3_blas:
                c3_blas.extend(rg.upload_scene(scenes[2]).blas)
            tl = rg.build_tlas(c3_blas, sc.xform, sc.blas_id, sc.inst_mat)
        else:
            tl = rg.upload_scene(sc)
        return (tl, rg.materials_array(sc.materials), sc.camera, sc.light), int(tl.buf.numel())

    cache = serve.ResidentCache(load)
    for k in range(len(scenes)):
        cache.get(k)
        cache.release(k)
    return scenes, cache


def _alone(cache, req):
    import torch
    import paper_2001_09792_amd as rg
    tl, ma, cam, light = cache.get(req.scene)
    img = torch.empty((req.height, req.width, 3), dtype=torch.float32, device="cuda")
    scratch = torch.empty(rg.render_sizes(req.width, req.height, req.depth, 0), dtype=torch.uint8, device="cuda")
    rg.render_into(tl, ma, cam, light, req.width, req.height, req.depth, img, scratch)
    cache.release(req.scene)
    return img


def _requests(n, seed, n_scenes=4):
    from paper_2001_09792_amd import serve
    return serve.poisson_requests(n, math.inf, n_scenes, seed, resolutions=SIZES, depths=(0, 1, 2, 3, 4))


def test_engine_scripted_overlap_matches_alone(pool):
    """Frames admitted one pass apart share passes at different depths."""
    import torch
    import paper_2001_09792_amd as rg
    scenes, cache = pool
    reqs = _requests(10, 21)
    for k, r in enumerate(reqs):
        r.depth = 4 if k % 2 == 0 else r.depth
    eng = rg.Engine(1 << 22, 1 << 20, max_jobs=16)
    imgs, done = {}, []
    print("[serve] scripted overlap, 10 frames", flush=True)
    for r in reqs:
        tl, ma, cam, light = cache.get(r.scene)
        imgs[r.rid] = torch.empty((r.height, r.width, 3), dtype=torch.float32, device="cuda")
        assert eng.admit(tl, ma, cam, light, r.width, r.height, r.depth, imgs[r.rid], r.rid)
        assert eng.step()
        done += eng.poll()
    while eng.step():
        done += eng.poll()
    while len(done) < len(reqs):
        done += eng.poll(wait=True)
    info = eng.info()
    print(info, flush=True)
    assert sorted(done) == [r.rid for r in reqs]
    assert info["max_frames_in_pass"] >= 4 and info["max_depths_in_pass"] >= 3
    assert info["frames_live"] == 0 and info["rays_reserved"] == 0
    for r in reqs:
        cache.release(r.scene)
        assert torch.equal(imgs[r.rid], _alone(cache, r)), f"request {r}"
    st = eng.stats()
    assert st["rays_traced"] >= sum(r.pixels for r in reqs)
    eng.close()


def test_serve_loop_mix_matches_alone(pool):
    """Poisson arrivals through serve(): every image equals the frame alone."""
    import torch
    import paper_2001_09792_amd as rg
    from paper_2001_09792_amd import serve
    scenes, cache = pool
    reqs = serve.poisson_requests(40, 2000.0, 4, 33, resolutions=SIZES, depths=(0, 1, 2, 3, 4))
    eng = rg.Engine(1 << 22, 1 << 20, max_jobs=32)
    ex = serve.EngineExecutor(eng, cache, keep_images=True)
    print("[serve] poisson mix, 40 frames", flush=True)
    info = serve.serve(reqs, ex, serve.RealClock())
    assert info["order"] == [r.rid for r in reqs]
    print(eng.info(), serve.summarize(reqs), flush=True)
    for r in reqs:
        assert torch.equal(ex.images[r.rid], _alone(cache, r)), f"request {r}"
    eng.close()


def test_tiny_budget_queues_and_stays_exact(pool):
    import torch
    import paper_2001_09792_amd as rg
    from paper_2001_09792_amd import serve
    scenes, cache = pool
    reqs = _requests(16, 44)
    big = max(rg.job_reservation(cache.get(r.scene)[1], r.width, r.height, r.depth)[0] for r in reqs)
    for r in reqs:
        cache.release(r.scene)
    eng = rg.Engine(big, 160 * 120, max_jobs=4)
    ex = serve.EngineExecutor(eng, cache, keep_images=True)
    print(f"[serve] tiny budget: {big} entries", flush=True)
    info = serve.serve(reqs, ex, serve.RealClock())
    assert info["max_waiting"] >= 8
    assert eng.info()["completed"] == len(reqs)
    for r in reqs:
        assert torch.equal(ex.images[r.rid], _alone(cache, r)), f"request {r}"
    eng.close()


def test_plain_executor_matches_engine(pool):
    import torch
    from paper_2001_09792_amd import serve
    scenes, cache = pool
    reqs = _requests(6, 55)
    ex = serve.PlainExecutor(cache, 160 * 120, 4, keep_images=True)
    serve.serve(reqs, ex, serve.RealClock())
    for r in reqs:
        assert torch.equal(ex.images[r.rid], _alone(cache, r))


def test_engine_frame_matches_oracle(pool):
    """A frame rendered in a mix against the FP64 oracle (small scene, full
    frame, and sampled pixels of a two-level frame)."""
    import torch
    import paper_2001_09792_amd as rg
    scenes, cache = pool
    eng = rg.Engine(1 << 22, 1 << 20, max_jobs=8)
    frames = [(0, 128, 128, 1), (1, 160, 90, 4), (0, 96, 64, 3)]
    imgs = []
    for k, (s, W, H, D) in enumerate(frames):
        tl, ma, cam, light = cache.get(s)
        imgs.append(torch.empty((H, W, 3), dtype=torch.float32, device="cuda"))
        assert eng.admit(tl, ma, cam, light, W, H, D, imgs[-1], k)
        eng.step()
    done = eng.poll()
    while eng.step():
        done += eng.poll()
    while len(done) < len(frames):
        done += eng.poll(wait=True)
    for s, *_ in frames:
        cache.release(s)
    sc0 = scenes[0]
    ref = oracle.Scene(sc0).render(width=128, height=128, max_depth=1)
    print(parity.check_image(imgs[0].cpu().numpy().reshape(-1, 3), ref, 0.002, "engine small"), flush=True)
    sc1 = scenes[1]
    px = sg.sample_pixels(160, 90, 1000, 13)
    ref = oracle.Scene(sc1, sphere_reject=True).render(px, width=160, height=90, max_depth=4)
    print(parity.check_image(imgs[1].cpu().numpy().reshape(-1, 3)[px], ref, 0.015, "engine two-level"), flush=True)
    eng.close()


def test_engine_admission_errors(pool):
    import torch
    import paper_2001_09792_amd as rg
    scenes, cache = pool
    tl, ma, cam, light = cache.get(0)
    img = torch.empty((64, 64, 3), dtype=torch.float32, device="cuda")
    eng = rg.Engine(64 * 64 * 2, 64 * 64 * 2, max_jobs=2)
    big = torch.empty((128, 128, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(rg.RgError) as e:
        eng.admit(tl, ma, cam, light, 128, 128, 1, big, 0)      # exceeds the whole engine
    assert e.value.status == -2
    assert eng.admit(tl, ma, cam, light, 64, 64, 1, img, 1)
    assert eng.admit(tl, ma, cam, light, 64, 64, 1, img, 2)
    assert not eng.admit(tl, ma, cam, light, 64, 64, 1, img, 3)  # full: retry later
    with pytest.raises(rg.RgError):
        eng.admit(tl, ma, cam, light, 64, 64, rg.MAX_DEPTH + 1, img, 4)
    while eng.step():
        pass
    done = []
    while len(done) < 2:
        done += eng.poll(wait=True)
    assert sorted(done) == [1, 2]
    assert eng.admit(tl, ma, cam, light, 64, 64, 1, img, 3)
    eng.close()
    w2 = rg.upload_scene(scenes[0], width=2)
    eng2 = rg.Engine(1 << 16, 1 << 16, max_jobs=2, width=4)
    with pytest.raises(rg.RgError) as e:
        eng2.admit(w2, ma, cam, light, 64, 64, 1, img, 0)       # another node width
    assert e.value.status == -4
    eng2.close()
    cache.release(0)


def test_full_pool_serving_mix_matches_alone():
    """The serving benchmark's own pool (64 resident scenes: 32 two-level
    scenes and 32 scenes over the 16 shared displaced tori of 560^2 segments,
    on the benchmark's hierarchy shape) and request mix (256^2 .. 1920x1080,
    depth 1..4): 60 requests arriving faster than they are served go through
    serve() with the continuous-batching engine, and every image is bitwise
    the frame rendered alone with rg_render."""
    import torch
    import paper_2001_09792_amd as rg
    from paper_2001_09792_amd import serve
    scenes = sg.config_serving_pool()
    assert len(scenes) == 64
    n_c2 = sum(1 for s in scenes if s.n_inst == 64)
    shared = []

    def load(k):
        sc = scenes[k]
        if k >= n_c2:
            if not shared:
                shared.extend(rg.upload_scene(sc, width=4, leaf_max=1, builder="treelet").blas)
            tl = rg.build_tlas(shared, sc.xform, sc.blas_id, sc.inst_mat, 4, builder="treelet")
        else:
            tl = rg.upload_scene(sc, width=4, leaf_max=1, builder="treelet")
        return (tl, rg.materials_array(sc.materials), sc.camera, sc.light), int(tl.buf.numel())

    cache = serve.ResidentCache(load)
    for k in range(64):
        cache.get(k)
        cache.release(k)
    reqs = serve.poisson_requests(60, 2000.0, 64, 77)
    assert {r.width for r in reqs} >= {256, 512, 1280, 1920}
    eng = rg.Engine(**rg.Engine.for_budget(8 << 30, max_jobs=64, width=4))
    ex = serve.EngineExecutor(eng, cache, keep_images=True)
    print(f"[serve] full pool, 60 requests: {sorted(set((r.width, r.height) for r in reqs))}", flush=True)
    info = serve.serve(reqs, ex, serve.RealClock())
    einfo = eng.info()
    print(einfo, serve.summarize(reqs), flush=True)
    assert einfo["completed"] == 60 and einfo["max_frames_in_pass"] >= 4
    for r in reqs:
        assert torch.equal(ex.images[r.rid], _alone(cache, r)), f"request {r}"
    eng.close()


def test_engine_holds_frame_buffers_until_polled(pool):
    """The engine's passes use a frame's top level and image after admit()
    returns: the binding keeps them alive until poll() hands back the tag, so
    a caller that drops its own references cannot free them under the GPU."""
    import gc
    import weakref
    import torch
    import paper_2001_09792_amd as rg
    scenes, cache = pool
    sc = scenes[1]
    eng = rg.Engine(1 << 22, 1 << 20, max_jobs=4)
    tl = rg.upload_scene(sc)
    img = torch.empty((90, 160, 3), dtype=torch.float32, device="cuda")
    w_tl, w_img = weakref.ref(tl), weakref.ref(img)
    assert eng.admit(tl, sc.materials, sc.camera, sc.light, 160, 90, 2, img, 7)
    del tl, img
    gc.collect()
    assert w_tl() is not None and w_img() is not None      # held by the engine
    done = []
    while eng.step():
        done += eng.poll()
    while 7 not in done:
        assert w_tl() is not None and w_img() is not None  # still in flight: still held
        done += eng.poll(wait=True)
    gc.collect()
    assert w_tl() is None and w_img() is None              # released with the tag
    eng.close()
