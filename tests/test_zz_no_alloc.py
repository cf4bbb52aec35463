"""rg_render_static (the render entry point that allocates nothing: its
scratch is a device array inside the library) against rg_render with a
caller-allocated scratch buffer, through the C ABI: images bitwise equal on
two calls in a row, the second with a smaller frame, then an AO frame;
frames beyond the array are refused before anything runs."""
import numpy as np
import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu


def _frames(rg, tl, sc, W, H, D, mode=0, seed=0):
    import torch
    ref = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    scratch = torch.empty(rg.render_sizes(W, H, D, mode), dtype=torch.uint8, device="cuda")
    rg.render_into(tl, sc.materials, sc.camera, sc.light, W, H, D, ref, scratch, mode=mode, seed=seed)
    out = torch.full((H, W, 3), float("nan"), dtype=torch.float32, device="cuda")
    rg.render_static(tl, sc.materials, sc.camera, sc.light, W, H, D, out, mode=mode, seed=seed)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_static_render_matches_rg_render():
    import paper_2001_09792_amd as rg
    sc = sg.config_two_level(width=160, height=120)
    tl = rg.upload_scene(sc, width=4, leaf_max=1)
    for (W, H, D) in [(160, 120, 3), (96, 64, 1)]:
        assert rg.render_sizes(W, H, D, 0) <= rg.STATIC_SCRATCH_BYTES
        print(f"[no-alloc] two-level {W}x{H} depth {D}", flush=True)
        ref, out = _frames(rg, tl, sc, W, H, D)
        assert np.isfinite(ref).all() and ref.max() > 0
        assert np.array_equal(ref, out), f"{W}x{H} D{D}: max diff {np.abs(ref - out).max()}"
    # ambient occlusion through the same entry point
    print("[no-alloc] ambient occlusion 64x48", flush=True)
    ref, out = _frames(rg, tl, sc, 64, 48, 0, mode=1, seed=7)
    assert np.array_equal(ref, out)


def test_static_render_refuses_large_frames():
    import torch
    import paper_2001_09792_amd as rg
    sc = sg.config_small()
    tl = rg.upload_scene(sc)
    W, H, D = 512, 512, 4
    assert rg.render_sizes(W, H, D, 0) > rg.STATIC_SCRATCH_BYTES
    img = torch.zeros((H, W, 3), dtype=torch.float32, device="cuda")
    with pytest.raises(rg.RgError) as e:
        rg.render_static(tl, sc.materials, sc.camera, sc.light, W, H, D, img)
    assert e.value.status == -2
    torch.cuda.synchronize()
    assert float(img.abs().max()) == 0.0  # nothing ran
