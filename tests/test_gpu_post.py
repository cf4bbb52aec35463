"""The frame's post-process passes on the GPU (roughness blur, FXAA) against
the FP64 oracle on synthetic aliased frames, element by element: the blur on
every pixel, FXAA on every pixel whose decisions float32 cannot flip; the
render's primary materials against the oracle's primary hits."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from oracle import post as opost

pytestmark = pytest.mark.gpu

ATOL, RTOL = 2e-5, 1e-5


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t if dtype is None else t.to(dtype)).cuda()


def _mat_dev(mat):
    import torch
    return _dev(np.ascontiguousarray(mat, np.uint32).view(np.int32), torch.int32)


def _close(g, o, mask=None, label=""):
    g = g.astype(np.float64)
    bad = np.abs(g - o) > ATOL + RTOL * np.abs(o)
    if mask is not None:
        bad &= mask[..., None]
    n = int(bad.any(axis=-1).sum())
    if n:
        i = np.argwhere(bad.any(axis=-1))[:5]
        print(f"{label}: {n} pixels differ, e.g. {i.tolist()}: gpu {g[tuple(i[0])]}, oracle {o[tuple(i[0])]}",
              flush=True)
    assert n == 0
    if mask is not None:
        return float(np.abs(g - o)[mask].max()) if mask.any() else 0.0
    return float(np.abs(g - o).max())


FRAMES = [(97, 61, 1), (256, 160, 2), (1920, 1080, 3), (1, 1, 4), (1, 37, 5), (53, 1, 6), (64, 4, 7)]


@pytest.mark.parametrize("w,h,seed", FRAMES)
@pytest.mark.parametrize("radius", [1, 8, 16])
def test_roughness_blur_matches_oracle(w, h, seed, radius):
    import paper_2001_09792_amd as rg
    img, mat = sg.post_frame(w, h, seed)
    rough = sg.roughness_table(8, seed)
    print(f"[blur] {w}x{h} R={radius}", flush=True)
    P = rg.Post(w, h)
    out = P.roughness_blur(_dev(img), _mat_dev(mat), _dev(rough), radius).cpu().numpy()
    ref = opost.roughness_blur(img, mat, rough, radius)
    err = _close(out, ref, label=f"blur {w}x{h} R{radius}")
    # pixels the blur leaves alone are copied bit for bit
    keep = (mat == sg.MISS) | (rough[np.minimum(mat, 7)] < 1.0 / 256.0)
    assert np.array_equal(out[keep], img[keep])
    print(f"  max |diff| {err:.3g}", flush=True)


@pytest.mark.parametrize("w,h,seed", FRAMES)
def test_fxaa_matches_oracle(w, h, seed):
    import paper_2001_09792_amd as rg
    img, _ = sg.post_frame(w, h, seed)
    print(f"[fxaa] {w}x{h}", flush=True)
    out = rg.Post(w, h).fxaa(_dev(img)).cpu().numpy()
    r = opost.fxaa(img)
    ok = ~r["amb"]
    # in images one pixel wide or tall every edge runs along the clamped
    # border, where the luma at the search's ends equals the local average up
    # to rounding: many pixels sit on that decision
    assert ok.mean() >= (0.99 if min(w, h) >= 8 else 0.5)
    err = _close(out, r["rgb"], ok, f"fxaa {w}x{h}")
    keep = ~r["active"] & ok
    assert np.array_equal(out[keep], img[keep])
    print(f"  active {r['active'].mean():.4f} ambiguous {1 - ok.mean():.5f} max |diff| {err:.3g}", flush=True)


def test_radius_zero_and_smooth_materials_copy_the_image():
    import paper_2001_09792_amd as rg
    img, mat = sg.post_frame(80, 50, 9)
    P = rg.Post(80, 50)
    rough = _dev(sg.roughness_table(8, 9))
    assert np.array_equal(P.roughness_blur(_dev(img), _mat_dev(mat), rough, 0).cpu().numpy(), img)
    assert np.array_equal(P.roughness_blur(_dev(img), _mat_dev(mat), _dev(np.zeros(8, np.float32)), 8)
                          .cpu().numpy(), img)
    sky = np.full_like(mat, sg.MISS)
    assert np.array_equal(P.roughness_blur(_dev(img), _mat_dev(sky), rough, 8).cpu().numpy(), img)


def test_flat_image_passes_fxaa_unchanged():
    import paper_2001_09792_amd as rg
    img = np.full((33, 70, 3), 0.37, np.float32)
    assert np.array_equal(rg.Post(70, 33).fxaa(_dev(img)).cpu().numpy(), img)


def test_render_primary_materials_match_the_oracle():
    """The material each primary ray shaded, against the material of the
    oracle's closest hit for the same camera ray (sky where it misses)."""
    import torch
    import paper_2001_09792_amd as rg
    sc = sg.config_two_level(width=200, height=120, max_depth=2)
    tl = rg.upload_scene(sc)
    pm = torch.empty((sc.height, sc.width), dtype=torch.int32, device="cuda")
    R = rg.Renderer(sc.width, sc.height, sc.max_depth)
    img = R.render(tl, sc.materials, sc.camera, sc.light, primary_mat=pm).cpu().numpy().copy()
    plain = rg.Renderer(sc.width, sc.height, sc.max_depth).render(tl, sc.materials, sc.camera, sc.light)
    assert np.array_equal(img, plain.cpu().numpy())          # the extra output changes nothing else
    got = pm.cpu().numpy().view(np.uint32).reshape(-1)
    px = sg.sample_pixels(sc.width, sc.height, 4000, 17)
    o = oracle.Scene(sc).primary_materials(px)
    ok = o["amb"] == 0
    assert ok.mean() > 0.97
    bad = np.nonzero(ok & (got[px] != o["mat"]))[0]
    assert bad.size == 0, f"{bad.size} pixels, e.g. {px[bad[:5]]}: {got[px[bad[:5]]]} vs {o['mat'][bad[:5]]}"
    hit = o["mat"] != sg.MISS
    assert hit.sum() > 200 and (~hit).sum() > 200 and np.unique(o["mat"][hit]).size > 1
    # mode 1 (ambient occlusion) has no primary material output
    with pytest.raises(rg.RgError):
        rg.Renderer(sc.width, sc.height, 0, mode=1).render(tl, sc.materials, sc.camera, sc.light, primary_mat=pm)

