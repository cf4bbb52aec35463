"""Trace parity inside a render (paper section 1: the closest-hit, any-hit
and miss outcome of every ray a dispatch spawns, recursively; section 2.1:
reflection, refraction and shadow rays).

rg_render_capture keeps each pass's queues: the closest-hit rays exactly as
the GPU traced them (secondary rays as its shading spawned them, in float32)
with their hits, and the shadow rays with their any-hit results.  The oracle
traces those very rays, so a traversal error in a later bounce shows as a
wrong hit instead of disappearing into the drift of secondary rays that the
image comparison has to tolerate.  The render keeps float32 t internally, so
t is held to max(1e-5 t*, delta) here (tests/parity.py, t_band)."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from tests import parity

pytestmark = pytest.mark.gpu


def _check_passes(sc, W, H, D, label, width=4, leaf=1, builder="treelet", sample=4000, max_amb=0.01, seed=5):
    import torch
    import paper_2001_09792_amd as rg
    print(f"[passes] {label}: {W}x{H} depth {D} W={width} L={leaf} {builder}", flush=True)
    tl = rg.upload_scene(sc, width=width, leaf_max=leaf, builder=builder)
    cap = W * H * (1 << D)
    img, passes = rg.render_capture(tl, sc.materials, sc.camera, sc.light, W, H, D, cap, seed=sc.seed)
    # the capture renders the same image as rg_render
    ref = rg.Renderer(W, H, D).render(tl, sc.materials, sc.camera, sc.light, sc.seed)
    torch.cuda.synchronize()
    assert torch.equal(img, ref)
    orc = oracle.Scene(sc, sphere_reject=True)
    rng = np.random.default_rng(seed)
    report = []
    n_checked = 0
    for k, p in enumerate(passes):
        nc, ns = p["counts"]
        assert p["rays"].shape[0] == nc and p["shadow"].shape[0] == ns  # capacity covers the worst case
        if k == 0:
            assert nc == W * H
        if nc:
            sel = np.sort(rng.choice(nc, min(nc, sample), replace=False))
            rays = p["rays"][sel]
            g = {"t": p["t"][sel], "inst": p["inst"][sel], "prim": p["prim"][sel]}
            rc = parity.check_closest(g, orc.trace(rays), max_amb, f"{label} pass {k} closest", t_band=True)
            n_checked += rc["n"]
            report.append((k, "closest", nc, rc["n"], rc["amb_frac"], rc["hits"]))
        if ns:
            sel = np.sort(rng.choice(ns, min(ns, sample), replace=False))
            ra = parity.check_any(p["occluded"][sel], orc.trace(p["shadow"][sel], any_hit=True), max_amb,
                                  f"{label} pass {k} shadow")
            n_checked += ra["n"]
            report.append((k, "shadow", ns, ra["n"], ra["amb_frac"], ra["occluded"]))
    for r in report:
        print(f"  pass {r[0]} {r[1]:7s}: {r[2]} queued, {r[3]} checked, ambiguous {r[4]:.4f}, hits {r[5]}", flush=True)
    return passes, n_checked


def test_small_frame_passes():
    sc = sg.config_small()
    passes, n = _check_passes(sc, 128, 128, sc.max_depth, "small", width=4, leaf=4, builder="lbvh", sample=40000)
    assert len(passes) == 2 and passes[1]["counts"][0] > 0   # mirror children were traced
    assert n == sum(p["counts"][0] + p["counts"][1] for p in passes)   # every ray of the frame checked


@pytest.mark.parametrize("width,builder", [(4, "treelet"), (8, "ploc")])
def test_two_level_frame_passes(width, builder):
    """The two-level scene at depth 4: reflection and refraction rays of
    every depth, both hierarchy shapes of the benchmark's frames."""
    sc = sg.config_two_level(width=320, height=180)
    passes, n = _check_passes(sc, 320, 180, 4, f"two-level {builder}", width=width, builder=builder, sample=6000)
    assert all(p["counts"][0] > 0 for p in passes)       # every depth has rays
    assert sum(p["counts"][1] for p in passes) > 0        # and shadow rays


def test_two_level_full_size_passes():
    """The benchmark's two-level frame (1920x1080, depth 4) at its own
    hierarchy shape: 3,000 sampled rays of each queue of each pass."""
    sc = sg.config_two_level()
    passes, n = _check_passes(sc, 1920, 1080, 4, "two-level 1080p", width=8, builder="treelet", sample=3000,
                              max_amb=0.01)
    assert all(p["counts"][0] > 0 for p in passes)
