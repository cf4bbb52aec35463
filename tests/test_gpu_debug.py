"""RG_DEBUG=1: the asynchronous entry points wait for their stream and check
for errors before returning; results do not change.  Run in a child process
(the variable is read once per process)."""
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CHILD = r"""
import sys, numpy as np, torch
sys.path.insert(0, {root!r})
import paper_2001_09792_amd as rg
import scenegen as sg
sc = sg.config_two_level(width=96, height=54, max_depth=2)
tl = rg.upload_scene(sc, 4, 1, builder="treelet")
rays = rg.rays_to_device(sg.random_rays(5000, 3, extent=20.0))
h = rg.trace_closest(tl, rays)
occ = rg.trace_any(tl, rays, cull=rg.RAY_CULL_BACK)
pm = torch.empty((sc.height, sc.width), dtype=torch.int32, device="cuda")
img = rg.Renderer(sc.width, sc.height, sc.max_depth).render(tl, sc.materials, sc.camera, sc.light, primary_mat=pm)
P = rg.Post(sc.width, sc.height)
out = P.fxaa(P.roughness_blur(img, pm, torch.full((len(sc.materials),), 0.5, device="cuda"), 4))
parts = [h["t"], h["inst"], h["prim"], occ, img, out]
np.save(sys.argv[1], np.concatenate([p.cpu().numpy().ravel().view(np.uint8) for p in parts]))
print("child ok", flush=True)
"""


def test_debug_mode_gives_the_same_results(tmp_path):
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    script = CHILD.format(root=root)
    outs = {}
    for dbg in ("0", "1"):
        env = dict(os.environ, RG_DEBUG=dbg)
        path = str(tmp_path / f"out{dbg}.npy")
        print(f"[debug] RG_DEBUG={dbg}", flush=True)
        r = subprocess.run([sys.executable, "-c", script, path], env=env, capture_output=True, text=True, timeout=240)
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
        outs[dbg] = np.load(path)
    assert np.array_equal(outs["0"], outs["1"])
