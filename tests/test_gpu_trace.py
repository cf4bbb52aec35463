"""GPU closest-hit / any-hit traversal (a8-a10) against the FP64 oracle, on the
same float32 rays, element by element, under the tolerance rules of
tests/parity.py.  Hierarchies are checked structurally before any traversal."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import scenegen as sg
from tests import bvh_check, parity
from tests.helpers import quad, ray, scene_from_meshes

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "triangle_hand_cases.json")


def _upload(scene, width=4, leaf=4, builder="lbvh"):
    import paper_2001_09792_amd as rg
    tl = rg.upload_scene(scene, width, leaf, builder=builder)
    for b in tl.blas:
        bvh_check.check_blas(b.buf.cpu().numpy(), b.desc)
    bvh_check.check_tlas(tl.buf.cpu().numpy(), tl.desc, [b.desc for b in tl.blas], scene.xform)
    return tl


def _trace(tl, rays_np, with_found=False):
    import paper_2001_09792_amd as rg
    r = rg.rays_to_device(rays_np)
    h = parity.hits_to_numpy(rg.trace_closest(tl, r))
    found = rg.alloc_hits(r.shape[1]) if with_found else None
    occ = rg.trace_any(tl, r, found=found).cpu().numpy()
    if with_found:
        return h, occ, parity.hits_to_numpy(found)
    return h, occ


def _both(scene, rays_np, label, max_amb=0.002, width=4, leaf=4, sphere=False, builder="lbvh"):
    print(f"[trace] {label}: {rays_np.shape[0]} rays W={width} L={leaf} {builder}", flush=True)
    tl = _upload(scene, width, leaf, builder)
    h, occ, found = _trace(tl, rays_np, with_found=True)
    orc = oracle.Scene(scene, sphere_reject=sphere)
    oc = orc.trace(rays_np)
    oa = orc.trace(rays_np, any_hit=True)
    sc = parity.check_closest(h, oc, max_amb, label, orc=orc, rays=rays_np)
    sa = parity.check_any(occ, oa, max_amb, label)
    sf = parity.check_found(found, occ, rays_np, orc, oa, label)
    # GPU-internal invariants: occluded == a closest hit exists; the closest
    # hit is no farther than the reported any hit (where float32 can order
    # the surfaces)
    assert np.array_equal(occ != 0, h["inst"].astype(np.uint32) != 0xFFFFFFFF)
    both = (occ != 0) & (oc["amb"] == 0) & (oa["amb"] == 0)
    assert (h["t"][both] <= found["t"][both] * (1 + 1e-6)).all()
    print(f"  closest {sc}\n  any {sa}\n  found {sf}", flush=True)
    return h, occ, oc


def test_hand_cases():
    g = json.load(open(GOLDEN))
    sc = scene_from_meshes([sg.triangles_mesh([g["triangle"]])])
    rays = np.stack([ray(c["o"], c["d"], 0.0, np.inf if c["tmax"] == "inf" else float(Fraction(c["tmax"])))
                     for c in g["cases"]])
    tl = _upload(sc)
    h, occ = _trace(tl, rays)
    for k, c in enumerate(g["cases"]):
        assert bool(occ[k]) == c["hit"], c["name"]
        if c["hit"]:
            assert h["t"][k] == pytest.approx(float(Fraction(c["t"])), rel=1e-6), c["name"]
            assert h["u"][k] == pytest.approx(float(Fraction(c["u"])), abs=1e-6), c["name"]
            assert h["v"][k] == pytest.approx(float(Fraction(c["v"])), abs=1e-6), c["name"]
        else:
            assert np.isinf(h["t"][k]) and np.uint32(h["inst"][k]) == 0xFFFFFFFF, c["name"]
    gp = g["ground"]
    sc = scene_from_meshes([sg.triangles_mesh([gp["P0"], gp["P1"]])])
    rays = np.stack([ray(c["o"], c["d"]) for c in gp["cases"]])
    h, _ = _trace(_upload(sc), rays)
    for k, c in enumerate(gp["cases"]):
        assert h["t"][k] == pytest.approx(float(Fraction(c["t"])), rel=1e-6)
        allowed = c.get("tie", [c["prim"]])
        assert h["prim"][k] in allowed


def _soup_rays(mesh, n, seed, extent=1.5):
    V = mesh.verts.astype(np.float64)
    cen = V[mesh.idx].mean(axis=1)
    rng = np.random.default_rng(seed)
    tgt = cen[rng.integers(0, cen.shape[0], n // 2)]
    rays = np.concatenate([sg.random_rays(n - n // 2, seed, extent), sg.rays_through_points(tgt, seed + 1, 2.5)])
    rays[::5, 7] = 0.9      # finite tmax
    rays[::11, 6] = 0.3     # nonzero tmin
    return rays


def test_soup_parity():
    mesh = sg.random_soup(5000, 41, extent=1.0, size=0.08)
    sc = scene_from_meshes([mesh])
    _both(sc, _soup_rays(mesh, 20000, 42), "soup")


@pytest.mark.parametrize("width,leaf", [(2, 1), (2, 4), (4, 1), (4, 8), (8, 2), (8, 4)])
def test_widths_and_leaf_sizes(width, leaf):
    mesh = sg.random_soup(3000, 51, extent=1.0, size=0.1)
    sc = scene_from_meshes([mesh])
    _both(sc, _soup_rays(mesh, 6000, 52), f"soup W{width} L{leaf}", width=width, leaf=leaf)


@pytest.mark.parametrize("width,leaf", [(2, 1), (4, 1), (4, 4), (8, 2)])
def test_clustered_hierarchy_parity(width, leaf):
    """Hierarchies from locally-ordered clustering trace to the same hits."""
    mesh = sg.random_soup(3000, 53, extent=1.0, size=0.1)
    sc = scene_from_meshes([mesh])
    _both(sc, _soup_rays(mesh, 6000, 54), f"soup ploc W{width} L{leaf}", width=width, leaf=leaf, builder="ploc")


def test_clustered_two_level_parity():
    import paper_2001_09792_amd as rg
    sc = sg.config_two_level(width=192, height=108)
    r = rg.camera_rays(sc.camera, 192, 108).cpu().numpy().T.copy()
    sel = sg.sample_pixels(192, 108, 3000, 17)
    rays = np.concatenate([r[sel], sg.random_rays(3000, 18, extent=22.0)])
    _both(sc, rays, "two-level ploc", sphere=True, builder="ploc")


@pytest.mark.parametrize("width,leaf", [(2, 1), (4, 4), (8, 2)])
def test_treelet_hierarchy_parity(width, leaf):
    """Hierarchies restructured by treelets trace to the same hits."""
    mesh = sg.random_soup(3000, 55, extent=1.0, size=0.1)
    sc = scene_from_meshes([mesh])
    _both(sc, _soup_rays(mesh, 6000, 56), f"soup treelet W{width} L{leaf}", width=width, leaf=leaf,
          builder="treelet")


def test_treelet_two_level_parity():
    import paper_2001_09792_amd as rg
    sc = sg.config_two_level(width=192, height=108)
    r = rg.camera_rays(sc.camera, 192, 108).cpu().numpy().T.copy()
    sel = sg.sample_pixels(192, 108, 3000, 19)
    rays = np.concatenate([r[sel], sg.random_rays(3000, 20, extent=22.0)])
    _both(sc, rays, "two-level treelet", sphere=True, builder="treelet")


def test_instanced_soup_parity():
    meshes = [sg.random_soup(2000, 61, 1.0, 0.1), sg.icosphere(3), sg.torus(40, 30, 1.0, 0.3)]
    rng = np.random.default_rng(62)
    xf = sg.random_instances(rng, 24, extent=3.0)
    sc = scene_from_meshes(meshes, xforms=xf, blas_id=np.arange(24) % 3)
    rays = sg.random_rays(20000, 63, extent=5.0)
    _both(sc, rays, "instanced")


def test_small_config_primary_rays():
    """Camera rays from the GPU's ray generation: directions within 1e-6 of the
    FP64 camera, then closest / any parity on those very rays."""
    import paper_2001_09792_amd as rg
    sc = sg.config_small()
    r = rg.camera_rays(sc.camera, sc.width, sc.height)
    rays = r.cpu().numpy().T.copy()
    ref = oracle.camera_rays(sc.camera, sc.width, sc.height, np.arange(sc.width * sc.height))
    assert np.abs(rays[:, 0:3] - ref[:, 0:3]).max() == 0.0
    assert np.abs(rays[:, 3:6] - ref[:, 3:6]).max() < 1e-6
    assert (rays[:, 6] == 0).all() and np.isinf(rays[:, 7]).all()
    h, _, oc = _both(sc, rays, "small primary", max_amb=0.01)
    assert (oc["hit"] == 1).mean() > 0.3


def test_two_level_primary_and_random_rays():
    import paper_2001_09792_amd as rg
    sc = sg.config_two_level(width=192, height=108)
    r = rg.camera_rays(sc.camera, 192, 108).cpu().numpy().T.copy()
    sel = sg.sample_pixels(192, 108, 3000, 7)
    rays = np.concatenate([r[sel], sg.random_rays(3000, 8, extent=22.0)])
    rays[3000::4, 7] = 6.0
    _both(sc, rays, "two-level", sphere=True)


def test_rigid_motion_on_gpu():
    """Exact motions of instance + ray leave the GPU result unchanged."""
    meshes = [sg.random_soup(500, 71, 1.0, 0.15), sg.icosphere(2)]
    X = np.zeros((4, 3, 4), np.float32)
    for i in range(4):
        X[i, :, :3] = np.eye(3) * [1, 2, 0.5, 1][i]
        X[i, :, 3] = [i - 2, 1 - i, i % 2]
    sc = scene_from_meshes(meshes, xforms=X, blas_id=[0, 1, 0, 1])
    rays = sg.random_rays(4000, 72, extent=3.0)
    rays[:, :6] = np.round(rays[:, :6] * 4096.0) / 4096.0
    G = np.array([[0, 0, 2], [-2, 0, 0], [0, 2, 0]], np.float64)
    gt = np.array([3.0, -1.0, 4.0])
    X2 = np.empty_like(X)
    X2[:, :, :3] = np.einsum("ij,njk->nik", G, X[:, :, :3])
    X2[:, :, 3] = X[:, :, 3] @ G.T + gt
    sc2 = scene_from_meshes(meshes, xforms=X2.astype(np.float32), blas_id=[0, 1, 0, 1])
    r2 = rays.copy()
    r2[:, 0:3] = rays[:, 0:3] @ G.T + gt
    r2[:, 3:6] = rays[:, 3:6] @ G.T
    h1, _ = _trace(_upload(sc), rays)
    h2, _ = _trace(_upload(sc2), r2.astype(np.float32))
    hit = h1["inst"] != -1
    assert hit.sum() > 300
    assert np.array_equal(h1["inst"], h2["inst"]) and np.array_equal(h1["prim"], h2["prim"])
    assert np.allclose(h1["t"][hit], h2["t"][hit], rtol=1e-6)


def test_degenerate_rays_and_empty_batch():
    import torch
    import paper_2001_09792_amd as rg
    sc = scene_from_meshes([sg.random_soup(100, 81)])
    tl = _upload(sc)
    rays = np.stack([ray((0, 0, 5), (0, 0, -1), 2.0, 1.0),      # empty interval
                     ray((0, 0, 5), (0, 0, 0)),                 # zero direction
                     ray((0, 0, 5), (0, 0, -1), 0.0, 0.0)])     # zero-length
    h, occ = _trace(tl, rays)
    assert np.uint32(h["inst"][0]) == 0xFFFFFFFF and occ[0] == 0
    assert np.uint32(h["inst"][1]) == 0xFFFFFFFF and occ[1] == 0
    empty = torch.empty((8, 0), dtype=torch.float32, device="cuda")
    rg.trace_closest(tl, empty)
    rg.trace_any(tl, empty)
    torch.cuda.synchronize()


def test_visit_counts():
    import paper_2001_09792_amd as rg
    mesh = sg.random_soup(3000, 91, 1.0, 0.1)
    sc = scene_from_meshes([mesh])
    tl = _upload(sc)
    rays = _soup_rays(mesh, 4000, 92)
    r = rg.rays_to_device(rays)
    cc = rg.trace_counts(tl, r).cpu().numpy()
    ca = rg.trace_counts(tl, r, any_hit=True).cpu().numpy()
    h = rg.trace_closest(tl, r)["inst"].cpu().numpy()
    hit = h != -1
    assert (cc[:, 2] <= 1).all() and (cc[hit, 2] == 1).all()
    assert (cc[hit, 1] >= 1).all() and (cc[:, 0] >= 1).all()
    # any-hit stops early: never more work than closest on hit rays on average
    assert ca[hit, 1].mean() <= cc[hit, 1].mean() * 1.5 + 1


def test_ao_directions_within_1e6_on_exact_normals():
    """AO directions from the same u1, u2 agree with the FP64 oracle to 1e-6.
    On a plane at integer coordinates seen through the identity instance the
    float32 normal, and so the tangent frame, is exact: what remains is the
    float32 rounding of the cosine-weighted hemisphere sample itself (the
    general test above also carries the normal's float32 error)."""
    import paper_2001_09792_amd as rg
    W, H = 64, 48
    plane = sg.triangles_mesh(quad(0.0, half=50.0))
    sc = scene_from_meshes([plane], width=W, height=H, mode=1, seed=7)
    tl = _upload(sc)
    cam = rg.camera_rays(sc.camera, W, H)
    hits = rg.trace_closest(tl, cam)
    assert (hits["inst"].cpu().numpy() != -1).all(), "every camera ray sees the plane"
    out, src, count = rg.ao_rays(tl, cam, hits, seed=sc.seed, tmax=5.0)
    n_ao = int(count.item())
    assert n_ao == 8 * W * H
    src = src[:n_ao].cpu().numpy()
    rays_ao = out[:, :n_ao].cpu().numpy().T
    ref = oracle.Scene(sc).ao_rays(cam.cpu().numpy().T.copy(), sc.seed)
    assert (ref["hit"] == 1).all()
    # camera rays through the quad's shared diagonal (pixels i + j = 55 of
    # this image, 1.6%) are flagged ambiguous; the rest are compared
    ok = ref["amb"][src // 8] == 0
    assert ok.mean() > 0.97
    r = ref["rays"][src[ok] // 8, src[ok] % 8]
    d_err = np.abs(rays_ao[ok, 3:6] - r[:, 3:6]).max()
    print(f"[ao] exact-normal directions: max error {d_err:.2e} over {int(ok.sum())} rays", flush=True)
    assert d_err < 1e-6
    assert (rays_ao[:, 5] > 0.0).all(), "directions in the upper hemisphere"
    assert np.abs(rays_ao[ok, 0:3] - r[:, 0:3]).max() < 2e-4


def test_ao_rays_match_oracle():
    import torch
    import paper_2001_09792_amd as rg
    sc = sg.config_incoherent(segments=24, width=96, height=54)
    tl = _upload(sc)
    cam = rg.camera_rays(sc.camera, 96, 54)
    hits = rg.trace_closest(tl, cam)
    out, src, count = rg.ao_rays(tl, cam, hits, seed=sc.seed, tmax=5.0)
    n_ao = int(count.item())
    prim_hit = hits["inst"].cpu().numpy() != -1
    assert n_ao == 8 * int(prim_hit.sum())
    src = src[:n_ao].cpu().numpy()
    expect_src = (np.nonzero(prim_hit)[0][:, None] * 8 + np.arange(8)[None, :]).ravel()
    assert np.array_equal(src, expect_src), "compaction keeps input order"

    rays_ao = out[:, :n_ao].cpu().numpy().T
    orc = oracle.Scene(sc, sphere_reject=True)
    ref = orc.ao_rays(cam.cpu().numpy().T.copy(), sc.seed)
    pix = src // 8
    k = src % 8
    assert np.array_equal(np.unique(pix), np.nonzero(prim_hit)[0])
    ok = ref["amb"][pix] == 0
    assert ok.mean() > 0.97
    r = ref["rays"][pix[ok], k[ok]]
    assert np.abs(rays_ao[ok, 3:6] - r[:, 3:6]).max() < 2e-5
    assert np.abs(rays_ao[ok, 0:3] - r[:, 0:3]).max() < 2e-4
    assert (rays_ao[:, 7] == 5.0).all() and (rays_ao[:, 6] == 0.0).all()
    # and the AO rays themselves trace to oracle parity
    sel = np.arange(0, n_ao, max(1, n_ao // 4000))
    h = parity.hits_to_numpy(rg.trace_closest(tl, rg.rays_to_device(rays_ao[sel])))
    oc = orc.trace(rays_ao[sel])
    print(parity.check_closest(h, oc, 0.002, "ao"), flush=True)
    torch.cuda.synchronize()


def test_launch_parameters_do_not_change_results():
    """Refill threshold, resident waves, LDS stack depth and the leaf /
    instance batching only reorder work: every hit is bitwise the same."""
    import paper_2001_09792_amd as rg
    sc = sg.config_two_level(width=192, height=108)
    tl = rg.upload_scene(sc, 4, 2)
    cam = rg.camera_rays(sc.camera, 192, 108).cpu().numpy().T.copy()
    rays = rg.rays_to_device(np.concatenate([cam, sg.random_rays(20000, 9, extent=22.0)]))
    saved = rg.trace_tuning()
    ref = None
    try:
        for cfg in (dict(refill=8, waves_per_cu=16, lds_depth=16, leaf_batch=1, inst_batch=1),
                    dict(refill=1, waves_per_cu=4, lds_depth=8, leaf_batch=64, inst_batch=64),
                    dict(refill=64, waves_per_cu=24, lds_depth=32, leaf_batch=16, inst_batch=8),
                    dict(refill=16, waves_per_cu=16, lds_depth=16, leaf_batch=32, inst_batch=1)):
            print(f"[trace] launch {cfg}", flush=True)
            rg.trace_tuning(**cfg)
            h = parity.hits_to_numpy(rg.trace_closest(tl, rays))
            occ = rg.trace_any(tl, rays).cpu().numpy()
            if ref is None:
                ref = (h, occ)
                continue
            for k in h:
                assert np.array_equal(h[k].view(np.uint32), ref[0][k].view(np.uint32)), (cfg, k)
            assert np.array_equal(occ, ref[1]), cfg
    finally:
        rg.trace_tuning(**saved)
