"""Dynamic scenes on the GPU (moving geometry, the per-frame update before the
path): a bottom level refitted to new vertex positions keeps its hierarchy
and holds the new triangles; refitting to unchanged vertices reproduces the
build bit for bit; a refitted scene with a rebuilt top level traces to the
very hits of a scene built from scratch at the new positions, and to the FP64
oracle's."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from tests import bvh_check, parity
from tests.helpers import scene_from_meshes

pytestmark = pytest.mark.gpu


def _dev(verts, idx):
    import torch
    v = torch.from_numpy(np.ascontiguousarray(verts, np.float32)).cuda()
    i = torch.from_numpy(np.ascontiguousarray(idx, np.uint32).view(np.int32)).cuda()
    return v, i


@pytest.mark.parametrize("builder", ["lbvh", "ploc", "treelet"])
@pytest.mark.parametrize("width,leaf", [(2, 1), (4, 1), (4, 4), (8, 3)])
def test_refit_to_unchanged_vertices_reproduces_the_build(builder, width, leaf):
    import paper_2001_09792_amd as rg
    mesh = sg.torus(48, 40, 1.0, 0.35, 0.08, 6.0, 3001)
    print(f"[refit same] {builder} W{width} L{leaf}", flush=True)
    v, i = _dev(mesh.verts, mesh.idx)
    b = rg.build_blas(v, i, None, width, leaf, builder=builder)
    before = b.buf.cpu().numpy().copy()
    lo, hi = list(b.desc.lo), list(b.desc.hi)
    assert rg.blas_state(b) == (lo, hi, 0)
    rg.refit_blas(b, v, i)
    after = b.buf.cpu().numpy()
    assert np.array_equal(before, after)      # header (root box, status) included
    assert rg.blas_state(b) == (lo, hi, 0)


@pytest.mark.parametrize("width,leaf,builder", [(2, 1, "lbvh"), (4, 1, "lbvh"), (8, 4, "lbvh"), (4, 1, "treelet")])
def test_refit_to_moved_vertices_holds_the_new_mesh(width, leaf, builder):
    """Structure and boxes checked on the host; the triangles in leaf order
    are the moved ones; hits against the oracle on the moved mesh."""
    import paper_2001_09792_amd as rg
    mesh = sg.torus(64, 48, 1.0, 0.35, 0.08, 6.0, 3002)
    moved = sg.Mesh(sg.animate_mesh(mesh, 0.35, amp=0.08, seed=5), mesh.idx)
    print(f"[refit moved] W{width} L{leaf} {builder}", flush=True)
    v0, i = _dev(mesh.verts, mesh.idx)
    b = rg.build_blas(v0, i, None, width, leaf, builder=builder)
    v1, _ = _dev(moved.verts, moved.idx)
    rg.refit_blas(b, v1, i)
    info = bvh_check.check_blas(b.buf.cpu().numpy(), b.desc, refitted=True)
    assert np.array_equal(info["verts"], moved.verts[moved.idx[info["prim"]]])
    lo, hi, status = rg.blas_state(b)
    assert status == 0
    assert np.array_equal(np.float32(lo), moved.verts.min(axis=0)) and np.array_equal(np.float32(hi),
                                                                                     moved.verts.max(axis=0))
    # trace through a top level built over the refitted bottom level
    tl = rg.build_tlas([b], sg.identity_xform(1), [0], [0], width)
    rng = np.random.default_rng(7)
    cen = moved.verts[moved.idx].mean(axis=1)
    rays = np.concatenate([sg.random_rays(3000, 8, extent=1.8),
                           sg.rays_through_points(cen[rng.integers(0, cen.shape[0], 3000)], 9, 3.0)])
    h = parity.hits_to_numpy(rg.trace_closest(tl, rg.rays_to_device(rays)))
    oc = oracle.Scene(scene_from_meshes([moved])).trace(rays)
    print(parity.check_closest(h, oc, 0.002, "refit moved"), flush=True)


def _moved_two_level(t):
    sc = sg.config_two_level(width=160, height=90, max_depth=3)
    meshes = [sg.Mesh(sg.animate_mesh(m, t, amp=0.04, seed=k), m.idx, m.prim_mat) for k, m in enumerate(sc.blas)]
    xf = sg.animate_instances(sc.xform, t, seed=11)
    return sc, meshes, xf


@pytest.mark.parametrize("builder", ["lbvh", "treelet"])
def test_refitted_scene_traces_like_a_fresh_build(builder):
    """Hits do not depend on the hierarchy (ties go to the lowest instance and
    input triangle, the instance slide point depends only on the root box,
    which a refit computes exactly): the refitted scene gives bitwise the hits
    of a scene built from scratch at the new positions."""
    import paper_2001_09792_amd as rg
    sc, moved, xf = _moved_two_level(0.3)
    print(f"[dynamic] two-level, refit + top-level rebuild ({builder})", flush=True)
    tl0 = rg.upload_scene(sc, 4, 1, builder=builder)
    for b, m in zip(tl0.blas, moved):
        v, i = _dev(m.verts, m.idx)
        rg.refit_blas(b, v, i)
    tl_refit = rg.build_tlas(tl0.blas, xf, sc.blas_id, sc.inst_mat, 4, builder=builder)
    fresh_scene = sg.Scene(sc.name, moved, xf, sc.blas_id, sc.inst_mat, sc.materials, sc.camera, sc.light,
                           sc.width, sc.height, sc.max_depth, sc.mode, sc.seed)
    tl_fresh = rg.upload_scene(fresh_scene, 4, 1, builder=builder)
    for b in tl_refit.blas:
        bvh_check.check_blas(b.buf.cpu().numpy(), b.desc, refitted=True)
    roots = [rg.blas_state(b)[:2] for b in tl_refit.blas]
    bvh_check.check_tlas(tl_refit.buf.cpu().numpy(), tl_refit.desc, [b.desc for b in tl_refit.blas], xf, roots)
    cam = rg.camera_rays(sc.camera, sc.width, sc.height).cpu().numpy().T.copy()
    rays = rg.rays_to_device(np.concatenate([cam, sg.random_rays(8000, 12, extent=22.0)]))
    h1 = parity.hits_to_numpy(rg.trace_closest(tl_refit, rays))
    h2 = parity.hits_to_numpy(rg.trace_closest(tl_fresh, rays))
    for k in h1:
        assert np.array_equal(h1[k].view(np.uint32), h2[k].view(np.uint32)), k
    assert np.array_equal(rg.trace_any(tl_refit, rays).cpu().numpy(), rg.trace_any(tl_fresh, rays).cpu().numpy())
    # the rendered frame against the oracle on the moved scene (sampled pixels)
    img = rg.render(tl_refit, sc.materials, sc.camera, sc.light, sc.width, sc.height, sc.max_depth)
    px = sg.sample_pixels(sc.width, sc.height, 800, 13)
    ref = oracle.Scene(fresh_scene, sphere_reject=True).render(px, width=sc.width, height=sc.height,
                                                               max_depth=sc.max_depth)
    print(parity.check_image(img.cpu().numpy().reshape(-1, 3)[px], ref, 0.015, "refit render"), flush=True)


@pytest.mark.parametrize("n_inst", [64, 1024, 1500])
def test_tlas_builder_matches_build_tlas(n_inst):
    """TlasBuilder rebuilds one buffer frame after frame: each build is byte
    for byte the top level rg_build_tlas writes for the same matrices (up to
    1,024 instances the instance step runs inside the one-workgroup build,
    above that in its own launches), also after a build with other matrices
    and with a bottom level's invalid refit reported."""
    import torch
    import paper_2001_09792_amd as rg
    sc = sg.config_two_level(width=64, height=48)
    tl = rg.upload_scene(sc, 4, 1, builder="lbvh")
    rng = np.random.default_rng(n_inst)
    nb = len(tl.blas)
    blas_id = rng.integers(0, nb, n_inst).astype(np.uint32)
    mat = rng.integers(0, len(sc.materials), n_inst).astype(np.uint32)
    frames = [sg.animate_instances(np.tile(sc.xform, (n_inst // len(sc.xform) + 1, 1, 1))[:n_inst], t, seed=9)
              for t in (0.1, 0.7, 0.1)]
    top = rg.TlasBuilder(tl.blas, blas_id, mat, 4)
    for k, xf in enumerate(frames):
        got = top.build(xf)
        ref = rg.build_tlas(tl.blas, xf, blas_id, mat, 4)
        torch.cuda.synchronize()
        assert got.desc.n_nodes == ref.desc.n_nodes and got.desc.depth == ref.desc.depth
        a, b = got.buf.cpu().numpy(), ref.buf.cpu().numpy()
        n = int(ref.buf.numel())
        assert a.shape == b.shape
        # nodes, records, record map and matrices: the same bytes (the node
        # order within a level follows the build's atomics, so compare sets)
        d = ref.desc
        recs = slice(d.inst_off, d.inst_off + 112 * n_inst)
        assert np.array_equal(a[recs], b[recs]), f"frame {k}: instance records differ"
        rmap = slice(d.rec_off, d.rec_off + 4 * n_inst)
        assert np.array_equal(a[rmap], b[rmap]), f"frame {k}: record map differs"
        xfs = slice(d.xf_off, d.xf_off + 48 * n_inst)
        assert np.array_equal(a[xfs], b[xfs]), f"frame {k}: matrices differ"
        bvh_check.check_tlas(a, got.desc, [x.desc for x in tl.blas], xf)
        rays = rg.rays_to_device(sg.random_rays(4000, 31 + k, extent=22.0))
        h1 = parity.hits_to_numpy(rg.trace_closest(got, rays))
        h2 = parity.hits_to_numpy(rg.trace_closest(ref, rays))
        for key in h1:
            assert np.array_equal(h1[key].view(np.uint32), h2[key].view(np.uint32)), (k, key)
    # a bottom level refitted to invalid input: both report it
    v, i = _dev(sc.blas[0].verts, sc.blas[0].idx)
    bad = v.clone()
    bad[0, 0] = float("nan")
    rg.refit_blas(tl.blas[0], bad, i)
    with pytest.raises(rg.RgError):
        top.build(frames[0])
    rg.refit_blas(tl.blas[0], v, i)
    top.build(frames[0])
    torch.cuda.synchronize()


@pytest.mark.parametrize("width", [2, 4, 8])
def test_refit_many_equals_one_by_one(width):
    """Bottom levels of different sizes and depths refitted in one call: every
    buffer (nodes, triangles, header) equals a refit of that level alone."""
    import paper_2001_09792_amd as rg
    meshes = [sg.torus(64, 48, 1.0, 0.35, 0.08, 6.0, 3003), sg.icosphere(2), sg.random_soup(5000, 4),
              sg.triangles_mesh([[(0, 0, 0), (1, 0, 0), (0, 1, 0)]])]
    print(f"[refit many] W{width}", flush=True)
    dev = [_dev(m.verts, m.idx) for m in meshes]
    moved = [_dev(sg.animate_mesh(m, 0.2, amp=0.05, seed=k), m.idx)[0] for k, m in enumerate(meshes)]
    one = [rg.build_blas(v, i, None, width, 2) for v, i in dev]
    # byte copies of the same builds (two builds of one mesh number their nodes
    # in whatever order the collapse's threads claim them)
    many = []
    for b in one:
        buf = b.buf.clone()
        d = rg.BlasDesc.from_buffer_copy(b.desc)
        d.buf = buf.data_ptr()
        many.append(rg.Blas(buf, d))
    for b, v, (_, i) in zip(one, moved, dev):
        rg.refit_blas(b, v, i)
    rg.refit_blas_many(many, moved, [i for _, i in dev])
    def content(b):
        # the arrays and the header's root box and status; not the header's
        # device addresses, nor the alignment padding between arrays
        buf, d = b.buf.cpu().numpy(), b.desc
        return (buf[32:64], buf[d.nodes_off: d.nodes_off + d.n_nodes * 32 * d.width],
                buf[d.tris_off: d.tris_off + 40 * d.n_tris])
    for m, (a, b) in enumerate(zip(one, many)):
        bvh_check.check_blas(a.buf.cpu().numpy(), a.desc, refitted=True)
        bvh_check.check_blas(b.buf.cpu().numpy(), b.desc, refitted=True)
        for part, x, y in zip(("header", "nodes", "triangles"), content(a), content(b)):
            bad = np.nonzero(x != y)[0]
            if bad.size:
                print(f"mesh {m} ({a.desc.n_tris} tris, depth {a.desc.depth}): {part} differs at {bad.size} "
                      f"bytes, first {bad[:8]}", flush=True)
            assert bad.size == 0


def test_refit_errors():
    import torch
    import paper_2001_09792_amd as rg
    mesh = sg.random_soup(200, 3)
    v, i = _dev(mesh.verts, mesh.idx)
    b = rg.build_blas(v, i)
    with pytest.raises(rg.RgError):
        rg.refit_blas(b, v, i[:100])          # other triangle count
    bad = v.clone()
    bad[7, 0] = float("inf")
    rg.refit_blas(b, bad, i)                  # found on the device: recorded, reported by the top level
    assert rg.blas_state(b)[2] != 0
    with pytest.raises(rg.RgError):
        rg.build_tlas([b], sg.identity_xform(1), [0], [0])
    bad_i = i.clone()
    bad_i[5, 1] = 10 ** 6
    rg.refit_blas(b, v, bad_i)                # an index out of range: never read, recorded
    assert rg.blas_state(b)[2] != 0
    # a valid refit afterwards restores the structure and clears the status
    rg.refit_blas(b, v, i)
    assert rg.blas_state(b)[2] == 0
    bvh_check.check_blas(b.buf.cpu().numpy(), b.desc)
    rg.build_tlas([b], sg.identity_xform(1), [0], [0])
    torch.cuda.synchronize()


@pytest.mark.parametrize("n_inst", [64, 1500, 6000])
def test_async_tlas_equals_sync(n_inst):
    """rg_build_tlas_async + rg_build_tlas_finish give rg_build_tlas's top
    level (node count, depth, box, records, record map, matrices, hits) for
    the fused one-workgroup build, the unfused one and the multi-launch one;
    an invalid refit of a bottom level is reported by finish; a finished
    ticket is rejected."""
    import torch
    import paper_2001_09792_amd as rg
    sc = sg.config_two_level(width=64, height=48)
    tl = rg.upload_scene(sc, 4, 1, builder="lbvh")
    rng = np.random.default_rng(n_inst + 5)
    blas_id = rng.integers(0, len(tl.blas), n_inst).astype(np.uint32)
    mat = rng.integers(0, len(sc.materials), n_inst).astype(np.uint32)
    xf = sg.animate_instances(np.tile(sc.xform, (n_inst // len(sc.xform) + 1, 1, 1))[:n_inst], 0.3, seed=11)
    print(f"[async tlas] {n_inst}", flush=True)
    ref = rg.build_tlas(tl.blas, xf, blas_id, mat, 4)
    s = torch.cuda.Stream()
    p = rg.build_tlas_async(tl.blas, xf, blas_id, mat, 4, stream=s)
    got = p.finish()
    torch.cuda.synchronize()
    for f in ("n_inst", "n_nodes", "width", "depth", "max_blas_depth", "has_inst_flags"):
        assert getattr(got.desc, f) == getattr(ref.desc, f), f
    assert list(got.desc.lo) == list(ref.desc.lo) and list(got.desc.hi) == list(ref.desc.hi)
    a, b, d = got.buf.cpu().numpy(), ref.buf.cpu().numpy(), ref.desc
    for off, size in ((d.inst_off, 112 * n_inst), (d.rec_off, 4 * n_inst), (d.xf_off, 48 * n_inst)):
        assert np.array_equal(a[off: off + size], b[off: off + size])
    bvh_check.check_tlas(a, got.desc, [x.desc for x in tl.blas], xf)
    rays = rg.rays_to_device(sg.random_rays(4000, 41, extent=22.0))
    h1 = parity.hits_to_numpy(rg.trace_closest(got, rays))
    h2 = parity.hits_to_numpy(rg.trace_closest(ref, rays))
    for key in h1:
        assert np.array_equal(h1[key].view(np.uint32), h2[key].view(np.uint32)), key
    with pytest.raises(rg.RgError):
        p.finish()
    v, i = _dev(sc.blas[0].verts, sc.blas[0].idx)
    bad = v.clone()
    bad[0, 0] = float("nan")
    rg.refit_blas(tl.blas[0], bad, i)
    with pytest.raises(rg.RgError) as e:
        rg.build_tlas_async(tl.blas, xf, blas_id, mat, 4).finish()
    assert e.value.status == -1
    rg.refit_blas(tl.blas[0], v, i)
    rg.build_tlas_async(tl.blas, xf, blas_id, mat, 4).finish()
    torch.cuda.synchronize()


@pytest.mark.parametrize("n_inst", [300, 3000])
def test_tlas_built_behind_queued_work_equals_idle_build(n_inst):
    """The synchronous top-level build uploads its host tables on a stream of
    its own while the caller's stream still has work queued (here a trace of
    4M rays), then makes that stream wait for the copy: the result is the
    top level built on an idle stream (records, record map, matrices, hits)."""
    import torch
    import paper_2001_09792_amd as rg
    sc = sg.config_two_level(width=64, height=48)
    tl = rg.upload_scene(sc, 4, 1, builder="lbvh")
    rng = np.random.default_rng(n_inst + 9)
    blas_id = rng.integers(0, len(tl.blas), n_inst).astype(np.uint32)
    mat = rng.integers(0, len(sc.materials), n_inst).astype(np.uint32)
    xf = sg.animate_instances(np.tile(sc.xform, (n_inst // len(sc.xform) + 1, 1, 1))[:n_inst], 0.3, seed=13)
    print(f"[tlas behind work] {n_inst}", flush=True)
    torch.cuda.synchronize()
    ref = rg.build_tlas(tl.blas, xf, blas_id, mat, 4)
    ref_buf = ref.buf.clone()
    torch.cuda.synchronize()
    rays = rg.rays_to_device(sg.random_rays(4_000_000, 43, extent=22.0))
    torch.cuda.synchronize()
    rg.trace_closest(tl, rays)  # queued: the stream is busy when the build is called
    got = rg.build_tlas(tl.blas, xf, blas_id, mat, 4)
    torch.cuda.synchronize()
    for f in ("n_inst", "n_nodes", "width", "depth", "max_blas_depth", "has_inst_flags"):
        assert getattr(got.desc, f) == getattr(ref.desc, f), f
    assert list(got.desc.lo) == list(ref.desc.lo) and list(got.desc.hi) == list(ref.desc.hi)
    a, b, d = got.buf.cpu().numpy(), ref_buf.cpu().numpy(), ref.desc
    for off, size in ((d.inst_off, 112 * n_inst), (d.rec_off, 4 * n_inst), (d.xf_off, 48 * n_inst)):
        assert np.array_equal(a[off: off + size], b[off: off + size])
    bvh_check.check_tlas(a, got.desc, [x.desc for x in tl.blas], xf)
    sample = rg.rays_to_device(sg.random_rays(4000, 47, extent=22.0))
    h1 = parity.hits_to_numpy(rg.trace_closest(got, sample))
    ref2 = rg.build_tlas(tl.blas, xf, blas_id, mat, 4)
    h2 = parity.hits_to_numpy(rg.trace_closest(ref2, sample))
    for key in h1:
        assert np.array_equal(h1[key].view(np.uint32), h2[key].view(np.uint32)), key
