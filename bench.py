"""Benchmark: closest-hit Mrays/s on primary + incoherent rays, one MI355X.

Workload (default, `--workload incoherent`): 1,024 instances of 16 seeded
displaced tori of 560x560 segments (627,200 triangles each, 10,035,200
unique, 642M instanced), camera 1920x1080; per step: ray generation, a
closest-hit pass over the 2,073,600 camera rays, ambient-occlusion ray
generation (8 cosine-weighted rays per primary hit, tmax 5) and a
closest-hit pass over those rays.  value = (primary + AO rays) / step time.
The hierarchies are built once, before timing, and stay resident in HBM.

`--workload two_level` times whole frames of the 64-instance scene instead
(1920x1080, Whitted recursion depth 4: camera, closest, shade, shadow any-
hit, reflection and refraction passes), value = all rays traced / frame time.

One JSON line is printed.  `roofline` refers to the dominant kernel (the
closest-hit traversal of the AO rays): algorithmic bytes per ray from the
traversal's own visit counts (ray 32 B + hit 20 B + nodes x 28W B rounded up
to 64 / 128 / 256 B + triangles x 40 B + instance entries x 56 B: the 3x4
inverse and the bottom level's root / id) over the kernel's event-timed
duration, against 8 TB/s and against the copy bandwidth measured on the same
GPU; beside it the surface-area cost of the hierarchies it walks.
`cpu_baseline` is the FP64 oracle timed on a bounded sample of the same rays
on this host's cores.  The default run also measures, on the same GPU, the
batched form (256 scenes: one batch against one rg_render per frame) and the
served form (64 resident scenes: saturated engine against plain dispatch,
p50 / p99 latency at 0.9 of plain dispatch's saturated rate).
"""
import argparse
import math
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
NODE_BYTES = {2: 64, 4: 128, 8: 256}  # 28 W rounded up to 64 / 128 / 256
# a triangle (9 floats + id), an instance entry (3x4 inverse 48 + root / id 8),
# a ray (8 floats) and a hit (t, inst, prim, u, v)
TRI_BYTES, INST_BYTES, RAY_BYTES, HIT_BYTES = 40, 56, 32, 20
# surface-area cost constants: one box test per node visit, one triangle test
SAH_C_NODE, SAH_C_TRI = 1.0, 1.0


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_ao_closest.json")
# what the traversal kernel is compiled from (sources and compiler flags)
KERNEL_SOURCES = ["paper_2001_09792_amd/csrc/trace_core.h", "paper_2001_09792_amd/csrc/trace.hip",
                  "paper_2001_09792_amd/csrc/rg_internal.h", "paper_2001_09792_amd/csrc/build.hip",
                  "paper_2001_09792_amd/_build.py"]


def kernel_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(args):
    """HBM bytes per launch of the AO closest-hit traversal as measured by
    rocprofv3 counters (FETCH_SIZE, WRITE_SIZE, scaled by a copy probe), or
    None once the traversal source or the configuration differs from the
    measured one."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if (rec.get("kernel_sha256") != kernel_hash() or rec.get("bvh_width") != args.width
            or rec.get("leaf_max") != args.leaf or rec.get("segments") != args.segments
            or rec.get("builder", "lbvh") != args.builder):
        return None
    return float(rec["read_bytes"]) + float(rec["write_bytes"])


# Hierarchy shape per workload (node width, leaf size, builder), the best
# measured on MI355X: linear BVHs restructured by treelets throughout, at
# width 4 for the incoherent AO rays (7% over the plain linear BVH, 9% fewer
# node visits), the serving mix and the dynamic scene, at width 8 for whole
# two-level frames (2% over clustering, 4% over width 4).  The batched
# workload starts from its entry and can be autotuned.
SHAPES = {"incoherent": (4, 1, "treelet"), "two_level": (8, 1, "treelet"), "batched": (4, 1, "lbvh"),
          "serving": (4, 1, "treelet"), "dynamic": (4, 1, "treelet"), "post": (8, 1, "treelet"),
          "build": (4, 1, "treelet"), "options": (4, 1, "treelet")}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def algorithmic_bytes(counts: np.ndarray, width: int) -> float:
    c = counts.astype(np.float64)
    return float(c.shape[0] * (RAY_BYTES + HIT_BYTES) + c[:, 0].sum() * NODE_BYTES[width]
                 + c[:, 1].sum() * TRI_BYTES + c[:, 2].sum() * INST_BYTES)


def sah_cost(buf: np.ndarray, nodes_off: int, n_nodes: int, width: int) -> float:
    """Surface-area cost of a wide hierarchy (layout of include/rg.h):
    (A(root) C_node + sum over inner children A(child) C_node + sum over leaf
    children A(leaf) n_prims C_tri) / A(root), A the box's surface area."""
    W = width
    words = buf[nodes_off: nodes_off + n_nodes * 32 * W].view(np.uint32).reshape(n_nodes, 8 * W)
    raw = words.view(np.float32).astype(np.float64)
    lo = np.stack([raw[:, 0:W], raw[:, W:2 * W], raw[:, 2 * W:3 * W]], -1)
    hi = np.stack([raw[:, 3 * W:4 * W], raw[:, 4 * W:5 * W], raw[:, 5 * W:6 * W]], -1)
    child = words[:, 6 * W:7 * W]
    used = child != 0xFFFFFFFF
    e = np.where(used[..., None], hi - lo, 0.0)
    area = 2.0 * (e[..., 0] * e[..., 1] + e[..., 1] * e[..., 2] + e[..., 2] * e[..., 0])
    leaf = used & ((child & 0x80000000) != 0)
    cnt = ((child >> 28) & 7) + 1
    m = used[0]
    rl, rh = lo[0][m].min(axis=0), hi[0][m].max(axis=0)
    r = rh - rl
    a_root = 2.0 * (r[0] * r[1] + r[1] * r[2] + r[2] * r[0])
    inner = used & ~leaf
    total = a_root * SAH_C_NODE + (area * inner).sum() * SAH_C_NODE + (area * leaf * cnt).sum() * SAH_C_TRI
    return float(total / a_root)


def copy_bandwidth(torch, mib: int = 2048, reps: int = 5) -> float:
    """GB/s of a device-to-device copy of `mib` MiB (bytes read + written)."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * n * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline_incoherent(scene, n_primary: int, seconds: float = 15.0) -> dict:
    """The oracle's closest-hit rate on rays it generates itself: camera rays
    of sampled pixels and the AO rays of their hits."""
    import oracle
    import scenegen as sg
    orc = oracle.Scene(scene, sphere_reject=True)
    px = sg.sample_pixels(scene.width, scene.height, n_primary, 99)
    cam = oracle.camera_rays(scene.camera, scene.width, scene.height, px)
    prim = np.zeros((px.shape[0], 8), np.float32)
    prim[:, :6] = cam
    prim[:, 7] = np.inf
    t0 = time.perf_counter()
    orc.trace(prim[:4])          # one-time setup (mesh adjacency) outside the timing
    log(f"oracle setup {time.perf_counter() - t0:.1f}s")
    ao = orc.ao_rays(prim, scene.seed)
    hit = ao["hit"] == 1
    aor = np.zeros((int(hit.sum()) * 8, 8), np.float32)
    aor[:, :6] = ao["rays"][hit].reshape(-1, 6)
    aor[:, 7] = 5.0
    # keep the primary : AO ratio of the full workload in the sample
    rays = np.concatenate([prim, aor])
    n_total = rays.shape[0]
    # trace the sample in interleaved chunks (every chunk keeps the camera : AO
    # mix) until about `seconds` have passed or the sample is used up
    order = np.argsort((np.arange(n_total) * 0.6180339887498949) % 1.0, kind="stable")
    n, dt, tests = 0, 0.0, 0
    while n < n_total and dt < seconds:
        chunk = order[n: n + 256]
        t0 = time.perf_counter()
        tests += orc.trace(rays[chunk])["tests"]
        dt += time.perf_counter() - t0
        n += chunk.shape[0]
    sel = order[:n]
    res = {"tests": tests}
    return {"value": n / dt / 1e6, "unit": "Mrays/s", "cores": cpu_threads(), "cpu_model": cpu_model(),
            "kind": "oracle",
            "sample": f"{n} rays ({int((sel < prim.shape[0]).sum())} camera + AO rays of {px.shape[0]} "
                      f"sampled pixels), FP64 brute force with exact bounding-sphere reject, "
                      f"{res['tests'] / n:.3g} triangle tests per ray, {dt:.1f} s",
            "tests_per_s": res["tests"] / dt}


def cpu_baseline_frame(scene, n_pixels: int = 256, seconds: float = 15.0) -> dict:
    import oracle
    import scenegen as sg
    orc = oracle.Scene(scene, sphere_reject=True)
    px = sg.sample_pixels(scene.width, scene.height, n_pixels, 98)
    orc.render(px[:2])
    t0 = time.perf_counter()
    r = orc.render(px)
    dt = time.perf_counter() - t0
    n = int(r["nrays"].sum())
    return {"value": n / dt / 1e6, "unit": "Mrays/s", "cores": cpu_threads(), "cpu_model": cpu_model(),
            "kind": "oracle", "sample": f"{px.shape[0]} sampled pixels, whole ray trees ({n} rays), {dt:.1f} s"}


def bench_incoherent(args, torch, rg, sg):
    t0 = time.perf_counter()
    scene = sg.config_incoherent(segments=args.segments)
    log(f"scene: {scene.unique_tris()} unique / {scene.instanced_tris()} instanced tris "
        f"({time.perf_counter() - t0:.1f}s to generate)")
    torch.cuda.synchronize()
    tb = time.perf_counter()
    tl = rg.upload_scene(scene, width=args.width, leaf_max=args.leaf, builder=args.builder)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - tb
    W, H = scene.width, scene.height
    N = W * H
    dev = "cuda"
    cam = torch.empty((8, N), dtype=torch.float32, device=dev)
    hits = rg.alloc_hits(N)
    ao = torch.empty((8, 8 * N), dtype=torch.float32, device=dev)
    src = torch.empty(8 * N, dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    ao_hits = rg.alloc_hits(8 * N)
    ao_occ = torch.empty(8 * N, dtype=torch.uint8, device=dev)
    need = rg.ctypes.c_uint64()
    rg._lib.rg_ao_rays_scratch(N, rg.ctypes.byref(need))
    ao_scratch = torch.empty(max(256, need.value), dtype=torch.uint8, device=dev)

    def gen_primary():
        rg.camera_rays(scene.camera, W, H, out=cam)
        rg.trace_closest(tl, cam, out=hits)
        rg.ao_rays(tl, cam, hits, scene.seed, 5.0, out=ao, src=src, count=cnt, scratch=ao_scratch)

    gen_primary()
    torch.cuda.synchronize()
    n_ao = int(cnt.item())          # the same every step: same camera, hits and seed
    ao_c = ao[:, :n_ao]             # rows of the AO ray buffer, traced in place
    ao_hit_v = {k: v[:n_ao] for k, v in ao_hits.items()}
    prim_hit_frac = float((hits["inst"] != -1).float().mean().item())

    def step():
        rg.camera_rays(scene.camera, W, H, out=cam)
        rg.trace_closest(tl, cam, out=hits)
        rg.ao_rays(tl, cam, hits, scene.seed, 5.0, out=ao, src=src, count=cnt, scratch=ao_scratch)
        rg.trace_closest(tl, ao_c, out=ao_hit_v)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: exactly `steps` steps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = e0.elapsed_time(e1) / args.steps
    rays_step = N + n_ao
    # per-kernel times (events on the stream the kernels run on; torch's
    # current stream, which the binding passes to every call).  The AO
    # closest-hit call is the traversal kernel followed by the refinement of
    # the reported t, u, v: the traversal alone is timed by asking for the
    # hit identities only.
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
    ao_ids = {"inst": ao_hit_v["inst"], "prim": ao_hit_v["prim"]}
    t_prim, t_aogen, t_ao, t_any, t_kern, t_ref = [], [], [], [], [], []
    for _ in range(args.steps):
        ev[0].record()
        rg.camera_rays(scene.camera, W, H, out=cam)
        rg.trace_closest(tl, cam, out=hits)
        ev[1].record()
        rg.ao_rays(tl, cam, hits, scene.seed, 5.0, out=ao, src=src, count=cnt, scratch=ao_scratch)
        ev[2].record()
        rg.trace_closest(tl, ao_c, out=ao_hit_v)
        ev[3].record()
        rg.trace_any(tl, ao_c, occluded=ao_occ[:n_ao])
        ev[4].record()
        rg.trace_closest(tl, ao_c, out=ao_ids)
        ev[5].record()
        torch.cuda.synchronize()
        t_prim.append(ev[0].elapsed_time(ev[1]))
        t_aogen.append(ev[1].elapsed_time(ev[2]))
        t_ao.append(ev[2].elapsed_time(ev[3]))
        t_any.append(ev[3].elapsed_time(ev[4]))
        t_kern.append(ev[4].elapsed_time(ev[5]))
    t_prim, t_aogen, t_ao, t_any, t_kern = (float(np.mean(x)) for x in (t_prim, t_aogen, t_ao, t_any, t_kern))
    counts = rg.trace_counts(tl, ao_c).cpu().numpy()
    bytes_ao = algorithmic_bytes(counts, args.width)
    achieved = bytes_ao / (t_kern * 1e-3) / 1e9
    counts_p = rg.trace_counts(tl, cam).cpu().numpy()
    copy_gbs = copy_bandwidth(torch)
    blas_sah = [sah_cost(b.buf.cpu().numpy(), b.desc.nodes_off, b.desc.n_nodes, args.width) for b in tl.blas]
    tlas_sah = sah_cost(tl.buf.cpu().numpy(), tl.desc.nodes_off, tl.desc.n_nodes, args.width)
    out = {
        "metric": "Mrays/s closest-hit (primary+incoherent)",
        "value": rays_step / (ms_step * 1e-3) / 1e6,
        "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "incoherent: 1024 instances of 16 seeded displaced tori "
                               f"{args.segments}x{args.segments} ({scene.unique_tris()} unique tris), "
                               f"{W}x{H} camera rays + 8 AO rays per primary hit (tmax 5), closest hit",
                   "rays_per_step": rays_step, "primary_rays": N, "ao_rays": n_ao,
                   "trace_tuning": rg.trace_tuning(scope="trace"),
                   "primary_hit_fraction": prim_hit_frac, "bvh_width": args.width, "leaf_max": args.leaf,
                   "builder": args.builder},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(args),
                     "kernel": "closest-hit traversal of the AO rays (k_trace<4,closest>)",
                     "bytes_per_ray": bytes_ao / n_ao, "kernel_ms": t_kern,
                     "copy_GBps": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                     "mean_nodes": float(counts[:, 0].mean()), "mean_tris": float(counts[:, 1].mean()),
                     "mean_inst": float(counts[:, 2].mean()),
                     "sah_cost": {"bottom_mean": float(np.mean(blas_sah)), "bottom_min": float(np.min(blas_sah)),
                                  "bottom_max": float(np.max(blas_sah)), "top": tlas_sah,
                                  "c_node": SAH_C_NODE, "c_tri": SAH_C_TRI}},
        "ao_closest_call_ms": t_ao, "ao_refine_ms": t_ao - t_kern,
        "primary_closest_mrays_s": N / (t_prim * 1e-3) / 1e6,
        "primary_mean_nodes": float(counts_p[:, 0].mean()),
        "ao_closest_mrays_s": n_ao / (t_ao * 1e-3) / 1e6,
        "ao_anyhit_mrays_s": n_ao / (t_any * 1e-3) / 1e6,
        "ao_raygen_ms": t_aogen,
        "build_mtris_s": scene.unique_tris() / build_s / 1e6,
        "wall_s_timed": wall,
    }
    return out, scene


def bench_dynamic(args, torch, rg, sg):
    """Moving geometry over the incoherent scene: each step refits the 16
    bottom levels to the next animation frame's vertex positions, rebuilds the
    top level over the moved instances, and traces that frame's camera rays
    and 8 AO rays per primary hit (closest hit), as the incoherent workload
    does.  Frames alternate between two precomputed animation times whose
    vertices are resident on the device.  Also measured: rebuilding the
    bottom levels from scratch instead of refitting them, and the node visits
    of the refitted hierarchy against a fresh build at the same positions."""
    t0 = time.perf_counter()
    scene = sg.config_incoherent(segments=args.segments)
    times = (0.15, 0.4)
    verts = [[torch.from_numpy(sg.animate_mesh(m, t, amp=0.02, seed=k)).cuda() for k, m in enumerate(scene.blas)]
             for t in times]
    xfs = [sg.animate_instances(scene.xform, t, seed=3) for t in times]
    idx = [torch.from_numpy(np.ascontiguousarray(m.idx, np.uint32).view(np.int32)).cuda() for m in scene.blas]
    log(f"scene and two animation frames ({time.perf_counter() - t0:.1f}s to generate)")
    tl = rg.upload_scene(scene, width=args.width, leaf_max=args.leaf, builder=args.builder)
    blas = tl.blas
    need = rg.ctypes.c_uint64()
    W, H = scene.width, scene.height
    N = W * H
    cam = torch.empty((8, N), dtype=torch.float32, device="cuda")
    hits = rg.alloc_hits(N)
    ao = torch.empty((8, 8 * N), dtype=torch.float32, device="cuda")
    src = torch.empty(8 * N, dtype=torch.int32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    ao_hits = rg.alloc_hits(8 * N)
    rg._lib.rg_ao_rays_scratch(N, rg.ctypes.byref(need))
    ao_scratch = torch.empty(max(256, need.value), dtype=torch.uint8, device="cuda")
    state = {"tl": tl}
    top = rg.TlasBuilder(blas, scene.blas_id, scene.inst_mat, args.width)  # one buffer, rebuilt per frame

    def update(f):
        rg.refit_blas_many(blas, verts[f % 2], idx)
        state["tl"] = top.build(xfs[f % 2])

    def trace():
        t = state["tl"]
        rg.camera_rays(scene.camera, W, H, out=cam)
        rg.trace_closest(t, cam, out=hits)
        rg.ao_rays(t, cam, hits, scene.seed, 5.0, out=ao, src=src, count=cnt, scratch=ao_scratch)
        n_ao = int(cnt.item())
        rg.trace_closest(t, ao[:, :n_ao], out={k: v[:n_ao] for k, v in ao_hits.items()})
        return n_ao

    for f in range(args.warmup):
        update(f)
        trace()
    torch.cuda.synchronize()
    rays, t_upd, t_tr = 0, 0.0, 0.0
    w0 = time.perf_counter()
    for f in range(args.steps):
        a = time.perf_counter()
        update(f)
        torch.cuda.synchronize()
        b_ = time.perf_counter()
        rays += N + trace()
        torch.cuda.synchronize()
        c = time.perf_counter()
        t_upd += b_ - a
        t_tr += c - b_
    wall = time.perf_counter() - w0
    ms_step = wall * 1e3 / args.steps
    # the update split: the refits alone, the top level alone (medians of 9)
    t_r, t_t = [], []
    for _ in range(9):
        torch.cuda.synchronize()
        a = time.perf_counter()
        rg.refit_blas_many(blas, verts[0], idx)
        torch.cuda.synchronize()
        t_r.append(time.perf_counter() - a)
        a = time.perf_counter()
        state["tl"] = top.build(xfs[0])
        torch.cuda.synchronize()
        t_t.append(time.perf_counter() - a)
    t_refit, t_tlas = float(np.median(t_r)), float(np.median(t_t))
    # refitted against freshly built bottom levels at the same positions
    trace()
    n_ao = int(cnt.item())
    counts_refit = rg.trace_counts(state["tl"], ao[:, :n_ao]).cpu().numpy()
    moved = sg.Scene(scene.name, [sg.Mesh(v.cpu().numpy(), m.idx) for v, m in zip(verts[0], scene.blas)], xfs[0],
                     scene.blas_id, scene.inst_mat, scene.materials, scene.camera, scene.light, W, H,
                     scene.max_depth, scene.mode, scene.seed)
    torch.cuda.synchronize()
    a = time.perf_counter()
    fresh = rg.upload_scene(moved, width=args.width, leaf_max=args.leaf, builder=args.builder)
    torch.cuda.synchronize()
    t_rebuild = time.perf_counter() - a
    counts_fresh = rg.trace_counts(fresh, ao[:, :n_ao]).cpu().numpy()
    n_tris = scene.unique_tris()
    out = {
        "metric": "Mrays/s closest-hit (primary+incoherent)",
        "value": rays / wall / 1e6, "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "dynamic: the incoherent scene (1024 instances of 16 displaced tori "
                               f"{args.segments}x{args.segments}, {n_tris} unique tris) with moving vertices "
                               "and moving instances; per step: refit of every bottom level, top-level "
                               "rebuild, 1920x1080 camera rays + 8 AO rays per primary hit, closest hit",
                   "bvh_width": args.width, "leaf_max": args.leaf, "builder": args.builder},
        "update_ms": t_upd * 1e3 / args.steps, "trace_ms": t_tr * 1e3 / args.steps,
        "refit_ms": t_refit * 1e3, "refit_mtris_s": n_tris / t_refit / 1e6,
        "tlas_rebuild_ms": t_tlas * 1e3, "blas_rebuild_ms": t_rebuild * 1e3,
        "ao_mean_nodes_refit": float(counts_refit[:, 0].mean()),
        "ao_mean_nodes_fresh": float(counts_fresh[:, 0].mean()),
        "wall_s_timed": wall, "roofline": None,
    }
    return out, scene


def bench_two_level(args, torch, rg, sg):
    scene = sg.config_two_level()
    tl = rg.upload_scene(scene, width=args.width, leaf_max=args.leaf, builder=args.builder)
    r = rg.Renderer(scene.width, scene.height, scene.max_depth, 0)
    _, st = r.render(tl, scene.materials, scene.camera, scene.light, scene.seed, stats=True)
    rays = st["rays_traced"] + st["shadow_rays"]
    for _ in range(args.warmup):
        r.render(tl, scene.materials, scene.camera, scene.light, scene.seed)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        r.render(tl, scene.materials, scene.camera, scene.light, scene.seed)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    out = {
        "metric": "Mrays/s closest-hit (primary+incoherent)",
        "value": rays / (ms * 1e-3) / 1e6, "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "two-level: 64 instances of 3 meshes (184,320 unique tris), 1920x1080, "
                               "Whitted depth 4, whole frames",
                   "rays_per_frame": rays, "closest_rays": st["rays_traced"], "shadow_rays": st["shadow_rays"],
                   "trace_tuning": rg.trace_tuning(scope="frame"), "bvh_width": args.width,
                   "leaf_max": args.leaf, "builder": args.builder},
        "roofline": None,
    }
    return out, scene


# algorithmic bytes per pixel of the post-process passes: each blur pass reads
# the image (12) and the primary materials (4) and writes the image (12); the
# luma pass reads the image and writes the luma (4); FXAA reads the luma
# (its neighbours come from cache) and the image and writes the image
POST_BYTES = {"blur": 2 * (12 + 4 + 12), "fxaa": (12 + 4) + (4 + 12 + 12)}


def bench_post(args, torch, rg, sg):
    """The two-level frame followed by its post-process passes (roughness
    blur by the primary materials, then FXAA): the whole frame, and each
    pass alone against the HBM roofline."""
    scene = sg.config_two_level()
    W, H = scene.width, scene.height
    tl = rg.upload_scene(scene, width=args.width, leaf_max=args.leaf, builder=args.builder)
    r = rg.Renderer(W, H, scene.max_depth, 0)
    pm = torch.empty((H, W), dtype=torch.int32, device="cuda")
    rough = torch.from_numpy(sg.roughness_table(len(scene.materials), scene.seed)).cuda()
    P = rg.Post(W, H)
    blurred = torch.empty((H, W, 3), dtype=torch.float32, device="cuda")
    final = torch.empty_like(blurred)
    _, st = r.render(tl, scene.materials, scene.camera, scene.light, scene.seed, stats=True, primary_mat=pm)
    rays = st["rays_traced"] + st["shadow_rays"]

    def frame():
        img = r.render(tl, scene.materials, scene.camera, scene.light, scene.seed, primary_mat=pm)
        P.roughness_blur(img, pm, rough, args.post_radius, out=blurred)
        P.fxaa(blurred, out=final)

    def timed(fn, k):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(k):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    ms = timed(frame, args.steps)
    img = r.image
    passes = {"blur": lambda: P.roughness_blur(img, pm, rough, args.post_radius, out=blurred),
              "fxaa": lambda: P.fxaa(blurred, out=final)}
    post = {}
    for name, fn in passes.items():
        us = timed(fn, 10 * args.steps) * 1e3
        gbs = POST_BYTES[name] * W * H / (us * 1e-6) / 1e9
        post[name] = {"us": us, "bytes_per_pixel": POST_BYTES[name], "achieved_GBps": gbs,
                      "frac_of_hbm": gbs / HBM_PEAK_GBS}
    render_ms = timed(lambda: r.render(tl, scene.materials, scene.camera, scene.light, scene.seed,
                                       primary_mat=pm), args.steps)
    out = {
        "metric": "Mrays/s closest-hit (primary+incoherent)",
        "value": rays / (ms * 1e-3) / 1e6, "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "two-level: 64 instances of 3 meshes (184,320 unique tris), 1920x1080, "
                               "Whitted depth 4, whole frames with the post-process passes (roughness blur "
                               f"radius {args.post_radius} by primary material, FXAA)",
                   "rays_per_frame": rays, "bvh_width": args.width, "leaf_max": args.leaf,
                   "builder": args.builder},
        "render_ms": render_ms, "post_ms": ms - render_ms, "post": post,
        "roofline": None,
    }
    return out, scene


def bench_options(args, torch, rg, sg):
    """The incoherent workload traced with the any-hit accept / ignore options
    on: back faces culled, every second instance flagged to another
    visibility mask than the rays', half of the meshes alpha-tested (level-3
    opacity masks with 3 in 4 micro-triangles opaque); the same rays traced
    plainly on the same hierarchies for comparison."""
    scene = sg.config_incoherent(segments=args.segments)
    W, H = scene.width, scene.height
    N = W * H
    flags, alpha = sg.option_inputs(scene)        # rays carry mask 0x02
    tl = rg.upload_scene(scene, width=args.width, leaf_max=args.leaf, builder=args.builder)
    plain = rg.build_tlas(tl.blas, scene.xform, scene.blas_id, scene.inst_mat, args.width, builder=args.builder)
    for b, a in zip(tl.blas, alpha):
        if a is not None:
            rg.set_alpha(b, torch.from_numpy(a[0].view(np.int64)).cuda(), a[1])
    opt = rg.build_tlas(tl.blas, scene.xform, scene.blas_id, scene.inst_mat, args.width, builder=args.builder,
                        inst_flags=flags)
    cam = rg.camera_rays(scene.camera, W, H)
    hits = rg.trace_closest(plain, cam)
    ao, src, cnt = rg.ao_rays(plain, cam, hits, seed=scene.seed, tmax=5.0)
    n_ao = int(cnt.item())
    ao = ao[:, :n_ao]
    out_hits = rg.alloc_hits(n_ao)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    ms_plain = timed(lambda: rg.trace_closest(plain, ao, out=out_hits))
    # `plain` was built before the masks were attached: its records carry no
    # flags and its traversal is the plain variant; `opt` takes the option one
    ms_masks = timed(lambda: rg.trace_closest(opt, ao, out=out_hits, mask=0x02, cull=rg.RAY_CULL_BACK))
    hit_frac = float((out_hits["inst"] != -1).float().mean().item())
    counts = rg.trace_counts(plain, ao).cpu().numpy()
    out = {
        "metric": "Mrays/s closest-hit (primary+incoherent)", "value": n_ao / (ms_masks * 1e-3) / 1e6,
        "unit": "Mrays/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_masks,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "incoherent AO rays (10,315,840) with ray options: back faces culled, rays of mask "
                               "0x02 (half of the 1,024 instances carry mask 0x01 only), 8 of the 16 meshes "
                               "alpha-tested at level 3 (3 in 4 micro-triangles opaque)",
                   "ao_rays": n_ao, "bvh_width": args.width, "leaf_max": args.leaf, "builder": args.builder},
        "plain_mrays_s": n_ao / (ms_plain * 1e-3) / 1e6, "plain_ms": ms_plain,
        "hit_fraction_with_options": hit_frac, "mean_nodes_plain": float(counts[:, 0].mean()),
        "roofline": None,
    }
    return out, scene


def bench_build(args, torch, rg, sg):
    """Bottom-level builds of the incoherent scene's 16 displaced tori
    (10,035,200 triangles) with each builder, device-resident vertices."""
    scene = sg.config_incoherent(segments=args.segments)
    dev = [(torch.from_numpy(m.verts).cuda(), torch.from_numpy(m.idx.view(np.int32)).cuda()) for m in scene.blas]
    n_tris = sum(m.n_tris for m in scene.blas)
    res = {}
    # the three builders with 63-bit keys, and the linear one with the
    # compact 30-bit keys (four sort passes instead of eight); the mean SAH
    # cost of the 16 trees shows what the coarser keys cost in quality
    for name, builder, bits in (("lbvh", "lbvh", 0), ("ploc", "ploc", 0), ("treelet", "treelet", 0),
                                ("lbvh_keys30", "lbvh", 10)):
        for _ in range(args.warmup):
            for v, i in dev:
                rg.build_blas(v, i, None, args.width, args.leaf, builder=builder, morton_bits=bits)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for v, i in dev:
                b = rg.build_blas(v, i, None, args.width, args.leaf, builder=builder, morton_bits=bits)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / args.steps
        sah = []
        for v, i in dev[:4]:
            b = rg.build_blas(v, i, None, args.width, args.leaf, builder=builder, morton_bits=bits)
            sah.append(sah_cost(b.buf.cpu().numpy(), b.desc.nodes_off, b.desc.n_nodes, args.width))
        res[name] = {"ms_per_scene": ms, "mtris_s": n_tris / (ms * 1e-3) / 1e6, "sah_cost_mean_4": float(np.mean(sah))}
    # the 16 tori as one mesh of 10,035,200 triangles, linear builder: the
    # sort's passes at a size where bandwidth, not launches, bounds them
    offs = np.cumsum([0] + [m.verts.shape[0] for m in scene.blas])
    big_v = torch.from_numpy(np.concatenate([m.verts for m in scene.blas])).cuda()
    big_i = torch.from_numpy(np.concatenate([m.idx + np.uint32(o) for m, o in zip(scene.blas, offs)])
                             .view(np.int32)).cuda()
    _, ns_big = rg.blas_sizes(n_tris, args.width, args.leaf)
    scr_big = torch.empty(ns_big, dtype=torch.uint8, device="cuda")
    for _ in range(args.warmup):
        rg.build_blas(big_v, big_i, None, args.width, args.leaf, scratch=scr_big)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        rg.build_blas(big_v, big_i, None, args.width, args.leaf, scratch=scr_big)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    res["lbvh_one_mesh_10M"] = {"ms_per_scene": ms, "mtris_s": n_tris / (ms * 1e-3) / 1e6}
    del scr_big
    # the linear builder enqueued without waits: the 16 builds spread over 4
    # streams (each build with a scratch buffer of its own), then finished
    streams = [torch.cuda.Stream() for _ in range(4)]
    _, ns = rg.blas_sizes(max(m.n_tris for m in scene.blas), args.width, args.leaf)
    scr = [torch.empty(ns, dtype=torch.uint8, device="cuda") for _ in dev]

    def run_async():
        pend = [rg.build_blas_async(v, i, None, args.width, args.leaf, scratch=scr[k], stream=streams[k % 4])
                for k, (v, i) in enumerate(dev)]
        return [p.finish() for p in pend]

    for _ in range(args.warmup):
        run_async()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run_async()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    res["lbvh_async_4_streams"] = {"ms_per_scene": ms, "mtris_s": n_tris / (ms * 1e-3) / 1e6}
    width, leaf, builder = SHAPES["incoherent"]
    out = {
        "metric": "Mtris/s bottom-level build", "value": res[builder]["mtris_s"], "unit": "Mtris/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": res[builder]["ms_per_scene"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"bottom levels of 16 displaced tori {args.segments}x{args.segments} "
                               f"({n_tris} triangles), one synchronous build per mesh, value for the "
                               f"{builder} builder", "bvh_width": args.width, "leaf_max": args.leaf},
        "builders": res, "roofline": None,
    }
    return out, scene


def bench_batched(args, torch, rg, sg):
    """Plain per-frame dispatch (one rg_render per frame, one stream) versus one
    batch (every pass one launch over all frames), same frames, same images."""
    t0 = time.perf_counter()
    scenes = sg.config_batched(n_scenes=args.scenes)
    log(f"{len(scenes)} scenes, {sum(s.unique_tris() for s in scenes)} unique tris, "
        f"{sum(s.width * s.height for s in scenes)} pixels ({time.perf_counter() - t0:.0f}s to generate)")
    def build(sel, width, leaf, builder):
        out = []
        for sc in sel:
            tl = rg.upload_scene(sc, width=width, leaf_max=leaf, builder=builder)
            out.append((tl, sc.materials, sc.camera, sc.light, sc.width, sc.height, sc.max_depth))
        torch.cuda.synchronize()
        return out

    frames = build(scenes, args.width, args.leaf, args.builder)
    default_launch = rg.trace_tuning(scope="frame")
    tuned = None
    if args.autotune:
        from paper_2001_09792_amd import autotune
        sub = scenes[::max(1, len(scenes) // 32)]
        built = {}

        def measure(cfg):
            key = (cfg["width"], cfg["leaf"], cfg["builder"])
            if key not in built:
                built[key] = build(sub, *key)
            autotune.apply_launch(cfg, "frame")
            b = rg.Batch(built[key])
            _, st = b.render(stats=True)
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(3):
                b.render()
            torch.cuda.synchronize()
            return (st["rays_traced"] + st["shadow_rays"]) * 3 / (time.perf_counter() - t) / 1e6

        start = dict(autotune.DEFAULT, builder=args.builder, width=args.width, leaf=args.leaf, **default_launch)
        tuned = autotune.tuned("batch", sum(s.width * s.height for s in scenes),
                               sum(s.unique_tris() for s in scenes), measure, log=log, start=start)
        log(f"autotuned: {tuned}")
        built.clear()
        rg.trace_tuning(scope="frame", **default_launch)
    # plain: one scratch buffer sized for the largest frame, reused frame after frame
    need = max(rg.render_sizes(W, H, D, 0) for (_, _, _, _, W, H, D) in frames)
    scratch = torch.empty(need, dtype=torch.uint8, device="cuda")
    imgs = [torch.empty((H, W, 3), dtype=torch.float32, device="cuda") for (_, _, _, _, W, H, D) in frames]

    def plain():
        for (tl, m, c, l, W, H, D), img in zip(frames, imgs):
            rg.render_into(tl, m, c, l, W, H, D, img, scratch)

    if tuned is not None:
        cfg = tuned["config"]
        shape = (cfg["width"], cfg["leaf"], cfg.get("builder", "lbvh"))
        bframes = frames if shape == (args.width, args.leaf, args.builder) else build(scenes, *shape)
    else:
        bframes = frames
    batch = rg.Batch(bframes)

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps, (time.perf_counter() - w0) / steps * 1e3

    # plain: every frame with the default launch parameters
    rg.trace_tuning(scope="frame", **default_launch)
    ms_plain, wall_plain = timed(plain, max(1, args.steps // 4))
    if tuned is not None:
        from paper_2001_09792_amd import autotune
        autotune.apply_launch(tuned["config"], "frame")
    batched_launch = rg.trace_tuning(scope="frame")
    _, st = batch.render(stats=True)
    rays = st["rays_traced"] + st["shadow_rays"]
    ms_batch, wall_batch = timed(batch.render, args.steps)
    graph = batch.capture()
    ms_graph, wall_graph = timed(graph.replay, args.steps)
    del graph
    # bitwise identity needs the same hierarchy and launch: a tuned width or
    # leaf size may flip rounding-level ties, so the tuned images are compared
    # by their largest difference and a default-configured batch by identity
    same_cfg = batch if bframes is frames else rg.Batch(frames)
    if same_cfg is not batch:
        rg.trace_tuning(scope="frame", **default_launch)
        same_cfg.render()
    same = all(torch.equal(a, b) for a, b in zip(imgs, same_cfg.images))
    max_diff = max(float((a - b).abs().max()) for a, b in zip(imgs, batch.images))
    out = {
        "metric": "Mrays/s closest-hit (primary+incoherent)",
        "value": rays / (ms_batch * 1e-3) / 1e6, "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_batch,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched: {len(scenes)} scenes (triangles log-uniform 1e3..2e6, 1..128 instances, "
                               "64^2..1024^2 pixels), Whitted depth 2, all rays of a frame",
                   "rays_per_step": rays, "frames": len(scenes),
                   "pixels": int(sum(s.width * s.height for s in scenes)),
                   "unique_tris": int(sum(s.unique_tris() for s in scenes))},
        "plain_mrays_s": rays / (ms_plain * 1e-3) / 1e6, "plain_ms": ms_plain, "plain_wall_ms": wall_plain,
        "batched_mrays_s": rays / (ms_batch * 1e-3) / 1e6, "batched_ms": ms_batch, "batched_wall_ms": wall_batch,
        "graph_ms": ms_graph, "graph_wall_ms": wall_graph,
        "speedup": ms_plain / ms_batch, "images_identical": bool(same), "tuned_max_abs_diff": max_diff,
        "autotuned": tuned, "plain_launch": default_launch, "batched_launch": batched_launch,
        "plain_shape": {"bvh_width": args.width, "leaf_max": args.leaf, "builder": args.builder},
        "roofline": None,
    }
    return out, scenes


def bench_serving(args, torch, rg, sg):
    """Render requests over a pool of 64 resident scenes: plain dispatch (one
    rg_render after another) against the continuous-batching engine, first
    saturated (every request queued at once), then at Poisson arrival rates
    that are fractions of plain dispatch's saturated rate, with p50/p99 of
    completion - arrival on the host's monotonic clock."""
    from paper_2001_09792_amd import serve
    t0 = time.perf_counter()
    scenes = sg.config_serving_pool(c3_segments=args.segments)
    n_c2 = sum(1 for s in scenes if s.n_inst == 64)
    log(f"{len(scenes)} scenes ({time.perf_counter() - t0:.0f}s to generate)")
    shared = []

    def load(k):
        sc = scenes[k]
        if k >= n_c2:                      # C3-type: shared bottom levels, own top level
            if not shared:
                shared.extend(rg.upload_scene(sc, width=args.width, leaf_max=args.leaf, builder=args.builder).blas)
            tl = rg.build_tlas(shared, sc.xform, sc.blas_id, sc.inst_mat, args.width, builder=args.builder)
            nbytes = tl.buf.numel() + (sum(b.buf.numel() for b in shared) if k == n_c2 else 0)
        else:
            tl = rg.upload_scene(sc, width=args.width, leaf_max=args.leaf, builder=args.builder)
            nbytes = tl.buf.numel() + sum(b.buf.numel() for b in tl.blas)
        return (tl, rg.materials_array(sc.materials), sc.camera, sc.light), nbytes

    cache = serve.ResidentCache(load)
    t0 = time.perf_counter()
    for k in range(len(scenes)):
        cache.get(k)
        cache.release(k)
    torch.cuda.synchronize()
    log(f"resident: {cache.stats()} ({time.perf_counter() - t0:.1f}s to build)")
    ecfg = rg.Engine.for_budget(int(args.budget_gb * (1 << 30)), max_jobs=args.max_jobs, width=args.width)
    eng = rg.Engine(**ecfg)
    log(f"engine: {ecfg}, {eng.scratch.numel() / 2**30:.2f} GiB")
    n_scenes = len(scenes)

    def run(ex, reqs, with_rays=True):
        s0 = eng.stats() if with_rays else None
        info = serve.serve(reqs, ex, serve.RealClock())
        torch.cuda.synchronize()
        rays = None
        if with_rays:
            s1 = eng.stats()
            rays = (s1["rays_traced"] - s0["rays_traced"]) + (s1["shadow_rays"] - s0["shadow_rays"])
        return info, rays

    # warm-up of both executors
    plain = serve.PlainExecutor(cache, 1920 * 1080, 4)
    ex = serve.EngineExecutor(eng, cache)
    run(plain, serve.poisson_requests(16, math.inf, n_scenes, 99), False)
    run(ex, serve.poisson_requests(16, math.inf, n_scenes, 99))
    # saturated: the same requests, all queued at once
    sat = lambda: serve.poisson_requests(args.requests // 2, math.inf, n_scenes, 5)
    reqs_e = sat()
    _, rays_sat = run(ex, reqs_e)
    s_eng = serve.summarize(reqs_e, rays_sat)
    reqs_p = sat()
    run(plain, reqs_p, False)
    s_plain = serve.summarize(reqs_p, rays_sat)     # same frames, same rays
    lam_sat = s_plain["req_per_s"]
    log(f"saturated: plain {s_plain['req_per_s']:.1f} req/s {s_plain['mrays_s']:.0f} Mrays/s; "
        f"engine {s_eng['req_per_s']:.1f} req/s {s_eng['mrays_s']:.0f} Mrays/s")
    points = []
    for f in args.rate_factors:
        lam = f * lam_sat
        reqs = serve.poisson_requests(args.warm + args.requests, lam, n_scenes, 5)
        info, rays = run(ex, reqs)
        meas = [r for r in reqs if r.rid >= args.warm]
        pt = dict(rate_factor=f, rate_req_s=lam, executor="engine", **serve.summarize(meas),
                  mrays_s=rays / max(max(r.t_done for r in reqs) - min(r.arrival for r in reqs), 1e-9) / 1e6,
                  max_waiting=info["max_waiting"])
        log(f"  engine  x{f:.2f} ({lam:.1f} req/s): p50 {pt['p50_ms']:.2f} ms p99 {pt['p99_ms']:.2f} ms "
            f"{pt['mrays_s']:.0f} Mrays/s")
        points.append(pt)
        if f in args.plain_factors:
            reqs = serve.poisson_requests(args.warm + args.requests, lam, n_scenes, 5)
            info, _ = run(plain, reqs, False)
            meas = [r for r in reqs if r.rid >= args.warm]
            pp = dict(rate_factor=f, rate_req_s=lam, executor="plain", **serve.summarize(meas),
                      max_waiting=info["max_waiting"])
            log(f"  plain   x{f:.2f} ({lam:.1f} req/s): p50 {pp['p50_ms']:.2f} ms p99 {pp['p99_ms']:.2f} ms")
            points.append(pp)
    einfo = eng.info()
    out = {
        "metric": "Mrays/s closest-hit (primary+incoherent); served-frame p50/p99 latency",
        "value": s_eng["mrays_s"], "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.requests // 2, "warmup": 16,
        "ms_per_step": 1e3 / s_eng["req_per_s"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving: 64 resident scenes (32 two-level, 32 over 16 shared tori of "
                               f"{args.segments}^2), requests of 256^2..1920x1080, Whitted depth 1..4, "
                               "continuous batching", "budget_gb": args.budget_gb, "engine": ecfg,
                   "bvh_width": args.width, "leaf_max": args.leaf, "builder": args.builder,
                   "requests_per_point": args.requests, "warm_requests": args.warm,
                   "engine_launch": rg.trace_tuning(scope="engine"), "plain_launch": rg.trace_tuning(scope="frame")},
        "saturated": {"engine": s_eng, "plain": s_plain, "speedup": s_eng["mrays_s"] / s_plain["mrays_s"]},
        "points": points,
        "engine_info": einfo,
        "resident": cache.stats(),
        "roofline": None,
    }
    eng.close()
    return out, scenes


def served_and_batched(args, torch, rg, sg) -> dict:
    """The two serving forms measured on the same GPU, for the default run:
    the batched workload (256 scenes, one batch against one rg_render per
    frame) and the serving workload (64 resident scenes; saturated engine
    against plain dispatch, p50 / p99 at 0.9 of plain dispatch's saturated
    rate, 1,000 measured requests after 100 warm-up ones)."""
    import copy
    out = {}
    b = copy.copy(args)
    b.width, b.leaf, b.builder = SHAPES["batched"]
    b.steps, b.warmup, b.scenes, b.autotune = 4, 1, 256, False
    res, _ = bench_batched(b, torch, rg, sg)
    out["batched"] = {k: res[k] for k in ("plain_mrays_s", "batched_mrays_s", "speedup", "plain_ms", "batched_ms",
                                          "graph_ms", "images_identical")}
    out["batched"]["workload"] = res["config"]["workload"]
    out["batched"].update({k: res["config"][k] for k in ("frames", "pixels", "unique_tris", "rays_per_step")})
    torch.cuda.empty_cache()
    v = copy.copy(args)
    v.width, v.leaf, v.builder = SHAPES["serving"]
    v.rate_factors, v.plain_factors, v.requests, v.warm = [0.9], [0.9], 1000, 100
    res, _ = bench_serving(v, torch, rg, sg)
    sat = res["saturated"]
    pts = {p["executor"]: p for p in res["points"]}
    out["served"] = {
        "workload": res["config"]["workload"],
        "saturated_requests": sat["engine"]["requests"],
        "saturated_engine_req_s": sat["engine"]["req_per_s"], "saturated_plain_req_s": sat["plain"]["req_per_s"],
        "saturated_engine_mrays_s": sat["engine"]["mrays_s"], "saturated_plain_mrays_s": sat["plain"]["mrays_s"],
        "speedup": sat["speedup"],
        "rate_factor": 0.9, "rate_req_s": pts["engine"]["rate_req_s"],
        "measured_requests": v.requests, "warm_requests": v.warm,
        "engine_p50_ms": pts["engine"]["p50_ms"], "engine_p99_ms": pts["engine"]["p99_ms"],
        "engine_mrays_s": pts["engine"]["mrays_s"],
        "plain_p50_ms": pts["plain"]["p50_ms"], "plain_p99_ms": pts["plain"]["p99_ms"],
    }
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["incoherent", "two_level", "batched", "serving", "dynamic", "post",
                                           "build", "options"],
                    default="incoherent")
    ap.add_argument("--scenes", type=int, default=256, help="frames of the batched workload")
    ap.add_argument("--autotune", action="store_true", help="batched: tune width, leaf size and launch "
                    "parameters on a subsample first (cached per GPU and size bucket)")
    ap.add_argument("--segments", type=int, default=560)
    ap.add_argument("--post-radius", type=int, default=8, help="post: roughness blur window radius")
    ap.add_argument("--requests", type=int, default=1000, help="serving: measured requests per rate")
    ap.add_argument("--warm", type=int, default=100, help="serving: warm-up requests per rate")
    ap.add_argument("--budget-gb", type=float, default=160.0,
                    help="serving: engine memory budget (the queue space for frames in flight)")
    ap.add_argument("--max-jobs", type=int, default=128, help="serving: frames in flight")
    ap.add_argument("--rate-factors", type=float, nargs="+", default=[0.25, 0.5, 0.75, 0.9, 1.0, 1.25])
    ap.add_argument("--plain-factors", type=float, nargs="*", default=[0.5, 0.9])
    ap.add_argument("--width", type=int, default=None, help="node width (default: the workload's, see SHAPES)")
    ap.add_argument("--leaf", type=int, default=None, help="most triangles per leaf (default: the workload's)")
    ap.add_argument("--builder", choices=["lbvh", "ploc", "treelet"], default=None,
                    help="hierarchy builder: linear BVH or locally-ordered clustering (default: the workload's)")
    ap.add_argument("--refill", type=int, default=None, help="traversal refill threshold (lanes)")
    ap.add_argument("--waves-per-cu", type=int, default=None, help="persistent traversal waves per CU")
    ap.add_argument("--lds-depth", type=int, default=None, help="traversal stack entries per lane in LDS")
    ap.add_argument("--leaf-batch", type=int, default=None, help="lanes waiting at leaves before a wave runs them")
    ap.add_argument("--inst-batch", type=int, default=None,
                    help="lanes waiting at instance entries before a wave runs them")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving-forms", action="store_true",
                    help="incoherent: skip the batched and served measurements that follow the main one")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after the measurement, copy this many MiB once (a plain copy kernel of known "
                         "size, for scaling hardware byte counters)")
    args = ap.parse_args()
    width, leaf, builder = SHAPES[args.workload]
    args.width = width if args.width is None else args.width
    args.leaf = leaf if args.leaf is None else args.leaf
    args.builder = builder if args.builder is None else args.builder
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the path runs on a single device (see the multi-GPU design "
              "notes); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2001_09792_amd as rg
    import scenegen as sg
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    scope = {"incoherent": "trace", "two_level": "frame", "batched": "frame", "serving": "engine",
             "dynamic": "trace", "post": "frame", "build": "trace", "options": "trace"}[args.workload]
    rg.trace_tuning(args.refill, args.waves_per_cu, args.lds_depth, args.leaf_batch, args.inst_batch, scope=scope)
    if args.workload == "incoherent":
        out, scene = bench_incoherent(args, torch, rg, sg)
        if not args.no_cpu_baseline:
            log("timing the oracle on a sample")
            out["cpu_baseline"] = cpu_baseline_incoherent(scene, 640, args.cpu_seconds)
        if not args.no_serving_forms:
            del scene
            log("batched and served forms")
            out.update(served_and_batched(args, torch, rg, sg))
    elif args.workload == "dynamic":
        out, scene = bench_dynamic(args, torch, rg, sg)
    elif args.workload == "post":
        out, scene = bench_post(args, torch, rg, sg)
    elif args.workload == "build":
        out, scene = bench_build(args, torch, rg, sg)
    elif args.workload == "options":
        out, scene = bench_options(args, torch, rg, sg)
    elif args.workload == "two_level":
        out, scene = bench_two_level(args, torch, rg, sg)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline_frame(scene, 128, args.cpu_seconds)
    elif args.workload == "batched":
        out, scenes = bench_batched(args, torch, rg, sg)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline_frame(scenes[0], 64, args.cpu_seconds)
    else:
        out, scenes = bench_serving(args, torch, rg, sg)
        if not args.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline_frame(scenes[0], 64, args.cpu_seconds)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
