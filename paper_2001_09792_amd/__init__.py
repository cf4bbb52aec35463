"""Python binding of librg.so (include/rg.h): argument marshalling only.

Every step of the ray-tracing path runs in the HIP kernels of librg.so;
this module only turns torch CUDA tensors into device pointers, owns the
caller-allocated buffers that the C ABI asks for, and maps status codes to
exceptions.  Importing it loads the library and fails loudly if it has not
been built (`python -m paper_2001_09792_amd._build`).
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np
# torch first: it ships its own HIP runtime (soname libamdhip64.so.7); loading
# torch before librg.so makes the dynamic loader bind librg.so to that same
# runtime instead of a second copy from /opt/rocm, which would not see the
# device torch has opened.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
# RG_LIBRARY names another build of the same sources (the sanitizer build of
# the host code used by tests/run_sanitizers.py)
LIB_PATH = os.environ.get("RG_LIBRARY") or os.path.join(_HERE, "librg.so")

RG_OK = 0
MISS = 0xFFFFFFFF
PER_PRIM = 0xFFFFFFFF
MAX_DEPTH = 8
RG_LEVELS_CAP = 255   # include/rg.h: deepest bottom level whose level table is kept
RG_BLUR_RADIUS_MAX = 16  # include/rg.h: widest roughness-blur window
RG_ALPHA_LEVEL_MAX = 3   # include/rg.h: finest opacity-mask subdivision (4^3 micro-triangles)

c_f = ctypes.c_float
c_i32 = ctypes.c_int32
c_i64 = ctypes.c_int64
c_u64 = ctypes.c_uint64
c_u32 = ctypes.c_uint32
c_p = ctypes.c_void_p


class BuildOpts(ctypes.Structure):
    _fields_ = [("width", c_i32), ("leaf_max", c_i32), ("builder", c_i32), ("radius", c_i32),
                ("morton_bits", c_i32)]


class Sizes(ctypes.Structure):
    _fields_ = [("bytes", c_u64), ("scratch_bytes", c_u64)]


class BlasDesc(ctypes.Structure):
    _fields_ = [("buf", c_p), ("nodes_off", c_u64), ("tris_off", c_u64), ("mats_off", c_u64),
                ("slots_off", c_u64), ("parents_off", c_u64), ("levels_off", c_u64), ("n_tris", c_i64), ("n_nodes", c_i64), ("width", c_i32),
                ("leaf_max", c_i32), ("depth", c_i32), ("has_mats", c_i32), ("lo", c_f * 3),
                ("hi", c_f * 3), ("has_alpha", c_i32), ("alpha_level", c_i32)]


class TlasDesc(ctypes.Structure):
    _fields_ = [("buf", c_p), ("nodes_off", c_u64), ("inst_off", c_u64), ("rec_off", c_u64), ("xf_off", c_u64),
                ("n_inst", c_i64), ("n_nodes", c_i64), ("width", c_i32), ("depth", c_i32),
                ("max_blas_depth", c_i32), ("has_inst_flags", c_i32), ("lo", c_f * 3), ("hi", c_f * 3)]


class Rays(ctypes.Structure):
    _fields_ = [(k, c_p) for k in ("ox", "oy", "oz", "dx", "dy", "dz", "tmin", "tmax")]


class TraceOpts(ctypes.Structure):
    _fields_ = [("flags", c_u32), ("mask", c_u32), ("ray_mask", c_p)]


class Hits(ctypes.Structure):
    _fields_ = [("t", c_p), ("inst", c_p), ("prim", c_p), ("u", c_p), ("v", c_p)]


class Capture(ctypes.Structure):
    _fields_ = [("capacity", c_i64), ("rays", c_p), ("t", c_p), ("inst", c_p), ("prim", c_p),
                ("shadow_rays", c_p), ("occluded", c_p), ("counts", c_p)]


class Material(ctypes.Structure):
    _fields_ = [("type", c_i32), ("rgb", c_f * 3), ("ior", c_f)]


class CameraDesc(ctypes.Structure):
    _fields_ = [("eye", c_f * 3), ("target", c_f * 3), ("up", c_f * 3), ("vfov_deg", c_f)]


class LightDesc(ctypes.Structure):
    _fields_ = [("pos", c_f * 3), ("intensity", c_f * 3), ("ambient", c_f)]


class TraceTune(ctypes.Structure):
    _fields_ = [("refill", c_i32), ("waves_per_cu", c_i32), ("lds_depth", c_i32), ("leaf_batch", c_i32),
                ("inst_batch", c_i32)]


class Job(ctypes.Structure):
    _fields_ = [("tlas", c_p), ("mats", c_p), ("n_mats", c_i32), ("cam", CameraDesc), ("light", LightDesc),
                ("width", c_i32), ("height", c_i32), ("max_depth", c_i32), ("mode", c_i32), ("seed", c_u64),
                ("image", c_p)]


class BatchDesc(ctypes.Structure):
    _fields_ = [("scratch", c_p), ("scratch_bytes", c_u64), ("n_jobs", c_i32), ("width", c_i32),
                ("max_depth", c_i32), ("n_mats", c_i32), ("total_pixels", c_i64), ("capacity", c_i64),
                ("cap_at", c_i64 * (MAX_DEPTH + 1)), ("has_inst_flags", c_i32), ("reserved", c_i32)]


class RenderStats(ctypes.Structure):
    _fields_ = [("rays_traced", c_u64), ("shadow_rays", c_u64), ("ms_total", c_f)]


class PoolUsage(ctypes.Structure):
    _fields_ = [("rays", c_i64), ("pixels", c_i64), ("largest_free_pixels", c_i64), ("jobs", c_i32),
                ("reserved", c_i32)]


class EngineDesc(ctypes.Structure):
    _fields_ = [("max_rays", c_i64), ("max_pixels", c_i64), ("max_jobs", c_i32), ("max_mats", c_i32),
                ("width", c_i32), ("reserved", c_i32)]


class EngineInfo(ctypes.Structure):
    _fields_ = [(k, c_i64) for k in ("passes", "passes_done", "frames_live", "frames_active", "admitted",
                                     "completed", "rays_reserved", "pixels_reserved", "max_frames_in_pass",
                                     "max_depths_in_pass")]


# name -> (restype, argtypes); every function of include/rg.h
SIGNATURES = {
    "rg_status_string": (ctypes.c_char_p, [c_i32]),
    "rg_last_error": (ctypes.c_char_p, []),
    "rg_blas_sizes": (c_i32, [c_i64, c_p, c_p]),
    "rg_build_blas": (c_i32, [c_p, c_i64, c_p, c_i64, c_p, c_p, c_p, c_u64, c_p, c_u64, c_p, c_p]),
    "rg_build_blas_async": (c_i32, [c_p, c_i64, c_p, c_i64, c_p, c_p, c_p, c_u64, c_p, c_u64, c_p, c_p]),
    "rg_build_blas_finish": (c_i32, [c_p, c_p]),
    "rg_tlas_ticket_bytes": (c_i32, [c_i64, c_i32, c_i32, c_p]),
    "rg_build_tlas_async": (c_i32, [c_p, c_i32, c_p, c_p, c_p, c_p, c_i64, c_p, c_p, c_u64, c_p, c_u64, c_p, c_p,
                                    c_u64]),
    "rg_build_tlas_finish": (c_i32, [c_p, c_p]),
    "rg_tlas_sizes": (c_i32, [c_i64, c_p, c_p]),
    "rg_build_tlas": (c_i32, [c_p, c_i32, c_p, c_p, c_p, c_i64, c_p, c_p, c_u64, c_p, c_u64, c_p, c_p]),
    "rg_trace_closest": (c_i32, [c_p, Rays, c_i64, Hits, c_p]),
    "rg_trace_any": (c_i32, [c_p, Rays, c_i64, c_p, c_p, c_p]),
    "rg_trace_closest_ex": (c_i32, [c_p, Rays, c_i64, Hits, c_p, c_p]),
    "rg_trace_any_ex": (c_i32, [c_p, Rays, c_i64, c_p, c_p, c_p, c_p]),
    "rg_build_tlas_ex": (c_i32, [c_p, c_i32, c_p, c_p, c_p, c_p, c_i64, c_p, c_p, c_u64, c_p, c_u64, c_p, c_p]),
    "rg_trace_counts": (c_i32, [c_p, Rays, c_i64, c_i32, c_p, c_p]),
    "rg_trace_tuning": (c_i32, [c_i32, c_p, c_p]),
    "rg_camera_rays": (c_i32, [c_p, c_i32, c_i32, c_p, c_p]),
    "rg_ao_rays": (c_i32, [c_p, Rays, c_i64, c_p, c_p, c_p, c_u64, c_f, c_p, c_p, c_p, c_p, c_u64, c_p]),
    "rg_ao_rays_scratch": (c_i32, [c_i64, c_p]),
    "rg_render_sizes": (c_i32, [c_i32, c_i32, c_i32, c_i32, c_p]),
    "rg_render": (c_i32, [c_p, c_p, c_i32, c_p, c_p, c_i32, c_i32, c_i32, c_i32, c_u64, c_p, c_p, c_u64,
                          c_p, c_p]),
    "rg_render_ex": (c_i32, [c_p, c_p, c_i32, c_p, c_p, c_i32, c_i32, c_i32, c_i32, c_u64, c_p, c_p, c_p,
                             c_u64, c_p, c_p]),
    "rg_render_static": (c_i32, [c_p, c_p, c_i32, c_p, c_p, c_i32, c_i32, c_i32, c_i32, c_u64, c_p, c_p]),
    "rg_render_capture": (c_i32, [c_p, c_p, c_i32, c_p, c_p, c_i32, c_i32, c_i32, c_u64, c_p, c_p, c_u64, c_p, c_p]),
    "rg_post_sizes": (c_i32, [c_i32, c_i32, c_p]),
    "rg_blas_set_alpha": (c_i32, [c_p, c_p, c_i32, c_p]),
    "rg_roughness_blur": (c_i32, [c_p, c_p, c_p, c_i32, c_i32, c_i32, c_i32, c_p, c_p, c_u64, c_p]),
    "rg_fxaa": (c_i32, [c_p, c_i32, c_i32, c_p, c_p, c_u64, c_p]),
    "rg_refit_sizes": (c_i32, [c_p, c_p]),
    "rg_refit_blas": (c_i32, [c_p, c_p, c_i64, c_p, c_i64, c_p, c_u64, c_p]),
    "rg_blas_state": (c_i32, [c_p, c_p, c_p, c_p, c_p]),
    "rg_refit_blas_many": (c_i32, [c_p, c_i32, c_p, c_p, c_p, c_p, c_p, c_u64, c_p]),
    "rg_lbvh_stages": (c_i32, [c_p, c_i64, c_p, c_i64, c_p, c_p, c_p, c_p, c_p, c_p, c_p, c_u64, c_p]),
    "rg_batch_sizes": (c_i32, [c_p, c_i32, c_p]),
    "rg_batch_prepare": (c_i32, [c_p, c_i32, c_p, c_u64, c_p, c_p]),
    "rg_batch_render": (c_i32, [c_p, c_p, c_p]),
    "rg_pool_create": (c_i32, [c_i64, c_i64, c_i32, c_p]),
    "rg_pool_destroy": (c_i32, [c_p]),
    "rg_pool_reserve": (c_i32, [c_p, c_i64, c_i64, c_p, c_p]),
    "rg_pool_release": (c_i32, [c_p, c_i32]),
    "rg_pool_get_usage": (c_i32, [c_p, c_p]),
    "rg_job_reservation": (c_i32, [c_p, c_p, c_p]),
    "rg_engine_sizes": (c_i32, [c_p, c_p]),
    "rg_engine_create": (c_i32, [c_p, c_p, c_u64, c_p, c_p]),
    "rg_engine_destroy": (c_i32, [c_p]),
    "rg_engine_admit": (c_i32, [c_p, c_p, c_i64, c_p]),
    "rg_engine_step": (c_i32, [c_p, c_p]),
    "rg_engine_poll": (c_i32, [c_p, c_i32, c_p, c_i32, c_p]),
    "rg_engine_get_info": (c_i32, [c_p, c_p]),
    "rg_engine_stats": (c_i32, [c_p, c_p]),
}


class RgError(RuntimeError):
    def __init__(self, fn: str, status: int, text: str):
        super().__init__(f"{fn} failed: {text} ({status})")
        self.status = status


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python paper_2001_09792_amd/_build.py` "
                          "(there is no fallback implementation)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = load_library()


def _check(fn: str, status: int):
    if status != RG_OK:
        text = _lib.rg_status_string(status).decode()
        if status == -3:
            text += " at " + _lib.rg_last_error().decode()
        raise RgError(fn, status, text)


def _torch():
    import torch
    return torch


def _stream(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _bytes(n: int, device):
    torch = _torch()
    return torch.empty(max(int(n), 256), dtype=torch.uint8, device=device)


# hierarchy builders (include/rg.h RG_BUILDER_*)
BUILDERS = {"lbvh": 0, "ploc": 1, "treelet": 2}
PLOC_RADIUS_DEFAULT = 16


def _opts(width: int, leaf_max: int, builder: str = "lbvh", radius: int = 0, morton_bits: int = 0) -> BuildOpts:
    if builder not in BUILDERS:
        raise ValueError(f"builder must be one of {sorted(BUILDERS)}")
    return BuildOpts(width, leaf_max, BUILDERS[builder], radius, morton_bits)


# -------------------------------------------------------------- bottom level
class Blas:
    """A bottom-level structure: the caller-owned buffer and its descriptor."""

    def __init__(self, buf, desc: BlasDesc):
        self.buf = buf
        self.desc = desc
        self.alpha = None  # opacity masks attached with set_alpha (kept alive here)

    @property
    def n_tris(self) -> int:
        return int(self.desc.n_tris)

    @property
    def depth(self) -> int:
        return int(self.desc.depth)


def blas_sizes(n_tris: int, width: int = 4, leaf_max: int = 4, builder: str = "lbvh", radius: int = 0,
               morton_bits: int = 0):
    s = Sizes()
    o = _opts(width, leaf_max, builder, radius, morton_bits)
    _check("rg_blas_sizes", _lib.rg_blas_sizes(n_tris, ctypes.byref(o), ctypes.byref(s)))
    return int(s.bytes), int(s.scratch_bytes)


def build_blas(verts, idx, prim_mat=None, width: int = 4, leaf_max: int = 4, scratch=None,
               stream=None, builder: str = "lbvh", radius: int = 0, morton_bits: int = 0) -> Blas:
    """verts: CUDA float32 [V,3]; idx: CUDA int32/uint32 [T,3]; prim_mat: CUDA
    int16 [T] or None; builder: "lbvh", "ploc" or "treelet" (radius 0: the
    default); morton_bits: 21 (0: the default) or 10 (30-bit keys, four sort
    passes, up to 2^20 triangles)."""
    n_tris = int(idx.shape[0])
    nb, ns = blas_sizes(n_tris, width, leaf_max, builder, radius, morton_bits)
    buf = _bytes(nb, verts.device)
    if scratch is None or scratch.numel() < ns:
        scratch = _bytes(ns, verts.device)
    d = BlasDesc()
    o = _opts(width, leaf_max, builder, radius, morton_bits)
    _check("rg_build_blas", _lib.rg_build_blas(
        _ptr(verts), int(verts.shape[0]), _ptr(idx), n_tris, _ptr(prim_mat), ctypes.byref(o),
        _ptr(buf), buf.numel(), _ptr(scratch), scratch.numel(), _stream(stream), ctypes.byref(d)))
    return Blas(buf, d)


BUILD_TICKET_BYTES = 1024


class PendingBlas:
    """A bottom-level build enqueued by build_blas_async: the inputs, the
    output and scratch buffers and the pinned ticket stay referenced here
    until finish() returns the Blas."""

    def __init__(self, keep, buf, ticket):
        self._keep = keep
        self.buf = buf
        self.ticket = ticket

    def finish(self) -> Blas:
        d = BlasDesc()
        _check("rg_build_blas_finish", _lib.rg_build_blas_finish(self.ticket.data_ptr(), ctypes.byref(d)))
        self._keep = None
        return Blas(self.buf, d)


def build_blas_async(verts, idx, prim_mat=None, width: int = 4, leaf_max: int = 4, scratch=None,
                     stream=None, morton_bits: int = 0) -> PendingBlas:
    """build_blas for the linear builder without the wait: the build is
    enqueued on `stream` and finish() on the result waits for it.  Builds
    in flight together need scratch buffers of their own (pass none to get
    a new one)."""
    torch = _torch()
    n_tris = int(idx.shape[0])
    nb, ns = blas_sizes(n_tris, width, leaf_max, "lbvh", 0, morton_bits)
    buf = _bytes(nb, verts.device)
    if scratch is None or scratch.numel() < ns:
        scratch = _bytes(ns, verts.device)
    ticket = torch.empty(BUILD_TICKET_BYTES, dtype=torch.uint8, pin_memory=True)
    o = _opts(width, leaf_max, "lbvh", 0, morton_bits)
    _check("rg_build_blas_async", _lib.rg_build_blas_async(
        _ptr(verts), int(verts.shape[0]), _ptr(idx), n_tris, _ptr(prim_mat), ctypes.byref(o),
        _ptr(buf), buf.numel(), _ptr(scratch), scratch.numel(), _stream(stream), ticket.data_ptr()))
    return PendingBlas((verts, idx, prim_mat, scratch), buf, ticket)


def refit_blas(blas: Blas, verts, idx, scratch=None, stream=None) -> Blas:
    """Refits `blas` in place to new vertex positions of the same triangles
    (verts: CUDA float32 [V,3]; idx: the index array it was built from),
    asynchronously.  Top levels over it must be rebuilt afterwards
    (build_tlas, which reports invalid vertex data found by the refit)."""
    need = ctypes.c_uint64()
    _check("rg_refit_sizes", _lib.rg_refit_sizes(ctypes.byref(blas.desc), ctypes.byref(need)))
    if scratch is None or scratch.numel() < need.value:
        scratch = _bytes(need.value, verts.device)
    _check("rg_refit_blas", _lib.rg_refit_blas(
        ctypes.byref(blas.desc), _ptr(verts), int(verts.shape[0]), _ptr(idx), int(idx.shape[0]),
        _ptr(scratch), scratch.numel(), _stream(stream)))
    return blas


def refit_blas_many(blas: Sequence[Blas], verts: Sequence, idx: Sequence, scratch=None, stream=None):
    """refit_blas for several bottom levels of one width in one call (one
    launch per level covers all of them); verts[k], idx[k] as for
    refit_blas."""
    n = len(blas)
    descs = (BlasDesc * n)(*[b.desc for b in blas])
    vp = (c_p * n)(*[_ptr(v) for v in verts])
    ip = (c_p * n)(*[_ptr(i) for i in idx])
    nv = (c_i64 * n)(*[int(v.shape[0]) for v in verts])
    nt = (c_i64 * n)(*[int(i.shape[0]) for i in idx])
    need = 0
    for b in blas:
        if b.desc.depth > RG_LEVELS_CAP:
            q = ctypes.c_uint64()
            _check("rg_refit_sizes", _lib.rg_refit_sizes(ctypes.byref(b.desc), ctypes.byref(q)))
            need = max(need, q.value)
    if need and (scratch is None or scratch.numel() < need):
        scratch = _bytes(need, verts[0].device)
    _check("rg_refit_blas_many", _lib.rg_refit_blas_many(
        descs, n, vp, nv, ip, nt, _ptr(scratch) if need else None, scratch.numel() if need else 0,
        _stream(stream)))
    return blas


def blas_state(blas: Blas, stream=None):
    """(root box lo, root box hi, status of the last refit) from the
    bottom level's header; waits for the stream."""
    lo, hi, st = (c_f * 3)(), (c_f * 3)(), ctypes.c_uint32()
    _check("rg_blas_state", _lib.rg_blas_state(ctypes.byref(blas.desc), lo, hi, ctypes.byref(st), _stream(stream)))
    return list(lo), list(hi), int(st.value)


# ----------------------------------------------------------------- top level
class Tlas:
    def __init__(self, buf, desc: TlasDesc, blas: Sequence[Blas]):
        self.buf = buf
        self.desc = desc
        self.blas = list(blas)   # keeps the bottom levels alive

    @property
    def ref(self):
        return ctypes.byref(self.desc)


def build_tlas(blas: Sequence[Blas], xform, blas_id, inst_mat, width: int = 4, stream=None,
               scratch=None, builder: str = "lbvh", radius: int = 0, inst_flags=None,
               morton_bits: int = 0) -> Tlas:
    """xform: host float32 [I,3,4]; blas_id, inst_mat: host uint32 [I];
    inst_flags: host uint32 [I] (visibility mask in bits 0-7,
    INST_CULL_DISABLE, INST_FLIP_FACING) or None (all visible);
    morton_bits as for build_blas."""
    torch = _torch()
    xform = np.ascontiguousarray(xform, np.float32).reshape(-1, 12)
    blas_id = np.ascontiguousarray(blas_id, np.uint32)
    inst_mat = np.ascontiguousarray(inst_mat, np.uint32)
    n = xform.shape[0]
    s = Sizes()
    o = _opts(width, 1, builder, radius, morton_bits)
    _check("rg_tlas_sizes", _lib.rg_tlas_sizes(n, ctypes.byref(o), ctypes.byref(s)))
    dev = blas[0].buf.device
    buf = _bytes(s.bytes, dev)
    if scratch is None or scratch.numel() < s.scratch_bytes:
        scratch = _bytes(s.scratch_bytes, dev)
    arr = (BlasDesc * len(blas))(*[b.desc for b in blas])
    d = TlasDesc()
    fl = np.ascontiguousarray(inst_flags, np.uint32).reshape(n) if inst_flags is not None else None
    _check("rg_build_tlas", _lib.rg_build_tlas_ex(
        arr, len(blas), xform.ctypes.data, blas_id.ctypes.data, inst_mat.ctypes.data,
        fl.ctypes.data if fl is not None else None, n,
        ctypes.byref(o), _ptr(buf), buf.numel(), _ptr(scratch), scratch.numel(), _stream(stream),
        ctypes.byref(d)))
    del torch
    return Tlas(buf, d, blas)


class PendingTlas:
    """A top-level build enqueued by build_tlas_async; finish() returns it."""

    def __init__(self, buf, blas, keep, ticket):
        self.buf = buf
        self.blas = list(blas)
        self._keep = keep
        self.ticket = ticket

    def finish(self) -> Tlas:
        d = TlasDesc()
        _check("rg_build_tlas_finish", _lib.rg_build_tlas_finish(self.ticket.data_ptr(), ctypes.byref(d)))
        self._keep = None
        return Tlas(self.buf, d, self.blas)


def build_tlas_async(blas: Sequence[Blas], xform, blas_id, inst_mat, width: int = 4, stream=None,
                     scratch=None, inst_flags=None, morton_bits: int = 0) -> PendingTlas:
    """build_tlas for the linear builder without the wait: the host tables go
    through a pinned ticket, the build is enqueued on `stream`, finish()
    waits for it."""
    torch = _torch()
    xform = np.ascontiguousarray(xform, np.float32).reshape(-1, 12)
    blas_id = np.ascontiguousarray(blas_id, np.uint32)
    inst_mat = np.ascontiguousarray(inst_mat, np.uint32)
    n = xform.shape[0]
    s = Sizes()
    o = _opts(width, 1, "lbvh", 0, morton_bits)
    _check("rg_tlas_sizes", _lib.rg_tlas_sizes(n, ctypes.byref(o), ctypes.byref(s)))
    dev = blas[0].buf.device
    buf = _bytes(s.bytes, dev)
    if scratch is None or scratch.numel() < s.scratch_bytes:
        scratch = _bytes(s.scratch_bytes, dev)
    fl = np.ascontiguousarray(inst_flags, np.uint32).reshape(n) if inst_flags is not None else None
    tb = ctypes.c_uint64()
    _check("rg_tlas_ticket_bytes", _lib.rg_tlas_ticket_bytes(n, len(blas), int(fl is not None), ctypes.byref(tb)))
    raw = torch.empty(tb.value + 256, dtype=torch.uint8, pin_memory=True)
    off = (-raw.data_ptr()) % 256
    ticket = raw[off: off + tb.value]
    arr = (BlasDesc * len(blas))(*[b.desc for b in blas])
    _check("rg_build_tlas_async", _lib.rg_build_tlas_async(
        arr, len(blas), xform.ctypes.data, blas_id.ctypes.data, inst_mat.ctypes.data,
        fl.ctypes.data if fl is not None else None, n, ctypes.byref(o), _ptr(buf), buf.numel(), _ptr(scratch),
        scratch.numel(), _stream(stream), ticket.data_ptr(), tb.value))
    return PendingTlas(buf, blas, (scratch, raw), ticket)


class TlasBuilder:
    """Rebuilds one top level over the same bottom levels, instance table and
    materials with new matrices, frame after frame, into one output buffer:
    the per-frame top-level update of a dynamic scene without a new buffer or
    new descriptor tables per call.  Every Tlas it returns shares that buffer,
    so the next build replaces the previous one (the caller orders it after
    the traces that still read it, e.g. on the same stream).  morton_bits:
    as for build_tlas (10: 30-bit keys, four sort passes, up to 2^20
    instances)."""

    def __init__(self, blas: Sequence[Blas], blas_id, inst_mat, width: int = 4, builder: str = "lbvh",
                 radius: int = 0, inst_flags=None, stream=None, morton_bits: int = 0):
        self.blas = list(blas)
        self.blas_id = np.ascontiguousarray(blas_id, np.uint32)
        self.inst_mat = np.ascontiguousarray(inst_mat, np.uint32)
        self.n = int(self.blas_id.shape[0])
        self.flags = np.ascontiguousarray(inst_flags, np.uint32).reshape(self.n) if inst_flags is not None else None
        self.opts = _opts(width, 1, builder, radius, morton_bits)
        s = Sizes()
        _check("rg_tlas_sizes", _lib.rg_tlas_sizes(self.n, ctypes.byref(self.opts), ctypes.byref(s)))
        dev = self.blas[0].buf.device
        self.buf = _bytes(s.bytes, dev)
        self.scratch = _bytes(s.scratch_bytes, dev)
        self.descs = (BlasDesc * len(self.blas))(*[b.desc for b in self.blas])
        self.stream = stream

    def build(self, xform) -> Tlas:
        """xform: host float32 [I,3,4] object->world."""
        xf = np.ascontiguousarray(xform, np.float32).reshape(-1, 12)
        if xf.shape[0] != self.n:
            raise ValueError(f"{xf.shape[0]} matrices for {self.n} instances")
        d = TlasDesc()
        _check("rg_build_tlas", _lib.rg_build_tlas_ex(
            self.descs, len(self.blas), xf.ctypes.data, self.blas_id.ctypes.data, self.inst_mat.ctypes.data,
            self.flags.ctypes.data if self.flags is not None else None, self.n, ctypes.byref(self.opts),
            _ptr(self.buf), self.buf.numel(), _ptr(self.scratch), self.scratch.numel(), _stream(self.stream),
            ctypes.byref(d)))
        return Tlas(self.buf, d, self.blas)


def upload_scene(scene, width: int = 4, leaf_max: int = 4, device="cuda", builder: str = "lbvh",
                 radius: int = 0, tlas_builder: Optional[str] = None, inst_flags=None) -> Tlas:
    """Builds every mesh and the instance level of a scene object with
    attributes blas (meshes with verts/idx/prim_mat), xform, blas_id, inst_mat.
    tlas_builder None: the instance level uses `builder` as well."""
    torch = _torch()
    built: List[Blas] = []
    for m in scene.blas:
        v = torch.from_numpy(np.ascontiguousarray(m.verts, np.float32)).to(device)
        i = torch.from_numpy(np.ascontiguousarray(m.idx, np.uint32).view(np.int32)).to(device)
        pm = None
        if m.prim_mat is not None:
            pm = torch.from_numpy(np.ascontiguousarray(m.prim_mat, np.uint16).view(np.int16)).to(device)
        built.append(build_blas(v, i, pm, width, leaf_max, builder=builder, radius=radius))
        del v, i, pm
    return build_tlas(built, scene.xform, scene.blas_id, scene.inst_mat, width,
                      builder=tlas_builder or builder, radius=radius, inst_flags=inst_flags)


# ------------------------------------------------------------------- rays
def rays_struct(r) -> Rays:
    """r: CUDA float32 [8, N] (ox oy oz dx dy dz tmin tmax rows); each row
    contiguous, rows may be strided (e.g. the first N columns of a larger
    buffer)."""
    if r.dim() != 2 or r.shape[0] != 8 or r.dtype != torch.float32:
        raise ValueError("rays must be float32 [8, N]")
    if not r.is_cuda or (r.shape[1] > 1 and r.stride(1) != 1):
        raise ValueError("rays must be a CUDA tensor with contiguous rows")
    base = r.data_ptr()
    s0 = r.stride(0)
    return Rays(*[base + 4 * s0 * k for k in range(8)])


def rays_to_device(rays_np, device="cuda"):
    """Host float32 [N,8] -> CUDA [8,N]."""
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(np.asarray(rays_np, np.float32).T)).to(device)


def alloc_hits(n: int, device="cuda"):
    torch = _torch()
    return dict(t=torch.empty(n, dtype=torch.float32, device=device),
                inst=torch.empty(n, dtype=torch.int32, device=device),
                prim=torch.empty(n, dtype=torch.int32, device=device),
                u=torch.empty(n, dtype=torch.float32, device=device),
                v=torch.empty(n, dtype=torch.float32, device=device))


def _hits_struct(h) -> Hits:
    """h: dict of CUDA tensors; a missing key skips that field (t, u, v need
    inst and prim)."""
    return Hits(_ptr(h.get("t")), _ptr(h.get("inst")), _ptr(h.get("prim")), _ptr(h.get("u")), _ptr(h.get("v")))


# ray visibility and facing (include/rg.h)
RAY_CULL_BACK, RAY_CULL_FRONT = 1, 2
INST_MASK_ALL, INST_CULL_DISABLE, INST_FLIP_FACING = 0xFF, 1 << 8, 1 << 9


def _opts_ref(cull: int, mask: int, ray_mask, n: int):
    if cull == 0 and mask == INST_MASK_ALL and ray_mask is None:
        return None
    if ray_mask is not None:
        torch = _torch()
        if ray_mask.dtype != torch.uint8 or not ray_mask.is_cuda or not ray_mask.is_contiguous() \
                or ray_mask.numel() < n:
            raise ValueError("ray_mask must be a contiguous CUDA uint8 tensor with one entry per ray")
    o = TraceOpts(cull, mask, _ptr(ray_mask) if ray_mask is not None else None)
    return ctypes.byref(o), o


def trace_closest(tlas: Tlas, rays, out=None, stream=None, cull: int = 0, mask: int = INST_MASK_ALL,
                  ray_mask=None):
    """cull: RAY_CULL_*; mask: visibility mask of every ray unless ray_mask
    (CUDA uint8 per ray) is given."""
    n = rays.shape[1]
    if out is None:
        out = alloc_hits(n, rays.device)
    o = _opts_ref(cull, mask, ray_mask, n)
    if o is None:
        _check("rg_trace_closest", _lib.rg_trace_closest(tlas.ref, rays_struct(rays), n, _hits_struct(out),
                                                         _stream(stream)))
    else:
        _check("rg_trace_closest_ex", _lib.rg_trace_closest_ex(tlas.ref, rays_struct(rays), n, _hits_struct(out),
                                                               o[0], _stream(stream)))
    return out


def trace_any(tlas: Tlas, rays, occluded=None, found=None, stream=None, cull: int = 0, mask: int = INST_MASK_ALL,
              ray_mask=None):
    torch = _torch()
    n = rays.shape[1]
    if occluded is None:
        occluded = torch.empty(n, dtype=torch.uint8, device=rays.device)
    fh = ctypes.byref(_hits_struct(found)) if found is not None else None
    o = _opts_ref(cull, mask, ray_mask, n)
    if o is None:
        _check("rg_trace_any", _lib.rg_trace_any(tlas.ref, rays_struct(rays), n, _ptr(occluded), fh,
                                                 _stream(stream)))
    else:
        _check("rg_trace_any_ex", _lib.rg_trace_any_ex(tlas.ref, rays_struct(rays), n, _ptr(occluded), fh, o[0],
                                                       _stream(stream)))
    return occluded


def trace_counts(tlas: Tlas, rays, any_hit: bool = False, counts=None, stream=None):
    torch = _torch()
    n = rays.shape[1]
    if counts is None:
        counts = torch.empty((n, 3), dtype=torch.int32, device=rays.device)
    _check("rg_trace_counts", _lib.rg_trace_counts(tlas.ref, rays_struct(rays), n, 1 if any_hit else 0,
                                                   _ptr(counts), _stream(stream)))
    return counts


TUNE_KEYS = ("refill", "waves_per_cu", "lds_depth", "leaf_batch", "inst_batch")
# families of calls with their own launch parameters (RG_TUNE_*)
TUNE_SCOPES = {"trace": 0, "frame": 1, "engine": 2}


def trace_tuning(refill: Optional[int] = None, waves_per_cu: Optional[int] = None,
                 lds_depth: Optional[int] = None, leaf_batch: Optional[int] = None,
                 inst_batch: Optional[int] = None, scope: str = "trace") -> dict:
    """Reads (and with arguments, sets) the traversal launch parameters of
    one family of calls: "trace" (trace_closest / trace_any / trace_counts),
    "frame" (render, Batch) or "engine" (Engine)."""
    sc = TUNE_SCOPES[scope]
    cur = TraceTune()
    _check("rg_trace_tuning", _lib.rg_trace_tuning(sc, None, ctypes.byref(cur)))
    args = dict(refill=refill, waves_per_cu=waves_per_cu, lds_depth=lds_depth, leaf_batch=leaf_batch,
                inst_batch=inst_batch)
    if any(v is not None for v in args.values()):
        new = TraceTune(*[getattr(cur, k) if args[k] is None else args[k] for k in TUNE_KEYS])
        _check("rg_trace_tuning", _lib.rg_trace_tuning(sc, ctypes.byref(new), ctypes.byref(cur)))
    return {k: int(getattr(cur, k)) for k in TUNE_KEYS}


def camera_desc(cam) -> CameraDesc:
    return CameraDesc((c_f * 3)(*cam.eye), (c_f * 3)(*cam.target), (c_f * 3)(*cam.up), cam.vfov_deg)


def light_desc(light) -> LightDesc:
    return LightDesc((c_f * 3)(*light.pos), (c_f * 3)(*light.intensity), light.ambient)


def camera_rays(cam, width: int, height: int, out=None, stream=None):
    torch = _torch()
    n = width * height
    if out is None:
        out = torch.empty((8, n), dtype=torch.float32, device="cuda")
    ptrs = (c_p * 8)(*[out.data_ptr() + 4 * n * k for k in range(8)])
    cd = camera_desc(cam)
    _check("rg_camera_rays", _lib.rg_camera_rays(ctypes.byref(cd), width, height, ptrs, _stream(stream)))
    return out


def ao_rays(tlas: Tlas, rays, hits, seed: int, tmax: float = 5.0, out=None, src=None, count=None,
            scratch=None, stream=None):
    """AO rays for every hit ray; returns (rays [8, 8N] (first `count` valid),
    src [8N], count tensor [1])."""
    torch = _torch()
    n = rays.shape[1]
    dev = rays.device
    if out is None:
        out = torch.empty((8, 8 * n), dtype=torch.float32, device=dev)
    if src is None:
        src = torch.empty(8 * n, dtype=torch.int32, device=dev)
    if count is None:
        count = torch.zeros(1, dtype=torch.int32, device=dev)
    need = ctypes.c_uint64()
    _check("rg_ao_rays_scratch", _lib.rg_ao_rays_scratch(n, ctypes.byref(need)))
    if scratch is None or scratch.numel() < need.value:
        scratch = _bytes(need.value, dev)
    cap = out.shape[1]
    ptrs = (c_p * 8)(*[out.data_ptr() + 4 * cap * k for k in range(8)])
    _check("rg_ao_rays", _lib.rg_ao_rays(tlas.ref, rays_struct(rays), n, _ptr(hits["inst"]), _ptr(hits["prim"]),
                                         _ptr(hits["t"]), seed, tmax, ptrs, _ptr(src), _ptr(count),
                                         _ptr(scratch), scratch.numel(), _stream(stream)))
    return out, src, count


def materials_array(mats) -> ctypes.Array:
    """Structured numpy (type, rgb[3], ior) -> rg_material[] (an
    rg_material[] passes through)."""
    if isinstance(mats, ctypes.Array):
        return mats
    arr = (Material * len(mats))()
    for i, m in enumerate(mats):
        arr[i].type = int(m["type"])
        for k in range(3):
            arr[i].rgb[k] = float(m["rgb"][k])
        arr[i].ior = float(m["ior"])
    return arr


def render_sizes(width: int, height: int, max_depth: int, mode: int) -> int:
    s = ctypes.c_uint64()
    _check("rg_render_sizes", _lib.rg_render_sizes(width, height, max_depth, mode, ctypes.byref(s)))
    return int(s.value)


class Renderer:
    """Owns the scratch buffer of rg_render for one image size / depth / mode."""

    def __init__(self, width: int, height: int, max_depth: int, mode: int = 0, device="cuda"):
        torch = _torch()
        self.width, self.height, self.max_depth, self.mode = width, height, max_depth, mode
        self.scratch = _bytes(render_sizes(width, height, max_depth, mode), device)
        self.image = torch.empty((height, width, 3), dtype=torch.float32, device=device)

    def render(self, tlas: Tlas, mats, camera, light, seed: int = 0, stats: bool = False, stream=None,
               primary_mat=None):
        """primary_mat: optional CUDA int32/uint32 [H, W] receiving the material
        each primary ray shaded (0xFFFFFFFF for the sky)."""
        ma = materials_array(mats)
        cd, ld = camera_desc(camera), light_desc(light)
        st = RenderStats()
        if primary_mat is not None:
            _need_image(primary_mat, self.height, self.width, 1, "primary_mat")
        _check("rg_render_ex", _lib.rg_render_ex(tlas.ref, ma, len(mats), ctypes.byref(cd), ctypes.byref(ld),
                                                 self.width, self.height, self.max_depth, self.mode, seed,
                                                 _ptr(self.image), _ptr(primary_mat), _ptr(self.scratch),
                                                 self.scratch.numel(), _stream(stream),
                                                 ctypes.byref(st) if stats else None))
        if stats:
            return self.image, dict(rays_traced=int(st.rays_traced), shadow_rays=int(st.shadow_rays),
                                    ms_total=float(st.ms_total))
        return self.image


def set_alpha(blas: Blas, masks, level: int = 3, stream=None) -> Blas:
    """Attaches opacity masks to a bottom level (rg_blas_set_alpha): masks is
    a CUDA int64 tensor with one 64-bit mask per input triangle (bit k: the
    k-th of the 4^level micro-triangles is opaque), or None to remove them.
    The bottom level keeps a reference to the tensor; top levels over it must
    be built again."""
    torch = _torch()
    if masks is not None:
        if masks.dtype not in (torch.int64,) + ((torch.uint64,) if hasattr(torch, "uint64") else ()) or \
                not masks.is_cuda or not masks.is_contiguous() or masks.numel() != blas.desc.n_tris:
            raise ValueError("masks must be a contiguous CUDA int64 tensor with one entry per triangle")
    _check("rg_blas_set_alpha", _lib.rg_blas_set_alpha(ctypes.byref(blas.desc), _ptr(masks), level,
                                                       _stream(stream)))
    blas.alpha = masks
    return blas


def _need_image(t, h: int, w: int, c: int, name: str):
    torch = _torch()
    want = (h, w, 3) if c == 3 else (h, w)
    ok_dtype = (torch.float32,) if c == 3 else (torch.int32, torch.uint32) if hasattr(torch, "uint32") \
        else (torch.int32,)
    if tuple(t.shape) != want or t.dtype not in ok_dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous CUDA tensor of shape {want} and dtype {ok_dtype}")


def post_sizes(width: int, height: int) -> int:
    s = ctypes.c_uint64()
    _check("rg_post_sizes", _lib.rg_post_sizes(width, height, ctypes.byref(s)))
    return int(s.value)


class Post:
    """The frame's post-process passes (rg_roughness_blur, rg_fxaa) with
    their scratch buffer for one image size."""

    def __init__(self, width: int, height: int, device="cuda"):
        self.width, self.height = width, height
        self.scratch = _bytes(post_sizes(width, height), device)

    def _out(self, image, out):
        torch = _torch()
        _need_image(image, self.height, self.width, 3, "image")
        if out is None:
            out = torch.empty_like(image)
        _need_image(out, self.height, self.width, 3, "out")
        return out

    def roughness_blur(self, image, primary_mat, roughness, radius: int = 8, out=None, stream=None):
        """roughness: CUDA float32 [n_mats]."""
        out = self._out(image, out)
        _need_image(primary_mat, self.height, self.width, 1, "primary_mat")
        _check("rg_roughness_blur", _lib.rg_roughness_blur(
            _ptr(image), _ptr(primary_mat), _ptr(roughness), roughness.numel(), self.width, self.height, radius,
            _ptr(out), _ptr(self.scratch), self.scratch.numel(), _stream(stream)))
        return out

    def fxaa(self, image, out=None, stream=None):
        out = self._out(image, out)
        _check("rg_fxaa", _lib.rg_fxaa(_ptr(image), self.width, self.height, _ptr(out), _ptr(self.scratch),
                                       self.scratch.numel(), _stream(stream)))
        return out


class Batch:
    """Many frames rendered together (rg_batch_*): `frames` is a list of
    (tlas, materials, camera, light, width, height, max_depth) tuples.  Owns
    the images and the scratch buffer; render() may be repeated, and is a
    pure launch sequence (capturable in a HIP graph)."""

    def __init__(self, frames, seed: int = 0, stream=None, device="cuda"):
        torch = _torch()
        self.frames = list(frames)
        n = len(self.frames)
        self.images = []
        self._mats = []
        jobs = (Job * n)()
        for k, (tl, mats, cam, light, W, H, D) in enumerate(self.frames):
            img = torch.empty((H, W, 3), dtype=torch.float32, device=device)
            self.images.append(img)
            ma = materials_array(mats)
            self._mats.append(ma)
            jobs[k] = Job(ctypes.addressof(tl.desc), ctypes.addressof(ma), len(mats), camera_desc(cam),
                          light_desc(light), W, H, D, 0, seed, img.data_ptr())
        need = ctypes.c_uint64()
        _check("rg_batch_sizes", _lib.rg_batch_sizes(jobs, n, ctypes.byref(need)))
        self.scratch = _bytes(need.value, device)
        self.desc = BatchDesc()
        _check("rg_batch_prepare", _lib.rg_batch_prepare(jobs, n, _ptr(self.scratch), self.scratch.numel(),
                                                         _stream(stream), ctypes.byref(self.desc)))

    def capture(self):
        """Captures one render() of the whole batch into a HIP graph
        (torch.cuda.CUDAGraph): graph.replay() re-renders every frame into
        the same images.  The batch is a launch sequence only (counters are
        cleared by kernels, nothing waits on the host), so it captures as is."""
        torch = _torch()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.render()             # warm-up outside the capture
        torch.cuda.current_stream().wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.render()
        return g

    def render(self, stats: bool = False, stream=None):
        st = RenderStats()
        _check("rg_batch_render", _lib.rg_batch_render(ctypes.byref(self.desc), _stream(stream),
                                                       ctypes.byref(st) if stats else None))
        if stats:
            return self.images, dict(rays_traced=int(st.rays_traced), shadow_rays=int(st.shadow_rays),
                                     ms_total=float(st.ms_total))
        return self.images


def render_capture(tlas: Tlas, mats, camera, light, width: int, height: int, max_depth: int, capacity: int,
                   seed: int = 0, stream=None):
    """rg_render_capture: renders a frame and keeps each pass's queues.
    Returns (image [H, W, 3], passes), passes[k] a dict of CPU numpy arrays:
    rays [m, 8] (the closest-hit rays as traced), t, inst, prim (their float32
    t and input-index hits), shadow [s, 8] and occluded [s], counts (queued
    closest-hit and shadow rays; m, s = min(count, capacity))."""
    torch = _torch()
    P = max_depth + 1
    dev = "cuda"
    rays = torch.empty((P, 8, capacity), dtype=torch.float32, device=dev)
    t = torch.empty((P, capacity), dtype=torch.float32, device=dev)
    inst = torch.empty((P, capacity), dtype=torch.int32, device=dev)
    prim = torch.empty((P, capacity), dtype=torch.int32, device=dev)
    srays = torch.empty((P, 8, capacity), dtype=torch.float32, device=dev)
    occ = torch.empty((P, capacity), dtype=torch.uint8, device=dev)
    counts = torch.zeros((P, 2), dtype=torch.int32, device=dev)
    image = torch.empty((height, width, 3), dtype=torch.float32, device=dev)
    scratch = _bytes(render_sizes(width, height, max_depth, 0), dev)
    cap = Capture(capacity, _ptr(rays), _ptr(t), _ptr(inst), _ptr(prim), _ptr(srays), _ptr(occ), _ptr(counts))
    ma = materials_array(mats)
    cd, ld = camera_desc(camera), light_desc(light)
    _check("rg_render_capture", _lib.rg_render_capture(tlas.ref, ma, len(mats), ctypes.byref(cd), ctypes.byref(ld),
                                                       width, height, max_depth, seed, _ptr(image), _ptr(scratch),
                                                       scratch.numel(), ctypes.byref(cap), _stream(stream)))
    torch.cuda.synchronize()
    cnt = counts.cpu().numpy().astype(np.int64)
    R, T, I, Pm, S, O = (x.cpu().numpy() for x in (rays, t, inst, prim, srays, occ))
    passes = []
    for k in range(P):
        m, sn = min(int(cnt[k, 0]), capacity), min(int(cnt[k, 1]), capacity)
        passes.append(dict(rays=R[k, :, :m].T.copy(), t=T[k, :m], inst=I[k, :m].view(np.uint32),
                           prim=Pm[k, :m].view(np.uint32), shadow=S[k, :, :sn].T.copy(), occluded=O[k, :sn],
                           counts=(int(cnt[k, 0]), int(cnt[k, 1]))))
    return image, passes


STATIC_SCRATCH_BYTES = 64 << 20  # RG_STATIC_SCRATCH_BYTES


def render_static(tlas: Tlas, mats, camera, light, width: int, height: int, max_depth: int, image,
                  mode: int = 0, seed: int = 0, stream=None):
    """rg_render_static: rg_render into a caller-owned image [H, W, 3] with the
    library's own device-resident scratch (no allocation; frames up to
    STATIC_SCRATCH_BYTES of render_sizes; calls on one GPU must not overlap)."""
    ma = materials_array(mats)
    cd, ld = camera_desc(camera), light_desc(light)
    _check("rg_render_static", _lib.rg_render_static(tlas.ref, ma, len(mats), ctypes.byref(cd), ctypes.byref(ld),
                                                     width, height, max_depth, mode, seed, _ptr(image),
                                                     _stream(stream)))
    return image


def render_into(tlas: Tlas, mats, camera, light, width: int, height: int, max_depth: int, image, scratch,
                mode: int = 0, seed: int = 0, stream=None):
    """rg_render into a caller-owned image [H, W, 3] with a caller-owned
    scratch buffer (at least render_sizes(...) bytes)."""
    ma = materials_array(mats)
    cd, ld = camera_desc(camera), light_desc(light)
    _check("rg_render", _lib.rg_render(tlas.ref, ma, len(mats), ctypes.byref(cd), ctypes.byref(ld), width, height,
                                       max_depth, mode, seed, _ptr(image), _ptr(scratch), scratch.numel(),
                                       _stream(stream), None))
    return image


def render(tlas: Tlas, mats, camera, light, width: int, height: int, max_depth: int, mode: int = 0,
           seed: int = 0, stream=None):
    r = Renderer(width, height, max_depth, mode)
    return r.render(tlas, mats, camera, light, seed, stream=stream).clone()


# ------------------------------------------------------------ serving
class Pool:
    """Admission accounting of the serving engine (rg_pool_*): host only."""

    def __init__(self, max_rays: int, max_pixels: int, max_jobs: int):
        self.h = c_p()
        _check("rg_pool_create", _lib.rg_pool_create(max_rays, max_pixels, max_jobs, ctypes.byref(self.h)))

    def reserve(self, rays: int, pixels: int):
        """(slot, pixel offset), or None when it does not fit now; raises
        RgError (RG_ERR_OUT_OF_MEMORY) when it never fits."""
        slot, off = c_i32(), c_i64()
        _check("rg_pool_reserve", _lib.rg_pool_reserve(self.h, rays, pixels, ctypes.byref(slot), ctypes.byref(off)))
        return None if slot.value < 0 else (slot.value, off.value)

    def release(self, slot: int):
        _check("rg_pool_release", _lib.rg_pool_release(self.h, slot))

    def usage(self) -> dict:
        u = PoolUsage()
        _check("rg_pool_get_usage", _lib.rg_pool_get_usage(self.h, ctypes.byref(u)))
        return dict(rays=u.rays, pixels=u.pixels, largest_free_pixels=u.largest_free_pixels, jobs=u.jobs)

    def close(self):
        if self.h:
            _lib.rg_pool_destroy(self.h)
            self.h = c_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def job_struct(tlas_desc_addr: int, mats, cam, light, width: int, height: int, max_depth: int,
               image_ptr: int = 0, mode: int = 0, seed: int = 0):
    """An rg_job; `mats` is a materials_array (kept alive by the caller)."""
    return Job(tlas_desc_addr, ctypes.addressof(mats), len(mats), camera_desc(cam), light_desc(light), width,
               height, max_depth, mode, seed, image_ptr)


def job_reservation(mats, width: int, height: int, max_depth: int):
    """(queue entries per pass at worst, pixels) of a frame (rg_job_reservation)."""
    ma = mats if isinstance(mats, ctypes.Array) else materials_array(mats)
    j = Job(None, ctypes.addressof(ma), len(ma), CameraDesc(), LightDesc(), width, height, max_depth, 0, 0, None)
    rays, pix = c_i64(), c_i64()
    _check("rg_job_reservation", _lib.rg_job_reservation(ctypes.byref(j), ctypes.byref(rays), ctypes.byref(pix)))
    return rays.value, pix.value


def engine_sizes(max_rays: int, max_pixels: int, max_jobs: int = 64, max_mats: int = 256, width: int = 4) -> int:
    d = EngineDesc(max_rays, max_pixels, max_jobs, max_mats, width, 0)
    need = c_u64()
    _check("rg_engine_sizes", _lib.rg_engine_sizes(ctypes.byref(d), ctypes.byref(need)))
    return int(need.value)


class Engine:
    """Continuous-batching renderer (rg_engine_*).  Owns its scratch buffer;
    frames are admitted with a tag and come back from poll() when complete.
    All work goes to one stream (the current one at construction)."""

    def __init__(self, max_rays: int, max_pixels: int, max_jobs: int = 64, max_mats: int = 256, width: int = 4,
                 stream=None, device="cuda"):
        torch = _torch()
        self.desc = EngineDesc(max_rays, max_pixels, max_jobs, max_mats, width, 0)
        self.scratch = _bytes(engine_sizes(max_rays, max_pixels, max_jobs, max_mats, width), device)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.h = c_p()
        _check("rg_engine_create", _lib.rg_engine_create(ctypes.byref(self.desc), _ptr(self.scratch),
                                                         self.scratch.numel(), _stream(self.stream),
                                                         ctypes.byref(self.h)))
        self._tags = (c_i64 * 4096)()
        # what the device reads or writes for each frame in flight (its top
        # level and the bottom levels behind it, its image), held by tag until
        # poll() returns the tag: the engine's side stream uses them after
        # admit() returns, where torch's caching allocator cannot see it
        self._held = {}

    @staticmethod
    def for_budget(budget_bytes: int, max_jobs: int = 64, max_mats: int = 256, width: int = 4) -> dict:
        """Largest max_rays (= max_pixels) whose engine fits budget_bytes."""
        unit = 1 << 20
        s1 = engine_sizes(unit, unit, max_jobs, max_mats, width)
        s2 = engine_sizes(2 * unit, 2 * unit, max_jobs, max_mats, width)
        per = (s2 - s1) / unit
        n = int(min((budget_bytes - (s1 - per * unit)) / per, 1 << 31))
        while n > 64 and engine_sizes(n, n, max_jobs, max_mats, width) > budget_bytes:
            n = int(n * 0.999)
        if n < 64:
            raise ValueError(f"a budget of {budget_bytes} bytes holds no engine")
        return dict(max_rays=n, max_pixels=n, max_jobs=max_jobs, max_mats=max_mats, width=width)

    def admit(self, tlas: Tlas, mats, cam, light, width: int, height: int, max_depth: int, image, tag: int) -> bool:
        ma = mats if isinstance(mats, ctypes.Array) else materials_array(mats)
        j = job_struct(ctypes.addressof(tlas.desc), ma, cam, light, width, height, max_depth, _ptr(image))
        ok = c_i32()
        _check("rg_engine_admit", _lib.rg_engine_admit(self.h, ctypes.byref(j), tag, ctypes.byref(ok)))
        if ok.value:
            self._held[int(tag)] = (tlas, image)
        return bool(ok.value)

    def step(self) -> bool:
        ran = c_i32()
        _check("rg_engine_step", _lib.rg_engine_step(self.h, ctypes.byref(ran)))
        return bool(ran.value)

    def poll(self, wait: bool = False) -> List[int]:
        n = c_i32()
        _check("rg_engine_poll", _lib.rg_engine_poll(self.h, 1 if wait else 0, self._tags, len(self._tags),
                                                     ctypes.byref(n)))
        done = [int(self._tags[i]) for i in range(n.value)]
        for t in done:
            self._held.pop(t, None)
        return done

    def info(self) -> dict:
        i = EngineInfo()
        _check("rg_engine_get_info", _lib.rg_engine_get_info(self.h, ctypes.byref(i)))
        return {k: int(getattr(i, k)) for k, _ in EngineInfo._fields_}

    def stats(self) -> dict:
        st = RenderStats()
        _check("rg_engine_stats", _lib.rg_engine_stats(self.h, ctypes.byref(st)))
        return dict(rays_traced=int(st.rays_traced), shadow_rays=int(st.shadow_rays))

    def close(self):
        if self.h:
            h, self.h = self.h, c_p()
            _check("rg_engine_destroy", _lib.rg_engine_destroy(h))   # waits for the stream
            self._held.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lbvh_stages(verts, idx, stream=None, builder: str = "lbvh", radius: int = 0, morton_bits: int = 0) -> dict:
    """Intermediate results of the bottom-level build (keys, ids, binary
    tree, boxes) for the given builder and key width."""
    torch = _torch()
    n = int(idx.shape[0])
    _, ns = blas_sizes(n, builder=builder, radius=radius, morton_bits=morton_bits)
    o = _opts(4, 4, builder, radius, morton_bits)
    scratch = _bytes(ns, verts.device)
    dev = verts.device
    keys = torch.empty(n, dtype=torch.int64, device=dev)
    ids = torch.empty(n, dtype=torch.int32, device=dev)
    left = torch.empty(max(n - 1, 1), dtype=torch.int32, device=dev)
    right = torch.empty(max(n - 1, 1), dtype=torch.int32, device=dev)
    boxes = torch.empty((2 * n - 1, 6), dtype=torch.float32, device=dev)
    _check("rg_lbvh_stages", _lib.rg_lbvh_stages(_ptr(verts), int(verts.shape[0]), _ptr(idx), n,
                                                 ctypes.byref(o), _ptr(keys),
                                                 _ptr(ids), _ptr(left), _ptr(right), _ptr(boxes),
                                                 _ptr(scratch), scratch.numel(), _stream(stream)))
    return dict(keys=keys, ids=ids, left=left[:n - 1], right=right[:n - 1], boxes=boxes)
