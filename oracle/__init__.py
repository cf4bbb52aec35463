"""CPU oracle for the ray-tracing path -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the CPU-baseline leg of
`bench.py` may import this package.  The product library never does, and
this package never imports the product package; both read the seeded inputs
from `scenegen`.

Contents
  rg_oracle.c    FP64 brute force: closest / any hit with tie sets and
                 ambiguity flags, the Whitted recursion, ambient occlusion.
  exact.py       exact rational ray-triangle arithmetic (fractions.Fraction)
                 that pins the FP64 oracle on tiny inputs.
  build_ref.py   plain definitions of the build steps (Morton codes, stable
                 sort, Karras hierarchy, box refit) in NumPy.
  post.py        the frame's post-process passes (roughness blur, FXAA) in
                 FP64 NumPy, with per-pixel decision margins.

Ambient occlusion is not in the paper; it is the incoherent workload's
definition: for each primary hit, 8 cosine-weighted directions (Malley's
method) in the Duff et al. 2017 basis around the faced normal, uniforms from
SplitMix64 (Steele, Lea & Flood 2014), origin offset along the faced
normal, tmax 5; the pixel is 1 - occluded/8 (1 on a miss).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rg_oracle.c")
# RG_ORACLE_LIBRARY names another build of rg_oracle.c (the sanitizer build
# made by tests/run_sanitizers.py); build() leaves it alone
_LIB = os.environ.get("RG_ORACLE_LIBRARY") or os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

MISS = 0xFFFFFFFF
MAX_TIES = 16
# ray visibility / facing (rg_oracle.c)
RAY_CULL_BACK, RAY_CULL_FRONT = 1, 2
INST_CULL_DISABLE, INST_FLIP_FACING = 1 << 8, 1 << 9


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (plain -O2, no fast-math, no contraction)."""
    if os.environ.get("RG_ORACLE_LIBRARY"):
        return _LIB
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
               "-shared", "-fPIC", "-pthread", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            _lib = _bind(_LIB)
        return _lib


def build_variant(source: str, path: str):
    """Compiles C source text with the oracle's own flags into `path` and
    returns the loaded library.  For tests that plant a mistake in a copy of
    the oracle and check that a pin catches it; the oracle itself is not
    changed."""
    src = path + ".c"
    with open(src, "w") as fh:
        fh.write(source)
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
                           "-shared", "-fPIC", "-pthread", src, "-o", path, "-lm"])
    return _bind(path)


def source() -> str:
    with open(_SRC) as fh:
        return fh.read()


def _bind(path: str):
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    lib.or_scene_new.restype = P
    lib.or_scene_new.argtypes = [i32, P, P, P, P, P, i64, P, P, P]
    lib.or_scene_free.argtypes = [P]
    lib.or_set_sphere_reject.argtypes = [P, i32]
    lib.or_set_materials.argtypes = [P, P, i32]
    lib.or_trace.restype = i64
    lib.or_trace.argtypes = [P, P, i64, i32, i32, P, P, P, P, P, P, P, P, P, P, P, P, i32, P,
                             ctypes.c_uint32, ctypes.c_uint32]
    lib.or_set_inst_flags.argtypes = [P, P]
    lib.or_set_alpha.argtypes = [P, i32, P, i32]
    lib.or_camera_rays.argtypes = [P, i32, i32, P, i64, P]
    lib.or_ao_uniforms.argtypes = [u64, u64, P, P]
    lib.or_ao_direction.argtypes = [P, ctypes.c_double, ctypes.c_double, P]
    lib.or_ao_rays.argtypes = [P, P, i64, u64, i32, P, P, P]
    lib.or_render.restype = i64
    lib.or_render.argtypes = [P, P, P, i32, i32, i32, i32, u64, P, i64, i32, P, P, P]
    lib.or_primary_materials.argtypes = [P, P, i32, i32, P, i64, i32, P, P]
    lib.or_eval_hits.argtypes = [P, P, i64, P, P, P]
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def camera_array(cam) -> np.ndarray:
    return np.array(list(cam.eye) + list(cam.target) + list(cam.up) + [cam.vfov_deg], np.float32)


def light_array(light) -> np.ndarray:
    return np.array(list(light.pos) + list(light.intensity) + [light.ambient], np.float32)


class Scene:
    """FP64 oracle view of a `scenegen.Scene` (or of explicit arrays)."""

    def __init__(self, scene, sphere_reject: bool = False, inst_flags=None, alpha=None, lib=None):
        """inst_flags: uint32 per instance (bits 0-7 visibility mask,
        INST_CULL_DISABLE, INST_FLIP_FACING), default 0xFF.  alpha: per
        bottom level None or (uint64 mask per triangle, level 0..3): the
        opacity of the triangle's 4^level micro-triangles (see or_set_alpha).
        lib: a library from build_variant (default: the oracle)."""
        lib = _load() if lib is None else lib
        self._lib = lib
        self.scene = scene
        vo, to = [0], [0]
        for m in scene.blas:
            vo.append(vo[-1] + m.verts.shape[0])
            to.append(to[-1] + m.idx.shape[0])
        self._vo = np.array(vo, np.int64)
        self._to = np.array(to, np.int64)
        self._verts = np.ascontiguousarray(np.concatenate([m.verts for m in scene.blas]), np.float32)
        self._idx = np.ascontiguousarray(np.concatenate([m.idx for m in scene.blas]), np.uint32)
        pms = []
        for m in scene.blas:
            pms.append(m.prim_mat if m.prim_mat is not None else np.zeros(m.n_tris, np.uint16))
        self._pm = np.ascontiguousarray(np.concatenate(pms), np.uint16)
        self._xf = np.ascontiguousarray(scene.xform, np.float32)
        self._bid = np.ascontiguousarray(scene.blas_id, np.uint32)
        self._im = np.ascontiguousarray(scene.inst_mat, np.uint32)
        self.h = lib.or_scene_new(len(scene.blas), _ptr(self._vo), _ptr(self._to), _ptr(self._verts),
                                  _ptr(self._idx), _ptr(self._pm), self._xf.shape[0], _ptr(self._xf),
                                  _ptr(self._bid), _ptr(self._im))
        self._mats = np.ascontiguousarray(scene.materials)
        lib.or_set_materials(self.h, _ptr(self._mats), len(self._mats))
        lib.or_set_sphere_reject(self.h, 1 if sphere_reject else 0)
        if inst_flags is not None:
            self._flags = np.ascontiguousarray(inst_flags, np.uint32)
            assert self._flags.shape == (self._xf.shape[0],)
            lib.or_set_inst_flags(self.h, _ptr(self._flags))
        self._alpha = []
        for b, a in enumerate(alpha or []):
            if a is None:
                continue
            mask, level = np.ascontiguousarray(a[0], np.uint64), int(a[1])
            assert mask.shape == (scene.blas[b].n_tris,) and 0 <= level <= 3
            self._alpha.append(mask)
            lib.or_set_alpha(self.h, b, _ptr(mask), level)

    def set_sphere_reject(self, on: bool):
        self._lib.or_set_sphere_reject(self.h, 1 if on else 0)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self._lib.or_scene_free(h)
            self.h = None

    def trace(self, rays: np.ndarray, any_hit: bool = False, threads: int = 0, ray_mask=None, mask: int = 0xFF,
              cull: int = 0) -> dict:
        """rays f32[N,8].  Returns dict of per-ray arrays (t, u, v, inst,
        prim, hit, amb, beta, delta, nties, ties[N,16,2], ties_tuv[N,16,3], tests);
        beta / delta are the float32 error bands of the hit's barycentrics / t.
        ray_mask: uint8 per ray (else `mask` for every ray); cull: RAY_CULL_*."""
        rays = np.ascontiguousarray(rays, np.float32).reshape(-1, 8)
        n = rays.shape[0]
        out = dict(t=np.empty(n), u=np.empty(n), v=np.empty(n), beta=np.empty(n), delta=np.empty(n),
                   inst=np.empty(n, np.uint32), prim=np.empty(n, np.uint32),
                   hit=np.empty(n, np.uint8), amb=np.empty(n, np.uint8),
                   nties=np.empty(n, np.int32), ties=np.zeros((n, MAX_TIES, 2), np.uint32),
                   ties_tuv=np.zeros((n, MAX_TIES, 3)))
        rm = np.ascontiguousarray(ray_mask, np.uint8).reshape(n) if ray_mask is not None else None
        tests = self._lib.or_trace(self.h, _ptr(rays), n, 1 if any_hit else 0,
                                   threads or default_threads(),
                                   _ptr(out["t"]), _ptr(out["u"]), _ptr(out["v"]), _ptr(out["beta"]),
                                   _ptr(out["delta"]),
                                   _ptr(out["inst"]), _ptr(out["prim"]), _ptr(out["hit"]),
                                   _ptr(out["amb"]), _ptr(out["nties"]), _ptr(out["ties"]),
                                   _ptr(out["ties_tuv"]), MAX_TIES,
                                   _ptr(rm) if rm is not None else None, mask, cull)
        out["tests"] = int(tests)
        return out

    def eval_hits(self, rays: np.ndarray, inst, prim) -> dict:
        """The given triangle (inst[i], prim[i]) against ray i in FP64: t, u,
        v, m (least barycentric weight, >= 0 inside), beta, delta (its float32
        error bands); NaN where inst is MISS."""
        rays = np.ascontiguousarray(rays, np.float32).reshape(-1, 8)
        n = rays.shape[0]
        inst = np.ascontiguousarray(inst, np.uint32).reshape(n)
        prim = np.ascontiguousarray(prim, np.uint32).reshape(n)
        out = np.empty((n, 6))
        self._lib.or_eval_hits(self.h, _ptr(rays), n, _ptr(inst), _ptr(prim), _ptr(out))
        return dict(t=out[:, 0], u=out[:, 1], v=out[:, 2], m=out[:, 3], beta=out[:, 4], delta=out[:, 5])

    def ao_rays(self, rays: np.ndarray, seed: int, threads: int = 0) -> dict:
        """The 8 ambient-occlusion rays spawned at each input ray's closest hit:
        rays [n,8,6] (origin, direction; undefined where hit == 0), hit, amb."""
        rays = np.ascontiguousarray(rays, np.float32).reshape(-1, 8)
        n = rays.shape[0]
        out = np.zeros((n, 8, 6))
        hit = np.empty(n, np.uint8)
        amb = np.empty(n, np.uint8)
        self._lib.or_ao_rays(self.h, _ptr(rays), n, seed, threads or default_threads(), _ptr(out),
                             _ptr(hit), _ptr(amb))
        return dict(rays=out, hit=hit, amb=amb)

    def render(self, pixels=None, threads: int = 0, width=None, height=None, max_depth=None,
               mode=None, seed=None) -> dict:
        """Renders the listed pixels (all if None).  Returns rgb f64[n,3],
        amb u8[n], nrays i64[n], tests."""
        sc = self.scene
        W = sc.width if width is None else width
        H = sc.height if height is None else height
        D = sc.max_depth if max_depth is None else max_depth
        M = sc.mode if mode is None else mode
        S = sc.seed if seed is None else seed
        if pixels is None:
            pixels = np.arange(W * H, dtype=np.int64)
        pixels = np.ascontiguousarray(pixels, np.int64)
        n = pixels.shape[0]
        cam = camera_array(sc.camera)
        light = light_array(sc.light)
        rgb = np.empty((n, 3))
        amb = np.empty(n, np.uint8)
        nrays = np.empty(n, np.int64)
        tests = self._lib.or_render(self.h, _ptr(cam), _ptr(light), W, H, D, M, S, _ptr(pixels), n,
                                    threads or default_threads(), _ptr(rgb), _ptr(amb), _ptr(nrays))
        return dict(rgb=rgb, amb=amb, nrays=nrays, tests=int(tests))


    def primary_materials(self, pixels, width=None, height=None, threads: int = 0) -> dict:
        """The material index of each listed pixel's primary hit (MISS for the
        sky) and whether that hit is ambiguous."""
        sc = self.scene
        W = sc.width if width is None else width
        H = sc.height if height is None else height
        pixels = np.ascontiguousarray(pixels, np.int64)
        n = pixels.shape[0]
        mat = np.empty(n, np.uint32)
        amb = np.empty(n, np.uint8)
        self._lib.or_primary_materials(self.h, _ptr(camera_array(sc.camera)), W, H, _ptr(pixels), n,
                                       threads or default_threads(), _ptr(mat), _ptr(amb))
        return dict(mat=mat, amb=amb)


def camera_rays(camera, width: int, height: int, pixels) -> np.ndarray:
    """FP64 primary rays for the listed pixels: [n, 6] = origin, unit direction."""
    lib = _load()
    pixels = np.ascontiguousarray(pixels, np.int64)
    out = np.empty((pixels.shape[0], 6))
    cam = camera_array(camera)
    lib.or_camera_rays(_ptr(cam), width, height, _ptr(pixels), pixels.shape[0], _ptr(out))
    return out


def ao_uniforms(seed: int, key: int):
    lib = _load()
    a = np.empty(1)
    b = np.empty(1)
    lib.or_ao_uniforms(ctypes.c_uint64(seed), ctypes.c_uint64(key), _ptr(a), _ptr(b))
    return float(a[0]), float(b[0])


def ao_direction(n, u1: float, u2: float) -> np.ndarray:
    lib = _load()
    n = np.ascontiguousarray(n, np.float64)
    out = np.empty(3)
    lib.or_ao_direction(_ptr(n), u1, u2, _ptr(out))
    return out
