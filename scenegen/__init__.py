"""Seeded synthetic scenes: the only code shared by the oracle and the GPU path.

The paper renders COLLADA models through a two-level structure of triangle
meshes (bottom level) and instances with transformation matrices (top level),
section 1 (Introduction) and section 2.2 (Other Systems). Its assets are not
available, so every scene here is procedural and seeded.  This module only
produces inputs: vertex and index arrays, instance matrices, materials, a
camera and a light.  It holds none of the method's arithmetic (no ray, box or
shading computation).

All geometry is produced in float64 and stored as float32; both sides read the
same float32 arrays.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

MISS = 0xFFFFFFFF
PER_PRIM = 0xFFFFFFFF

DIFFUSE, MIRROR, GLASS = 0, 1, 2


# ----------------------------------------------------------------------------
# containers
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Mesh:
    verts: np.ndarray            # f32[V,3]
    idx: np.ndarray              # u32[T,3], counter-clockwise seen from outside
    prim_mat: Optional[np.ndarray] = None   # u16[T] or None

    @property
    def n_tris(self) -> int:
        return int(self.idx.shape[0])


@dataclasses.dataclass
class Camera:
    eye: tuple
    target: tuple
    up: tuple
    vfov_deg: float


@dataclasses.dataclass
class Light:
    pos: tuple
    intensity: tuple = (1.0, 1.0, 1.0)
    ambient: float = 0.1


@dataclasses.dataclass
class Scene:
    name: str
    blas: List[Mesh]
    xform: np.ndarray            # f32[I,3,4] object -> world
    blas_id: np.ndarray          # u32[I]
    inst_mat: np.ndarray         # u32[I]; PER_PRIM = use the mesh's prim_mat
    materials: np.ndarray        # structured: type i32, rgb f32[3], ior f32
    camera: Camera
    light: Light
    width: int
    height: int
    max_depth: int
    mode: int = 0                # 0 Whitted, 1 ambient occlusion
    seed: int = 0

    @property
    def n_inst(self) -> int:
        return int(self.xform.shape[0])

    def unique_tris(self) -> int:
        return sum(m.n_tris for m in self.blas)

    def instanced_tris(self) -> int:
        return int(sum(self.blas[b].n_tris for b in self.blas_id))


MATERIAL_DTYPE = np.dtype([("type", np.int32), ("rgb", np.float32, (3,)),
                           ("ior", np.float32)])


def materials(rows) -> np.ndarray:
    """rows: iterable of (type, (r,g,b), ior) -> structured array."""
    rows = list(rows)
    out = np.zeros(len(rows), dtype=MATERIAL_DTYPE)
    for i, (t, rgb, ior) in enumerate(rows):
        out[i]["type"] = t
        out[i]["rgb"] = rgb
        out[i]["ior"] = ior
    return out


# ----------------------------------------------------------------------------
# improved Perlin noise (Perlin 2002, "Improving Noise"), seeded permutation
# ----------------------------------------------------------------------------
def _fade(t):
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def _grad(h, x, y, z):
    h = h & 15
    u = np.where(h < 8, x, y)
    v = np.where(h < 4, y, np.where((h == 12) | (h == 14), x, z))
    return np.where((h & 1) == 0, u, -u) + np.where((h & 2) == 0, v, -v)


def perlin3(x, y, z, seed: int) -> np.ndarray:
    """One octave of improved noise at float64 points; range about [-1, 1]."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    p = rng.permutation(256).astype(np.int64)
    p = np.concatenate([p, p])
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    z = np.asarray(z, np.float64)
    fx, fy, fz = np.floor(x), np.floor(y), np.floor(z)
    X = fx.astype(np.int64) & 255
    Y = fy.astype(np.int64) & 255
    Z = fz.astype(np.int64) & 255
    x, y, z = x - fx, y - fy, z - fz
    u, v, w = _fade(x), _fade(y), _fade(z)
    A = p[X] + Y
    AA, AB = p[A] + Z, p[A + 1] + Z
    B = p[X + 1] + Y
    BA, BB = p[B] + Z, p[B + 1] + Z

    def lerp(t, a, b):
        return a + t * (b - a)

    return lerp(w,
                lerp(v, lerp(u, _grad(p[AA], x, y, z), _grad(p[BA], x - 1, y, z)),
                     lerp(u, _grad(p[AB], x, y - 1, z), _grad(p[BB], x - 1, y - 1, z))),
                lerp(v, lerp(u, _grad(p[AA + 1], x, y, z - 1), _grad(p[BA + 1], x - 1, y, z - 1)),
                     lerp(u, _grad(p[AB + 1], x, y - 1, z - 1),
                          _grad(p[BB + 1], x - 1, y - 1, z - 1))))


# ----------------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------------
def _orient_outward(verts64: np.ndarray, idx: np.ndarray, outward: np.ndarray) -> np.ndarray:
    """Flip every face whose winding normal disagrees with `outward` (per face)."""
    a, b, c = verts64[idx[:, 0]], verts64[idx[:, 1]], verts64[idx[:, 2]]
    n = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", n, outward) < 0
    idx = idx.copy()
    idx[flip, 1], idx[flip, 2] = idx[flip, 2].copy(), idx[flip, 1].copy()
    return idx


def icosphere(level: int, radius: float = 1.0) -> Mesh:
    """Icosahedron, `level` midpoint subdivisions, projected to the sphere.

    20*4**level triangles, 10*4**level+2 vertices, counter-clockwise outward.
    Each level splits every face (a, b, c) into (a, ab, ca), (b, bc, ab),
    (c, ca, bc), (ab, bc, ca); edge midpoints are shared between faces.
    """
    t = (1.0 + math.sqrt(5.0)) / 2.0
    V = np.array([(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
                  (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
                  (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)], np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = np.array([(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
                  (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
                  (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
                  (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)], np.int64)
    for _ in range(level):
        m = F.shape[0]
        E = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])   # ab, bc, ca
        E.sort(axis=1)
        uniq, inv = np.unique(E, axis=0, return_inverse=True)
        inv = inv.reshape(-1)
        mid = V[uniq[:, 0]] + V[uniq[:, 1]]
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        base = V.shape[0]
        V = np.concatenate([V, mid])
        ab, bc, ca = base + inv[:m], base + inv[m:2 * m], base + inv[2 * m:]
        a, b, c = F[:, 0], F[:, 1], F[:, 2]
        F = np.stack([np.stack([a, ab, ca], -1), np.stack([b, bc, ab], -1),
                      np.stack([c, ca, bc], -1), np.stack([ab, bc, ca], -1)], 1).reshape(-1, 3)
    V = V * radius
    cen = (V[F[:, 0]] + V[F[:, 1]] + V[F[:, 2]]) / 3.0
    F = _orient_outward(V, F, cen)
    return Mesh(V.astype(np.float32), F.astype(np.uint32))


def torus(m: int, n: int, R: float, r: float, disp_amp: float = 0.0,
          disp_freq: float = 0.0, disp_seed: int = 0) -> Mesh:
    """Torus in the xz-plane, m segments around the major circle, n around
    the tube: m*n vertices and 2*m*n triangles, counter-clockwise outward.
    Optional radial displacement along the tube normal by
    disp_amp * perlin3(disp_freq * p) evaluated at the undisplaced point p."""
    i = np.arange(m, dtype=np.float64)[:, None]
    j = np.arange(n, dtype=np.float64)[None, :]
    th = 2.0 * np.pi * i / m
    ph = 2.0 * np.pi * j / n
    nx = np.cos(ph) * np.cos(th)
    ny = np.sin(ph) * np.ones_like(th)
    nz = np.cos(ph) * np.sin(th)
    cx = R * np.cos(th) * np.ones_like(ph)
    cz = R * np.sin(th) * np.ones_like(ph)
    px, py, pz = cx + r * nx, r * ny, cz + r * nz
    if disp_amp != 0.0:
        h = disp_amp * perlin3(disp_freq * px, disp_freq * py, disp_freq * pz, disp_seed)
        px, py, pz = px + h * nx, py + h * ny, pz + h * nz
    V = np.stack([px, py, pz], axis=-1).reshape(-1, 3)
    ii, jj = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    i0, j0 = ii.ravel(), jj.ravel()
    i1, j1 = (i0 + 1) % m, (j0 + 1) % n
    q00, q10, q11, q01 = i0 * n + j0, i1 * n + j0, i1 * n + j1, i0 * n + j1
    F = np.empty((2 * m * n, 3), np.int64)
    F[0::2] = np.stack([q00, q01, q11], -1)
    F[1::2] = np.stack([q00, q11, q10], -1)
    # outward reference: tube normal at the face's (undisplaced) centre
    cen = (V[F[:, 0]] + V[F[:, 1]] + V[F[:, 2]]) / 3.0
    ring = cen.copy()
    ring[:, 1] = 0.0
    ring_n = np.linalg.norm(ring, axis=1, keepdims=True)
    out = cen - R * ring / np.maximum(ring_n, 1e-30)
    F = _orient_outward(V, F, out)
    return Mesh(V.astype(np.float32), F.astype(np.uint32))


def grid(m: int, n: int, amp: float = 0.0, freq: float = 0.0, seed: int = 0) -> Mesh:
    """Height field over [-1,1]^2 in the xz-plane, (m+1)*(n+1) vertices,
    2*m*n triangles, counter-clockwise seen from +y.  Height
    amp * perlin3(freq*x + 0.5, 0.5, freq*z + 0.5)."""
    x = -1.0 + 2.0 * np.arange(m + 1, dtype=np.float64) / m
    z = -1.0 + 2.0 * np.arange(n + 1, dtype=np.float64) / n
    X, Z = np.meshgrid(x, z, indexing="ij")
    Y = np.zeros_like(X)
    if amp != 0.0:
        Y = amp * perlin3(freq * X + 0.5, np.full_like(X, 0.5), freq * Z + 0.5, seed)
    V = np.stack([X, Y, Z], -1).reshape(-1, 3)
    ii, jj = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
    i0, j0 = ii.ravel(), jj.ravel()
    q00 = i0 * (n + 1) + j0
    q10 = (i0 + 1) * (n + 1) + j0
    q11 = (i0 + 1) * (n + 1) + j0 + 1
    q01 = i0 * (n + 1) + j0 + 1
    F = np.empty((2 * m * n, 3), np.int64)
    F[0::2] = np.stack([q00, q01, q11], -1)
    F[1::2] = np.stack([q00, q11, q10], -1)
    up = np.zeros((F.shape[0], 3))
    up[:, 1] = 1.0
    F = _orient_outward(V, F, up)
    return Mesh(V.astype(np.float32), F.astype(np.uint32))


GROUND_P0 = ((-8.0, -1.0, -8.0), (-8.0, -1.0, 8.0), (8.0, -1.0, 8.0))
GROUND_P1 = ((-8.0, -1.0, -8.0), (8.0, -1.0, 8.0), (8.0, -1.0, -8.0))


def merge(meshes: List[Mesh]) -> Mesh:
    verts, idx, pm = [], [], []
    off = 0
    for k, m in enumerate(meshes):
        verts.append(m.verts)
        idx.append(m.idx.astype(np.int64) + off)
        pm.append(m.prim_mat if m.prim_mat is not None
                  else np.full(m.n_tris, k, np.uint16))
        off += m.verts.shape[0]
    return Mesh(np.concatenate(verts).astype(np.float32),
                np.concatenate(idx).astype(np.uint32),
                np.concatenate(pm).astype(np.uint16))


def triangles_mesh(tris) -> Mesh:
    """Unshared triangles given as an array [T,3,3]."""
    tris = np.asarray(tris, np.float64).reshape(-1, 3, 3)
    V = tris.reshape(-1, 3)
    F = np.arange(V.shape[0]).reshape(-1, 3)
    return Mesh(V.astype(np.float32), F.astype(np.uint32))


def random_soup(n_tris: int, seed: int, extent: float = 1.0, size: float = 0.2) -> Mesh:
    """Random triangles: centres uniform in [-extent, extent]^3, vertices
    offset by up to `size`."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    c = rng.uniform(-extent, extent, (n_tris, 1, 3))
    d = rng.uniform(-size, size, (n_tris, 3, 3))
    return triangles_mesh(c + d)


# ----------------------------------------------------------------------------
# instances
# ----------------------------------------------------------------------------
def uniform_quaternion(rng, n: int) -> np.ndarray:
    """Shoemake's uniform random rotation quaternion (x, y, z, w)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    return np.stack([a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2),
                     b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)], -1)


def quat_to_matrix(q: np.ndarray) -> np.ndarray:
    x, y, z, w = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
    ], -2)


def random_instances(rng, n: int, scale=(0.5, 2.0), extent: float = 20.0) -> np.ndarray:
    """Object->world 3x4 matrices: uniform rotation, scale U[scale], position
    U[-extent, extent]^3."""
    R = quat_to_matrix(uniform_quaternion(rng, n))
    s = rng.uniform(scale[0], scale[1], n)
    p = rng.uniform(-extent, extent, (n, 3))
    X = np.zeros((n, 3, 4))
    X[:, :, :3] = R * s[:, None, None]
    X[:, :, 3] = p
    return X.astype(np.float32)


def identity_xform(n: int = 1) -> np.ndarray:
    X = np.zeros((n, 3, 4), np.float32)
    X[:, 0, 0] = X[:, 1, 1] = X[:, 2, 2] = 1.0
    return X


# ----------------------------------------------------------------------------
# animation (dynamic scenes): moving vertices and moving instances
# ----------------------------------------------------------------------------
def animate_mesh(mesh: Mesh, t: float, amp: float = 0.05, seed: int = 0) -> np.ndarray:
    """Vertex positions of `mesh` at time t: a travelling wave along a seeded
    direction, displacing each vertex by up to `amp` times the mesh's extent
    along a second seeded direction (same triangles, new positions)."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 77]))
    k = rng.normal(size=3)
    k /= np.linalg.norm(k)
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    v = mesh.verts.astype(np.float64)
    ext = float(np.max(v.max(axis=0) - v.min(axis=0)))
    phase = 2.0 * np.pi * (v @ k) / max(ext, 1e-9) + 2.0 * np.pi * t
    return (v + amp * ext * np.sin(phase)[:, None] * a[None, :]).astype(np.float32)


def animate_instances(xform: np.ndarray, t: float, seed: int = 0, spin: float = 0.5,
                      drift: float = 1.0) -> np.ndarray:
    """Instance matrices at time t: each instance turns about its own seeded
    axis by spin*t*2pi radians (applied before its own rotation and scale) and
    moves by drift*sin(2pi t + phase) along a seeded direction."""
    X = np.asarray(xform, np.float64).reshape(-1, 3, 4)
    n = X.shape[0]
    rng = np.random.default_rng(np.random.SeedSequence([seed, 78]))
    axis = rng.normal(size=(n, 3))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    dirn = rng.normal(size=(n, 3))
    dirn /= np.linalg.norm(dirn, axis=1, keepdims=True)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    ang = spin * t * 2.0 * np.pi
    q = np.concatenate([axis * np.sin(ang / 2.0), np.full((n, 1), np.cos(ang / 2.0))], axis=1)
    R = quat_to_matrix(q)
    out = np.empty_like(X)
    out[:, :, :3] = X[:, :, :3] @ R
    out[:, :, 3] = X[:, :, 3] + drift * np.sin(2.0 * np.pi * t + ph)[:, None] * dirn
    return out.astype(np.float32)


# ----------------------------------------------------------------------------
# configurations
# ----------------------------------------------------------------------------
def config_small(seed: int = 1) -> Scene:
    """Icosphere level 3 (1,280 tris, mirror 0.8) plus the two ground
    triangles at y=-1 (diffuse 0.8) in one mesh, one identity instance,
    256x256, mirror depth 1."""
    sph = icosphere(3)
    sph.prim_mat = np.zeros(sph.n_tris, np.uint16)
    ground = triangles_mesh([GROUND_P0, GROUND_P1])
    ground.prim_mat = np.ones(2, np.uint16)
    mesh = merge([sph, ground])
    mats = materials([(MIRROR, (0.8, 0.8, 0.8), 1.5), (DIFFUSE, (0.8, 0.8, 0.8), 1.5)])
    return Scene("small: icosphere L3 + ground, 1 instance, 256x256, D=1",
                 [mesh], identity_xform(1), np.zeros(1, np.uint32),
                 np.full(1, PER_PRIM, np.uint32), mats,
                 Camera((0.0, 1.0, 4.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0),
                 Light((4.0, 6.0, 3.0)), 256, 256, 1, 0, seed)


def _random_materials(rng, n: int) -> np.ndarray:
    rows = []
    kinds = rng.integers(0, 3, n)
    for k in kinds:
        if k == DIFFUSE:
            rows.append((DIFFUSE, tuple(rng.uniform(0.2, 0.9, 3)), 1.5))
        elif k == MIRROR:
            rows.append((MIRROR, (0.9, 0.9, 0.9), 1.5))
        else:
            rows.append((GLASS, (1.0, 1.0, 1.0), 1.5))
    return materials(rows)


C2_BLAS_CACHE = {}


def c2_meshes(seed: int = 2) -> List[Mesh]:
    key = seed
    if key not in C2_BLAS_CACHE:
        C2_BLAS_CACHE[key] = [icosphere(5), torus(128, 128, 1.0, 0.3),
                              grid(256, 256, 0.15, 4.0, seed * 1000 + 7)]
    return C2_BLAS_CACHE[key]


def config_two_level(seed: int = 2, width: int = 1920, height: int = 1080,
                     max_depth: int = 4) -> Scene:
    """64 instances over icosphere L5 / torus 128x128 / displaced grid
    256x256 (184,320 unique triangles), per-instance diffuse, mirror or glass
    material, 1920x1080, depth 4."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    meshes = c2_meshes(seed)
    n_inst = 64
    xf = random_instances(rng, n_inst)
    mats = _random_materials(rng, n_inst)
    return Scene(f"two-level: 64 instances of 3 meshes, {width}x{height}, D={max_depth}",
                 meshes, xf, (np.arange(n_inst) % 3).astype(np.uint32),
                 np.arange(n_inst, dtype=np.uint32), mats,
                 Camera((0.0, 0.0, 45.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0),
                 Light((30.0, 50.0, 40.0)), width, height, max_depth, 0, seed)


def c3_meshes(segments: int = 560) -> List[Mesh]:
    return [torus(segments, segments, 1.0, 0.35, 0.25 * 0.35, 6.0, 3000 + k)
            for k in range(16)]


def config_incoherent(seed: int = 3, segments: int = 560, width: int = 1920,
                      height: int = 1080, meshes: Optional[List[Mesh]] = None) -> Scene:
    """1,024 instances over 16 displaced tori of segments x segments
    (560 -> 627,200 tris each, 10,035,200 unique); ambient-occlusion mode,
    8 cosine rays per primary hit, tmax 5."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    if meshes is None:
        meshes = c3_meshes(segments)
    n_inst = 1024
    xf = random_instances(rng, n_inst)
    bid = rng.integers(0, 16, n_inst).astype(np.uint32)
    mats = materials([(DIFFUSE, (0.8, 0.8, 0.8), 1.5)])
    return Scene(f"incoherent: 1024 instances of 16 displaced tori {segments}x{segments}, "
                 f"{width}x{height}, AO 8 spp",
                 meshes, xf, bid, np.zeros(n_inst, np.uint32), mats,
                 Camera((0.0, 0.0, 45.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0),
                 Light((30.0, 50.0, 40.0)), width, height, 0, 1, seed)


def serving_c3_scene(seed: int, meshes: List[Mesh], width: int = 1920, height: int = 1080,
                     max_depth: int = 4) -> Scene:
    """A Whitted scene over the 16 displaced tori: 1,024 instances placed as
    in the incoherent configuration, each with one of 64 random diffuse /
    mirror / glass materials."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    n_inst = 1024
    xf = random_instances(rng, n_inst)
    bid = rng.integers(0, len(meshes), n_inst).astype(np.uint32)
    mats = _random_materials(rng, 64)
    return Scene(f"serving C3-type: 1024 instances of {len(meshes)} shared tori, Whitted",
                 meshes, xf, bid, (np.arange(n_inst) % 64).astype(np.uint32), mats,
                 Camera((0.0, 0.0, 45.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0),
                 Light((30.0, 50.0, 40.0)), width, height, max_depth, 0, seed)


def config_serving_pool(c3_segments: int = 560, n_c2: int = 32, n_c3: int = 32) -> List[Scene]:
    """The serving pool: n_c2 two-level scenes (seeds 5000...) with their own
    meshes, then n_c3 scenes (seeds 5100...) that share the 16 tori of
    c3_meshes(c3_segments) and differ in instances and materials."""
    pool = [config_two_level(seed=5000 + k) for k in range(n_c2)]
    if n_c3:
        shared = c3_meshes(c3_segments)
        pool += [serving_c3_scene(5100 + k, shared) for k in range(n_c3)]
    return pool


def _mesh_near(kind: int, tris: float, seed: int) -> Mesh:
    """A mesh of the given kind (0 icosphere, 1 torus, 2 displaced grid) at
    the resolution whose triangle count is nearest (in log) to `tris`."""
    tris = max(tris, 20.0)
    if kind == 0:
        level = int(np.clip(np.round(math.log(tris / 20.0, 4)), 0, 9))
        return icosphere(level)
    m = int(max(3, round(math.sqrt(tris / 2.0))))
    if kind == 1:
        return torus(m, m, 1.0, 0.3)
    return grid(m, m, 0.15, 4.0, seed)


def config_batched(seed: int = 4, n_scenes: int = 256, tri_range=(1e3, 2e6), max_inst: int = 128,
                   pix_range=(64 ** 2, 1024 ** 2), max_depth: int = 2) -> List[Scene]:
    """Independent scenes of uneven size: triangles log-uniform in tri_range,
    instances log-uniform in [1, max_inst] over min(instances, 4) meshes
    (icosphere / torus / displaced grid, the triangle budget split evenly),
    positions in [-c, c]^3 with c = 2 instances^(1/3), pixels log-uniform in
    pix_range (square images), per-instance materials as in the two-level
    scene, camera at (0, 0, 3c + 4) looking at the origin, depth 2."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    out = []
    for k in range(n_scenes):
        T = float(np.round(np.exp(rng.uniform(math.log(tri_range[0]), math.log(tri_range[1])))))
        I = int(np.round(np.exp(rng.uniform(0.0, math.log(max_inst)))))
        nb = min(I, 4)
        meshes = [_mesh_near(b % 3, T / nb, seed * 100000 + k * 10 + b) for b in range(nb)]
        c = 2.0 * I ** (1.0 / 3.0)
        xf = random_instances(rng, I, extent=c)
        mats = _random_materials(rng, I)
        P = float(np.exp(rng.uniform(math.log(pix_range[0]), math.log(pix_range[1]))))
        W = max(1, int(round(math.sqrt(P))))
        cam = Camera((0.0, 0.0, 3.0 * c + 4.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0)
        light = Light((c + 5.0, 2.0 * c + 10.0, c + 8.0))
        out.append(Scene(f"batched #{k}: {I} instances of {nb} meshes, {W}x{W}", meshes, xf,
                         (np.arange(I) % nb).astype(np.uint32), np.arange(I, dtype=np.uint32), mats,
                         cam, light, W, W, max_depth, 0, seed * 1000 + k))
    return out


# ----------------------------------------------------------------------------
# ray sets (inputs for trace tests that do not go through the camera)
# ----------------------------------------------------------------------------
def random_rays(n: int, seed: int, extent: float = 1.5, tmax: float = np.inf) -> np.ndarray:
    """f32[n,8] rays (ox,oy,oz,dx,dy,dz,tmin,tmax): origins uniform in the
    cube, directions uniform on the sphere, lengths U[0.5, 2]."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    o = rng.uniform(-extent, extent, (n, 3))
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    d *= rng.uniform(0.5, 2.0, (n, 1))
    r = np.zeros((n, 8), np.float32)
    r[:, 0:3] = o
    r[:, 3:6] = d
    r[:, 6] = 0.0
    r[:, 7] = tmax
    return r


def rays_through_points(targets: np.ndarray, seed: int, dist: float = 5.0) -> np.ndarray:
    """Rays that start `dist` away from each target point along a random
    direction and point at it (unit direction)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    n = targets.shape[0]
    d = rng.normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = np.zeros((n, 8), np.float32)
    r[:, 0:3] = targets + dist * d
    r[:, 3:6] = -d
    r[:, 7] = np.inf
    return r


def sample_pixels(width: int, height: int, n: int, seed: int) -> np.ndarray:
    """n distinct pixel indices (y*width + x), sorted, seeded."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    n = min(n, width * height)
    return np.sort(rng.choice(width * height, n, replace=False)).astype(np.int64)


# ----------------------------------------------------------------------------
# ray-option inputs: instance visibility flags and opacity masks
# ----------------------------------------------------------------------------
def option_inputs(scene: Scene, seed: int = 7, level: int = 3):
    """Instance flags and opacity masks for tracing `scene` with the ray
    options on: even-numbered instances carry visibility mask 0x01 only, the
    others 0x03 (so rays of mask 0x02 see half of them); every second mesh is
    alpha-tested at `level`, each of its triangles with a 64-bit mask whose
    bits are set with probability 3/4 (the OR of two uniform words).

    Returns (flags uint32[n_inst], alpha), alpha[b] = (uint64 mask per
    triangle, level) for the tested meshes and None for the others."""
    n_inst = scene.xform.shape[0]
    flags = np.where(np.arange(n_inst) % 2 == 0, 0x01, 0x03).astype(np.uint32)
    rng = np.random.default_rng(seed)
    alpha = []
    for b, m in enumerate(scene.blas):
        if b % 2:
            alpha.append(None)
            continue
        w = rng.integers(0, 2 ** 64, (m.idx.shape[0], 2), dtype=np.uint64)
        alpha.append((w[:, 0] | w[:, 1], level))
    return flags, alpha


# ----------------------------------------------------------------------------
# post-process inputs: a traced frame and its primary-hit materials
# ----------------------------------------------------------------------------
def roughness_table(n_mats: int, seed: int) -> np.ndarray:
    """Roughness per material in [0, 1]; about a quarter of the materials
    are perfectly smooth (0)."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.0, 1.0, n_mats)
    r[rng.random(n_mats) < 0.25] = 0.0
    return r.astype(np.float32)


def post_frame(width: int, height: int, seed: int, n_mats: int = 8, n_shapes: int = 40):
    """A frame as the tracer leaves it, drawn with one sample per pixel centre
    (so every edge is aliased): a sky gradient (material MISS) behind
    overlapping discs, triangles and half-planes, each of one material, with a
    smooth shading ramp, a checker texture on some and values up to 2.
    Returns image f32[H,W,3], primary material u32[H,W]."""
    rng = np.random.default_rng(seed)
    yy, xx = np.mgrid[0:height, 0:width].astype(np.float64) + 0.5
    u, v = xx / width, yy / height
    img = np.stack([1.0 - 0.5 * v, 1.0 - 0.3 * v, np.ones_like(v)], axis=-1)
    mat = np.full((height, width), MISS, np.uint32)
    scale = max(width, height)
    for _ in range(n_shapes):
        kind = rng.integers(0, 3)
        if kind == 0:
            c = rng.uniform(0, 1, 2) * np.array([width, height])
            rad = rng.uniform(0.02, 0.25) * scale
            inside = (xx - c[0]) ** 2 + (yy - c[1]) ** 2 <= rad * rad
        elif kind == 1:
            p = rng.uniform(-0.1, 1.1, (3, 2)) * np.array([width, height])
            d = [(p[(k + 1) % 3, 0] - p[k, 0]) * (yy - p[k, 1]) - (p[(k + 1) % 3, 1] - p[k, 1]) * (xx - p[k, 0])
                 for k in range(3)]
            inside = ((d[0] >= 0) & (d[1] >= 0) & (d[2] >= 0)) | ((d[0] <= 0) & (d[1] <= 0) & (d[2] <= 0))
        else:
            a = rng.uniform(0, 2 * np.pi)
            off = rng.uniform(0.2, 0.8, 2) * np.array([width, height])
            inside = (np.cos(a) * (xx - off[0]) + np.sin(a) * (yy - off[1])) > rng.uniform(0.1, 0.4) * scale
        m = rng.integers(0, n_mats)
        col = rng.uniform(0.0, 1.0, 3) * (2.0 if rng.random() < 0.2 else 1.0)
        ramp = 0.6 + 0.4 * np.cos(rng.uniform(2, 9) * u + rng.uniform(2, 9) * v + rng.uniform(0, 6))
        if rng.random() < 0.3:
            k = rng.integers(4, 24)
            ramp = ramp * np.where(((xx // k + yy // k) % 2) == 0, 1.0, 0.55)
        img[inside] = (ramp[..., None] * col)[inside]
        mat[inside] = m
    return img.astype(np.float32), mat
