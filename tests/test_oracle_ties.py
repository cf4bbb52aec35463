"""Pins of the oracle's tie set and ambiguity flag (paper section 1: the
closest-hit / any-hit / miss outcome of each ray, decided here by a float32
traversal whose answer the FP64 oracle must be able to judge).

The oracle marks a ray ambiguous (`amb`) where float32 cannot decide its
outcome: a crossing within the barycentric band beta of a triangle edge that
no neighbour covers, a hit within the t band delta of tmin or tmax, a second
surface within float32 reach of the hit, a grazing hit; a crossing near one
interior edge whose neighbour lies on the other side of the edge as seen along
the ray is covered (a watertight test hits one of the two), so both triangles
join the tie set and the ray stays decidable.

Three kinds of pin:
  * the bands against a float32 model of the traversal's arithmetic
    (tests/f32_model.py): they must contain every error float32 makes, and
    must not be so wide that they contain nothing (then the flag would hide
    real failures);
  * hand cases whose outcome follows from the geometry: a covered interior
    edge, a silhouette ridge, a boundary edge, a vertex, the ends of the
    interval, two stacked surfaces, a grazing ray;
  * planted mistakes: each is applied to a copy of the oracle's source, built
    and run through the pins, and at least one pin must fail.
"""
import os

import numpy as np
import pytest

import oracle
import scenegen as sg
from tests.f32_model import trace_tri
from tests.helpers import ray, scene_from_meshes

EPS32 = 2.0 ** -24


def _trace(mesh, rays, lib=None, any_hit=False, xform=None):
    sc = scene_from_meshes([mesh], xforms=xform)
    return oracle.Scene(sc, lib=lib).trace(np.asarray(rays, np.float32).reshape(-1, 8), any_hit=any_hit)


def _ties(res, i=0):
    return {(int(a), int(b)) for a, b in res["ties"][i, :res["nties"][i]]}


# ----------------------------------------------------------------- geometry
def square_mesh(x0=0.0):
    """Unit square in z = 0 split along its diagonal (0,0)-(1,1) into two
    triangles that share vertices 0 and 2: triangle 0 below the diagonal
    (x > y), triangle 1 above it."""
    V = np.array([[x0, 0, 0], [x0 + 1, 0, 0], [x0 + 1, 1, 0], [x0, 1, 0]], np.float32)
    return sg.Mesh(V, np.array([[0, 1, 2], [0, 2, 3]], np.uint32))


def fin_mesh():
    """A knife-edge ridge: two triangles sharing the edge (0,0,0)-(1,0,0)
    and hanging down from it, one leaning towards -y, one towards +y.  Seen
    along +y both lie below the ridge, on the same side of the shared edge:
    the ridge is a silhouette."""
    V = np.array([[0, 0, 0], [1, 0, 0], [0.5, -0.125, -1], [0.5, 0.125, -1]], np.float32)
    return sg.Mesh(V, np.array([[0, 1, 2], [1, 0, 3]], np.uint32))


def roof_mesh():
    """A roof: two triangles sharing the ridge (0,0,0)-(1,0,0), sloping down
    at 45 degrees towards -y (triangle 0) and +y (triangle 1).  Seen from
    above the ridge separates them: a shared interior edge."""
    V = np.array([[0, 0, 0], [1, 0, 0], [0.5, -1, -1], [0.5, 1, -1]], np.float32)
    return sg.Mesh(V, np.array([[0, 1, 2], [1, 0, 3]], np.uint32))


def single_mesh(x0=0.0):
    V = np.array([[x0, 0, 0], [x0 + 1, 0, 0], [x0, 1, 0]], np.float32)
    return sg.Mesh(V, np.array([[0, 1, 2]], np.uint32))


def stacked_mesh(x0, gap):
    """Two parallel unit right triangles, at z = 0 and z = -gap (no shared
    vertices)."""
    V = np.array([[x0, 0, 0], [x0 + 1, 0, 0], [x0, 1, 0],
                  [x0, 0, -gap], [x0 + 1, 0, -gap], [x0, 1, -gap]], np.float32)
    return sg.Mesh(V, np.array([[0, 1, 2], [3, 4, 5]], np.uint32))


DOWN = (0.0, 0.0, -1.0)


# ------------------------------------------------------------------ checks
# Each check takes the oracle library to run (None: the oracle itself) and
# asserts what the geometry fixes.  The tests below run them on the oracle;
# test_planted_mistakes runs them on planted copies.

def check_covered_interior_edge(lib=None):
    """A ray a few float32 ulps from the square's diagonal, inside triangle
    0: far inside the band beta (about 1e-6 here) of the shared edge, whose
    neighbour lies across it as seen along the ray.  Float32 may hit either
    triangle; both are correct: tie set {0, 1}, not ambiguous, for closest
    and any hit."""
    m = square_mesh()
    r = ray((0.5 + 2 ** -24, 0.5 - 2 ** -25, 1.0), DOWN)
    res = _trace(m, r, lib)
    assert res["hit"][0] == 1 and res["prim"][0] == 0 and res["amb"][0] == 0
    assert _ties(res) == {(0, 0), (0, 1)}
    assert res["t"][0] == pytest.approx(1.0, abs=1e-12)
    ra = _trace(m, r, lib, any_hit=True)
    assert ra["hit"][0] == 1 and ra["amb"][0] == 0


def check_interior_off_edge(lib=None):
    """The same triangle 3e-5 (about 26 beta) from the diagonal: decided,
    only triangle 0 in the tie set."""
    m = square_mesh()
    r = ray((0.5 + 2 ** -16, 0.5 - 2 ** -16, 1.0), DOWN)
    res = _trace(m, r, lib)
    assert res["hit"][0] == 1 and res["amb"][0] == 0
    assert _ties(res) == {(0, 0)}
    assert res["beta"][0] < (2 * 2 ** -16) / 10  # the crossing is well outside the band


def check_silhouette_ridge(lib=None):
    """A ray along +y passing 2^-30 below the fin's ridge: it crosses
    triangle 0 within beta of the shared edge, but the neighbour lies on
    the same side of that edge as seen along the ray, so a ray perturbed
    upwards misses both.  Ambiguous for closest and any hit."""
    m = fin_mesh()
    r = ray((0.5, -4.0, -2.0 ** -30), (0.0, 1.0, 0.0))
    res = _trace(m, r, lib)
    assert res["hit"][0] == 1 and res["amb"][0] == 1
    ra = _trace(m, r, lib, any_hit=True)
    assert ra["hit"][0] == 1 and ra["amb"][0] == 1


def check_fin_far_below_ridge(lib=None):
    """The same ray 1/8 below the ridge: a robust hit of triangle 0."""
    m = fin_mesh()
    r = ray((0.5, -4.0, -0.125), (0.0, 1.0, 0.0))
    res = _trace(m, r, lib)
    assert res["hit"][0] == 1 and res["prim"][0] == 0 and res["amb"][0] == 0
    assert _ties(res) == {(0, 0)}


def check_folded_edge(lib=None):
    """A ray straight down 2^-20 (about half of beta) on triangle 1's side of
    the roof's ridge.  The other face's plane is crossed 2 * 2^-20 higher up
    (45 degree slopes).  From 1 above the ridge that is 1.9e-6 of t: a
    covered crossing, both faces in the tie set.  From 0.1 above it is
    1.9e-5 of t, beyond 1e-5: float32 cannot tell which face is hit and the
    two t differ by more than the tolerance, so the ray is ambiguous."""
    m = roof_mesh()
    far = _trace(m, ray((0.5, 2 ** -20, 1.0), DOWN), lib)
    assert far["hit"][0] == 1 and far["prim"][0] == 1 and far["amb"][0] == 0
    assert _ties(far) == {(0, 0), (0, 1)}
    near = _trace(m, ray((0.5, 2 ** -20, 0.1), DOWN), lib)
    assert near["hit"][0] == 1 and near["prim"][0] == 1 and near["amb"][0] == 1
    assert _trace(m, ray((0.5, 2 ** -20, 0.1), DOWN), lib, any_hit=True)["amb"][0] == 0


def check_boundary_edge(lib=None):
    """A lone triangle: a crossing 2^-26 from its edge y = 0 has no neighbour
    to cover it (ambiguous, closest and any); 2^-12 from it is decided."""
    m = single_mesh()
    near = _trace(m, ray((0.5, 2 ** -26, 1.0), DOWN), lib)
    assert near["hit"][0] == 1 and near["amb"][0] == 1
    near_any = _trace(m, ray((0.5, 2 ** -26, 1.0), DOWN), lib, any_hit=True)
    assert near_any["amb"][0] == 1
    # just outside the edge: a miss in FP64, but within the band: ambiguous
    out = _trace(m, ray((0.5, -2 ** -26, 1.0), DOWN), lib)
    assert out["hit"][0] == 0 and out["amb"][0] == 1
    far = _trace(m, ray((0.5, 2 ** -12, 1.0), DOWN), lib)
    assert far["hit"][0] == 1 and far["amb"][0] == 0


def check_vertex(lib=None):
    """Near the square's corner (0,0), where the crossing is within beta of
    two edges at once: no single neighbour covers it, ambiguous."""
    m = square_mesh()
    res = _trace(m, ray((2 ** -27, 2 ** -28, 1.0), DOWN), lib)
    assert res["hit"][0] == 1 and res["amb"][0] == 1


def _far_case_delta(lib=None):
    """The t band of a hit at t = 1 on a unit triangle 1000 units from the
    origin: float32 coordinates there carry about 6e-5 of rounding each, so
    delta is about 2.4e-4, well above 1e-5 t."""
    res = _trace(single_mesh(1000.0), ray((1000.25, 0.25, 1.0), DOWN), lib)
    assert res["hit"][0] == 1 and res["amb"][0] == 0
    return float(res["delta"][0])


def check_tmax_band(lib=None):
    """tmax a tenth of delta past or short of the hit: float32 may place the
    hit on either side of tmax (ambiguous); ten deltas away: decided."""
    dl = _far_case_delta(lib)
    assert 1e-4 < dl < 1e-3
    m = single_mesh(1000.0)
    r = ray((1000.25, 0.25, 1.0), DOWN, 0.0, 1.0 + 0.1 * dl)
    assert _trace(m, r, lib)["amb"][0] == 1
    assert _trace(m, r, lib, any_hit=True)["amb"][0] == 1
    r = ray((1000.25, 0.25, 1.0), DOWN, 0.0, 1.0 + 10 * dl)
    res = _trace(m, r, lib)
    assert res["hit"][0] == 1 and res["amb"][0] == 0
    assert _trace(m, r, lib, any_hit=True)["amb"][0] == 0
    # just short of the hit: a miss in FP64 that float32 may turn into a hit
    r = ray((1000.25, 0.25, 1.0), DOWN, 0.0, 1.0 - 0.1 * dl)
    res = _trace(m, r, lib)
    assert res["hit"][0] == 0 and res["amb"][0] == 1
    r = ray((1000.25, 0.25, 1.0), DOWN, 0.0, 1.0 - 10 * dl)
    res = _trace(m, r, lib)
    assert res["hit"][0] == 0 and res["amb"][0] == 0


def check_tmin_band(lib=None):
    dl = _far_case_delta(lib)
    m = single_mesh(1000.0)
    r = ray((1000.25, 0.25, 1.0), DOWN, 1.0 - 0.1 * dl)
    assert _trace(m, r, lib)["amb"][0] == 1
    r = ray((1000.25, 0.25, 1.0), DOWN, 1.0 - 10 * dl)
    res = _trace(m, r, lib)
    assert res["hit"][0] == 1 and res["amb"][0] == 0


def check_second_surface(lib=None):
    """Two parallel triangles a gap apart along the ray.  A gap of a tenth of
    delta cannot be ordered in float32 (and is not a tie, being far above
    1e-6 t): ambiguous.  Ten deltas: decided, the upper one is the hit.
    A gap below 1e-6 t is a tie: both in the tie set."""
    dl = _far_case_delta(lib)
    r = ray((1000.25, 0.25, 1.0), DOWN)
    res = _trace(stacked_mesh(1000.0, 0.1 * dl), r, lib)
    assert res["hit"][0] == 1 and res["prim"][0] == 0 and res["amb"][0] == 1
    res = _trace(stacked_mesh(1000.0, 10 * dl), r, lib)
    assert res["hit"][0] == 1 and res["prim"][0] == 0 and res["amb"][0] == 0
    assert _ties(res) == {(0, 0)}
    res = _trace(stacked_mesh(1000.0, 2 ** -21), r, lib)
    assert res["hit"][0] == 1 and _ties(res) == {(0, 0), (0, 1)}
    # any hit does not care which surface is nearer
    assert _trace(stacked_mesh(1000.0, 0.1 * dl), r, lib, any_hit=True)["amb"][0] == 0


def check_grazing(lib=None):
    """A ray at cos = 5e-4 to the plane is ambiguous; at cos = 0.05 it is
    not (the crossing is far from the edges in both cases)."""
    m = single_mesh()
    for c, amb in ((5e-4, 1), (0.05, 0)):
        d = np.array([1.0, 0.0, -c])
        o = np.array([0.25, 0.25, 0.0]) - d * 4.0
        res = _trace(m, ray(o, d), lib)
        assert res["hit"][0] == 1 and res["amb"][0] == amb, (c, res["amb"][0])


HAND_CHECKS = [check_covered_interior_edge, check_interior_off_edge, check_silhouette_ridge, check_folded_edge,
               check_fin_far_below_ridge, check_boundary_edge, check_vertex, check_tmax_band, check_tmin_band,
               check_second_surface, check_grazing]


@pytest.mark.parametrize("check", HAND_CHECKS, ids=lambda f: f.__name__[6:])
def test_hand_case(check):
    check()


# ------------------------------------------------ bands vs float32 model
def _band_sample(n, seed, near, edge, inst):
    """n random (triangle, instance, ray) configurations, each ray aimed at a
    point of its triangle: triangles of size 1e-3..1 placed in [-3,3]^3,
    meshes whose box is the triangle's grown by 1e-3..3, random rotation,
    scale 0.5..2 and translation in [-20,20]^3 (or the identity), origins
    1..50 (far) or 1e-3..1e-1 (near, like secondary rays leaving a surface)
    from the aimed point, direction lengths 0.3..3; `edge` aims within
    1e-8..1e-4 (barycentric) of an edge, on either side."""
    rng = np.random.default_rng(seed)
    size = np.exp(rng.uniform(np.log(1e-3), 0.0, n))
    cen = rng.uniform(-3, 3, (n, 3))
    tri = (cen[:, None, :] + size[:, None, None] * rng.normal(size=(n, 3, 3))).astype(np.float32)
    grow = np.exp(rng.uniform(np.log(1e-3), np.log(3.0), n))[:, None]
    lo = (tri.min(1) - grow).astype(np.float32)
    hi = (tri.max(1) + grow).astype(np.float32)
    X = np.zeros((n, 3, 4))
    if inst:
        X[:, :, :3] = sg.quat_to_matrix(sg.uniform_quaternion(rng, n)) * rng.uniform(0.5, 2.0, n)[:, None, None]
        X[:, :, 3] = rng.uniform(-20, 20, (n, 3))
    else:
        X[:, :, :3] = np.eye(3)
    X = X.astype(np.float32)
    w = rng.dirichlet([1, 1, 1], n)
    if edge:
        k = rng.integers(0, 3, n)
        w[np.arange(n), k] = np.exp(rng.uniform(np.log(1e-8), np.log(1e-4), n)) * rng.choice([-1, 1], n)
        w /= w.sum(1, keepdims=True)
    p = np.einsum("nk,nkj->nj", w, tri.astype(np.float64))
    pw = np.einsum("nij,nj->ni", X[:, :, :3].astype(np.float64), p) + X[:, :, 3]
    dirs = rng.normal(size=(n, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    dist = np.exp(rng.uniform(np.log(1e-3), np.log(1e-1), n) if near else rng.uniform(0.0, np.log(50), n))
    o = (pw - dirs * dist[:, None]).astype(np.float32)
    d = (dirs * np.exp(rng.uniform(np.log(0.3), np.log(3), n))[:, None]).astype(np.float32)
    # each configuration is its own mesh: the triangle plus two zero-area
    # triangles at the box corners (never hit, they only set the box)
    meshes = [sg.Mesh(np.concatenate([tri[i], [lo[i]] * 3, [hi[i]] * 3]).astype(np.float32),
                      np.arange(9, dtype=np.uint32).reshape(3, 3)) for i in range(n)]
    rays = np.zeros((n, 8), np.float32)
    rays[:, :3], rays[:, 3:6], rays[:, 7] = o, d, np.inf
    return dict(scene=scene_from_meshes(meshes, xforms=X), rays=rays,
                model=trace_tri(X, lo, hi, o, d, rays[:, 6], rays[:, 7], tri))


@pytest.fixture(scope="module")
def band_samples():
    out = []
    for k, (near, edge, inst) in enumerate([(False, False, True), (True, False, True), (False, True, True),
                                            (True, True, True), (True, False, False)]):
        out.append(_band_sample(600, 100 + k, near, edge, inst))
    return out


def band_ratios(samples, lib=None):
    """Largest float32 error over band, for t (delta) and for u, v (beta),
    and the number of inside/outside decisions float32 takes differently
    from FP64 although the crossing lies outside the band beta."""
    rt, ru, wrong = 0.0, 0.0, 0
    for s in samples:
        n = s["rays"].shape[0]
        ev = oracle.Scene(s["scene"], lib=lib).eval_hits(s["rays"], np.arange(n), np.zeros(n))
        m = s["model"]
        ok = np.isfinite(ev["t"])
        et = np.abs(m["t"].astype(np.float64) - ev["t"])
        euv = np.maximum(np.abs(m["u"] - ev["u"]), np.abs(m["v"] - ev["v"]))
        rt = max(rt, float(np.max(et[ok] / ev["delta"][ok])))
        ru = max(ru, float(np.max(euv[ok] / ev["beta"][ok])))
        dec = ok & (np.abs(ev["m"]) > ev["beta"])
        wrong += int((dec & (m["hit"] != (ev["m"] >= 0))).sum())
    return rt, ru, wrong


# the bands must hold every float32 error, and the largest error must use a
# visible share of them (measured: 0.31 of delta, 0.11 of beta)
T_FLOOR, UV_FLOOR = 0.05, 0.03


def check_bands(samples, lib=None):
    rt, ru, wrong = band_ratios(samples, lib)
    assert rt <= 1.0, f"float32 t error exceeds delta ({rt:.3g} of it)"
    assert ru <= 1.0, f"float32 barycentric error exceeds beta ({ru:.3g} of it)"
    assert wrong == 0, f"{wrong} float32 inside/outside decisions differ outside the band"
    assert rt >= T_FLOOR, f"delta is vacuous: float32 uses at most {rt:.3g} of it"
    assert ru >= UV_FLOOR, f"beta is vacuous: float32 uses at most {ru:.3g} of it"


def test_bands_contain_float32_error(band_samples):
    rt, ru, wrong = band_ratios(band_samples)
    assert rt <= 1.0 and ru <= 1.0 and wrong == 0, (rt, ru, wrong)


def test_bands_are_not_vacuous(band_samples):
    check_bands(band_samples)


def test_float32_t_error_exceeds_1e5_near_surfaces(band_samples):
    """Why the reported t is not float32's: for rays leaving a surface the
    float32 t is off by far more than 1e-5 t (the library recomputes the
    reported hit in double)."""
    s = band_samples[1]
    n = s["rays"].shape[0]
    ev = oracle.Scene(s["scene"]).eval_hits(s["rays"], np.arange(n), np.zeros(n))
    ok = np.isfinite(ev["t"])
    rel = np.abs(s["model"]["t"].astype(np.float64) - ev["t"])[ok] / ev["t"][ok]
    assert rel.max() > 1e-4


# -------------------------------------------------------- planted mistakes
# (name, text in rg_oracle.c, replacement): each must occur exactly once
MUTATIONS = [
    ("silhouette test dropped",
     "    if (!(v_dot(cj, F->d) * v_dot(ckx, F->d) < 0.0)) return -1;\n", "\n"),
    ("delta x 100",
     "    e->delta = pos_err * nlen / Sabs + OR_K * OR_EPS32 * fabs(e->t);",
     "    e->delta = 100.0 * (pos_err * nlen / Sabs + OR_K * OR_EPS32 * fabs(e->t));"),
    ("delta / 100",
     "    e->delta = pos_err * nlen / Sabs + OR_K * OR_EPS32 * fabs(e->t);",
     "    e->delta = 0.01 * (pos_err * nlen / Sabs + OR_K * OR_EPS32 * fabs(e->t));"),
    ("beta x 100", "    e->beta = pos_err * P * F->dl / Sabs;", "    e->beta = 100.0 * pos_err * P * F->dl / Sabs;"),
    ("beta / 100", "    e->beta = pos_err * P * F->dl / Sabs;", "    e->beta = 0.01 * pos_err * P * F->dl / Sabs;"),
    ("K x 16", "#define OR_K 4.0", "#define OR_K 64.0"),
    ("neighbour slot swapped", "    int sk = B->nslot[3 * j + near];", "    int sk = (B->nslot[3 * j + near] + 1) % 3;"),
    ("second-surface rule dropped", "                    res->amb = 1; /* a second surface within float32 reach of t*, not a tie */",
     "                    ; /* dropped */"),
    ("tmax band dropped",
     "                if (m >= -beta && fin_tmax && fabs(t - R->tmax) <= tmax_band &&\n"
     "                    (!res->hit || t <= tlim * (1.0 + 1e-5) + delta))\n"
     "                    res->amb = 1;",
     "                ;"),
    ("grazing flag dropped", "                    if (e.cosg < 1e-3) res->amb = 1;", "                    ;"),
    ("covered pair t tolerance widened to delta", "                    double ttol = res->hit ? 1e-5 * res->t : 0.0;",
     "                    double ttol = res->hit ? fmax(1e-5 * res->t, 100.0 * e.delta) : 0.0;"),
]


def _fails(fn, *a):
    try:
        fn(*a)
    except AssertionError:
        return True
    return False


@pytest.mark.parametrize("mut", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistakes(mut, tmp_path, band_samples):
    name, old, new = mut
    src = oracle.source()
    assert src.count(old) == 1, f"mutation '{name}' does not match the oracle's source"
    lib = oracle.build_variant(src.replace(old, new), os.path.join(str(tmp_path), "liboracle_variant.so"))
    caught = [f.__name__ for f in HAND_CHECKS if _fails(f, lib)]
    if _fails(check_bands, band_samples, lib):
        caught.append("check_bands")
    assert caught, f"planted mistake '{name}' passes every pin"
