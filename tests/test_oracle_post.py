"""The post-process passes of the oracle (roughness blur, FXAA) pinned by
what fixes them independently of their code: a library Gaussian filter on an
impulse, identities and symmetries the definitions must keep, a straight edge
worked out by hand, and the purpose of anti-aliasing itself (it brings an
aliased edge closer to the edge's exact coverage)."""
import numpy as np
import pytest
from scipy import ndimage

import scenegen as sg
from oracle import post

MISS = post.MISS


def _flat(H, W, m=0):
    return np.full((H, W), m, np.uint32)


# ------------------------------------------------------------ roughness blur
def test_blur_identities():
    img, mat = sg.post_frame(64, 48, 1)
    for rough in (np.zeros(8), np.full(8, 1e-3)):                  # smooth, or below 1/256
        assert np.array_equal(post.roughness_blur(img, mat, rough, 6), img.astype(np.float64))
    sky = np.full_like(mat, MISS)
    assert np.array_equal(post.roughness_blur(img, sky, np.ones(8), 6), img.astype(np.float64))
    assert np.array_equal(post.roughness_blur(img, mat, np.ones(8), 0), img.astype(np.float64))
    # ids beyond the table are left as they are
    assert np.array_equal(post.roughness_blur(img, mat + 100, np.ones(8), 6), img.astype(np.float64))


@pytest.mark.parametrize("r,radius", [(1.0, 6), (0.55, 8), (0.3, 9)])
def test_blur_impulse_is_the_library_gaussian(r, radius):
    """One material, an impulse far from the borders: the two passes are the
    separable Gaussian of scipy.ndimage with sigma = r R / 3 truncated at R."""
    H, W = 41, 47
    img = np.zeros((H, W, 3))
    img[20, 23] = (1.0, 2.0, -3.0)
    out = post.roughness_blur(img, _flat(H, W, 2), np.array([0, 0, r]), radius)
    sigma = r * radius / 3.0
    for c in range(3):
        ref = ndimage.gaussian_filter(img[..., c], sigma, truncate=radius / sigma, mode="constant")
        assert np.allclose(out[..., c], ref, rtol=0, atol=1e-13)


def test_blur_constant_stays_constant_and_materials_do_not_bleed():
    rng = np.random.default_rng(3)
    H, W = 40, 52
    mat = np.where(np.arange(W)[None, :] < 23, 0, 1).astype(np.uint32).repeat(H, 0)
    mat[10:30, 30:40] = 2
    img = np.full((H, W, 3), 0.7)
    out = post.roughness_blur(img, mat, np.array([1.0, 0.6, 0.9]), 7)
    assert np.allclose(out, 0.7, atol=1e-15)
    # changing what material 1 and 2 show leaves material 0's pixels unchanged
    img2 = img.copy()
    img2[mat != 0] = rng.uniform(0, 5, ((mat != 0).sum(), 3))
    out2 = post.roughness_blur(img2, mat, np.array([1.0, 0.6, 0.9]), 7)
    assert np.array_equal(out2[mat == 0], out[mat == 0])


def test_blur_mirror_and_linearity():
    img, mat = sg.post_frame(60, 44, 2)
    rough = sg.roughness_table(8, 2)
    out = post.roughness_blur(img, mat, rough, 5)
    flip = post.roughness_blur(img[:, ::-1], mat[:, ::-1], rough, 5)
    assert np.allclose(flip[:, ::-1], out, atol=1e-12)
    out2 = post.roughness_blur(2.0 * img + 1.0, mat, rough, 5)
    assert np.allclose(out2, 2.0 * out + 1.0, atol=1e-12)


# ------------------------------------------------------------------- FXAA
def test_fxaa_leaves_flat_and_low_contrast_images():
    img = np.full((30, 40, 3), 0.4)
    assert np.array_equal(post.fxaa(img)["rgb"], img)
    rng = np.random.default_rng(4)
    noisy = 0.5 + 0.004 * rng.standard_normal((30, 40, 3))    # luma range far below 1/16
    r = post.fxaa(noisy)
    assert not r["active"].any() and np.array_equal(r["rgb"], noisy)


def test_fxaa_straight_edge_by_hand():
    """Black left of column 10, white from it: the two pixels beside the edge
    see an edge that never ends (the distances tie, the edge offset is 0),
    and a 3x3 low-pass a third of the way across: sub-pixel offset
    ((3 - 2/3)(1/3)^2)^2 * 3/4 = (7/27)^2 * 3/4 towards the other side."""
    H, W = 24, 20
    img = np.zeros((H, W, 3))
    img[:, 10:] = 1.0
    r = post.fxaa(img)
    f = (7.0 / 27.0) ** 2 * 0.75
    assert np.allclose(r["rgb"][:, 9], f, atol=1e-15)
    assert np.allclose(r["rgb"][:, 10], 1.0 - f, atol=1e-15)
    others = np.ones(W, bool)
    others[[9, 10]] = False
    assert np.array_equal(r["rgb"][:, others], img[:, others])
    assert r["tie"][:, [9, 10]].all()


def _halfplane(H, W, slope, off, ss=1):
    """Coverage of y > slope x + off per pixel with ss x ss samples."""
    k = (np.arange(ss) + 0.5) / ss
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    cov = np.zeros((H, W))
    for a in k:
        for b in k:
            cov += (yy + b) > slope * (xx + a) + off
    return cov / (ss * ss)


@pytest.mark.parametrize("slope,off", [(0.125, 10.3), (1.0 / 3.0, 4.7), (-0.2, 30.1), (3.0, -40.2), (0.6, 2.2)])
def test_fxaa_brings_aliased_edges_towards_coverage(slope, off):
    H, W = 48, 64
    alias = _halfplane(H, W, slope, off)
    cover = _halfplane(H, W, slope, off, ss=16)
    out = post.fxaa(np.repeat(alias[..., None], 3, axis=2))["rgb"][..., 0]
    e0 = np.sqrt(np.mean((alias - cover) ** 2))
    e1 = np.sqrt(np.mean((out - cover) ** 2))
    assert e1 < 0.8 * e0, (e0, e1)


def test_fxaa_symmetries():
    """Transposing or mirroring the image transposes or mirrors the result on
    every pixel where no decision is a tie or within float reach of one."""
    img, _ = sg.post_frame(72, 72, 6)
    img = img.astype(np.float64)
    r = post.fxaa(img)
    ok = ~(r["amb"] | r["tie"])
    for fwd, back in ((lambda a: a.transpose(1, 0, 2), lambda a: a.transpose(1, 0, 2)),
                      (lambda a: a[:, ::-1], lambda a: a[:, ::-1]), (lambda a: a[::-1], lambda a: a[::-1])):
        t = post.fxaa(fwd(img))
        okt = ok & back((~(t["amb"] | t["tie"]))[..., None])[..., 0]
        assert okt.mean() > 0.9
        assert np.allclose(back(t["rgb"])[okt], r["rgb"][okt], atol=1e-12)


def test_fxaa_blends_with_one_neighbour():
    img, _ = sg.post_frame(80, 50, 7)
    img = img.astype(np.float64)
    r = post.fxaa(img)
    f = r["offset"]
    assert f.min() >= 0.0 and f.max() <= 0.75
    adj = np.abs(r["nx"] - np.arange(80)[None, :]) + np.abs(r["ny"] - np.arange(50)[:, None])
    assert (adj[r["active"]] <= 1).all()
    expect = (1 - f)[..., None] * img + f[..., None] * img[r["ny"], r["nx"]]
    assert np.allclose(r["rgb"], expect, atol=1e-12)
    assert r["active"].mean() > 0.02 and r["amb"].mean() < 0.01


def test_fxaa_edge_end_by_hand():
    """A horizontal edge (black rows above, white below) that steps down one
    row at column 8.  White pixel (2, 4): the edge runs both ways from the
    point (2, 3.5); to the left it never ends (26.5 pixels of steps), to the
    right the bilinear luma at x = 8.5 falls to 0 after steps 1+1+1+1+1+1.5
    = 6.5, half a gradient away from the average 1/2; that end darkens away
    from the pixel's luma, so the edge offset is 1/2 - 6.5 / 33 towards the
    black pixel above (the sub-pixel offset, (7/27)^2 3/4, is smaller)."""
    H, W = 10, 40
    img = np.zeros((H, W, 3))
    img[4:, :8] = 1.0
    img[5:, 8:] = 1.0
    r = post.fxaa(img)
    off = 0.5 - 6.5 / 33.0
    assert r["active"][4, 2] and not r["amb"][4, 2] and not r["tie"][4, 2]
    assert r["offset"][4, 2] == pytest.approx(off, abs=1e-15)
    assert np.allclose(r["rgb"][4, 2], 1.0 - off, atol=1e-15)
    assert (r["nx"][4, 2], r["ny"][4, 2]) == (2, 3)


def test_primary_materials_by_hand():
    """Two quads side by side at z = 0 seen from z = 5 (vertical field of view
    90 degrees, so the image plane at z = 0 spans y in [-5, 5]): the left quad
    x in [-2, 0] has per-triangle materials 3 (lower triangle) and 4, the
    right one x in [0, 2] the instance material 1; pixels whose centre ray
    meets neither are sky."""
    import oracle
    from tests.helpers import scene_from_meshes
    left = sg.triangles_mesh([[(-2, -2, 0), (0, -2, 0), (0, 2, 0)], [(-2, -2, 0), (0, 2, 0), (-2, 2, 0)]])
    left.prim_mat = np.array([3, 4], np.uint16)
    right = sg.triangles_mesh([[(0, -2, 0), (2, -2, 0), (2, 2, 0)], [(0, -2, 0), (2, 2, 0), (0, 2, 0)]])
    mats = sg.materials([(sg.DIFFUSE, (0.5, 0.5, 0.5), 1.5)] * 5)
    W = H = 20
    sc = scene_from_meshes([left, right], inst_mat=[sg.PER_PRIM, 1], mats=mats, width=W, height=H,
                           camera=sg.Camera((0.0, 0.0, 5.0), (0.0, 0.0, 0.0), (0.0, 1.0, 0.0), 90.0))
    px = np.arange(W * H)
    r = oracle.Scene(sc).primary_materials(px)
    # pixel centre (i + 1/2, j + 1/2) -> world x = (i + 1/2 - 10) / 2, y = (10 - j - 1/2) / 2 at z = 0
    i, j = px % W, px // W
    x, y = (i + 0.5 - W / 2) / 2.0, (H / 2 - j - 0.5) / 2.0
    # the left quad's diagonal runs from (-2, -2) to (0, 2): below it (y < 2x + 2) is triangle 0
    want = np.where((np.abs(x) > 2) | (np.abs(y) > 2), sg.MISS,
                    np.where(x > 0, 1, np.where(y < 2 * x + 2, 3, 4))).astype(np.uint32)
    ok = r["amb"] == 0
    assert ok.mean() > 0.9
    assert np.array_equal(r["mat"][ok], want[ok])
    assert set(np.unique(want[ok])) == {1, 3, 4, sg.MISS}
