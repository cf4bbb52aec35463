"""The seeded synthetic inputs: sizes of the configurations and mesh
orientation (counter-clockwise seen from outside)."""
import numpy as np
import pytest

import scenegen as sg


def _signed_volume(m):
    V = m.verts.astype(np.float64)
    a, b, c = V[m.idx[:, 0]], V[m.idx[:, 1]], V[m.idx[:, 2]]
    return np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0


@pytest.mark.parametrize("level,tris,verts", [(0, 20, 12), (3, 1280, 642), (5, 20480, 10242)])
def test_icosphere_counts(level, tris, verts):
    m = sg.icosphere(level)
    assert m.idx.shape == (tris, 3) and m.verts.shape == (verts, 3)
    assert np.allclose(np.linalg.norm(m.verts, axis=1), 1.0, atol=1e-6)
    # closed and outward: volume positive and below the unit ball's
    vol = _signed_volume(m)
    assert 0 < vol < 4.0 / 3.0 * np.pi


def test_torus_and_grid():
    t = sg.torus(128, 128, 1.0, 0.3)
    assert t.idx.shape == (32768, 3) and t.verts.shape == (16384, 3)
    assert _signed_volume(t) == pytest.approx(2 * np.pi ** 2 * 1.0 * 0.3 ** 2, rel=2e-3)
    g = sg.grid(256, 256, 0.15, 4.0, 7)
    assert g.idx.shape == (131072, 3) and g.verts.shape == (66049, 3)
    V = g.verts.astype(np.float64)
    n = np.cross(V[g.idx[:, 1]] - V[g.idx[:, 0]], V[g.idx[:, 2]] - V[g.idx[:, 0]])
    assert (n[:, 1] > 0).all()
    assert np.abs(V[:, 1]).max() <= 0.15


def test_displaced_torus_outward():
    t = sg.torus(64, 64, 1.0, 0.35, 0.25 * 0.35, 6.0, 3000)
    assert t.idx.shape == (8192, 3)
    assert _signed_volume(t) > 0


def test_small_config():
    sc = sg.config_small()
    assert sc.unique_tris() == 1282 and sc.n_inst == 1
    assert (sc.blas[0].prim_mat[:1280] == 0).all() and (sc.blas[0].prim_mat[1280:] == 1).all()
    assert (sc.width, sc.height, sc.max_depth) == (256, 256, 1)


def test_two_level_config():
    sc = sg.config_two_level()
    assert sc.unique_tris() == 184320 and sc.n_inst == 64
    assert sc.instanced_tris() == 3891200
    assert len(sc.materials) == 64
    assert set(np.unique(sc.materials["type"])) <= {0, 1, 2}
    s = np.linalg.norm(sc.xform[:, :, :3], axis=1)  # column norms = scale
    assert (s > 0.49).all() and (s < 2.01).all()
    again = sg.config_two_level()
    assert np.array_equal(sc.xform, again.xform)


def test_incoherent_config_small_segments():
    sc = sg.config_incoherent(segments=20)
    assert sc.n_inst == 1024 and len(sc.blas) == 16
    assert sc.blas[0].n_tris == 800
    assert sc.mode == 1


def test_option_inputs():
    """Instance flags alternate between mask 0x01 and 0x03, every second
    mesh carries one 64-bit opacity mask per triangle with about 3 in 4
    bits set, and the same seed gives the same masks."""
    sc = sg.config_incoherent(segments=24)
    flags, alpha = sg.option_inputs(sc)
    assert flags.dtype == np.uint32 and flags.shape == (sc.xform.shape[0],)
    assert np.array_equal(flags[0::2], np.full_like(flags[0::2], 0x01))
    assert np.array_equal(flags[1::2], np.full_like(flags[1::2], 0x03))
    assert len(alpha) == len(sc.blas)
    bits = []
    for b, (a, m) in enumerate(zip(alpha, sc.blas)):
        if b % 2:
            assert a is None
            continue
        mask, level = a
        assert level == 3 and mask.dtype == np.uint64 and mask.shape == (m.n_tris,)
        bits.append(np.unpackbits(mask.view(np.uint8)).mean())
    assert abs(np.mean(bits) - 0.75) < 0.01
    again = sg.option_inputs(sc)[1]
    assert all((x is None and y is None) or np.array_equal(x[0], y[0]) for x, y in zip(alpha, again))
