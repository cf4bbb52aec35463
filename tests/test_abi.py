"""The C-ABI library: it loads, exports every function include/rg.h declares,
and its host-side argument validation rejects bad calls before any GPU work
(so these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rg.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rg_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("rg_build_blas", "rg_build_tlas", "rg_trace_closest", "rg_trace_any", "rg_render"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2001_09792_amd as rg
    lib = ctypes.CDLL(rg.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding covers the whole header
    assert set(_declared()) == set(rg.SIGNATURES)


def test_status_strings():
    import paper_2001_09792_amd as rg
    assert rg._lib.rg_status_string(0) == b"ok"
    assert rg._lib.rg_status_string(-1) == b"invalid argument"
    assert rg._lib.rg_status_string(-2) == b"buffer too small"


def test_sizes_validation():
    import paper_2001_09792_amd as rg
    nb, ns = rg.blas_sizes(1000)
    assert nb > 1000 * 40 and ns > 0
    for bad in (0, -1, 2 ** 28 + 1):
        with pytest.raises(rg.RgError):
            rg.blas_sizes(bad)
    with pytest.raises(rg.RgError):
        rg.blas_sizes(10, width=3)
    with pytest.raises(rg.RgError):
        rg.blas_sizes(10, leaf_max=9)
    # wider nodes are bigger
    assert rg.blas_sizes(10000, 8)[0] > rg.blas_sizes(10000, 2)[0]
    # builders: clustering needs more scratch, the same output; radius 1..32
    nb_p, ns_p = rg.blas_sizes(1000, builder="ploc")
    assert nb_p == nb and ns_p > ns
    for r in (1, 32):
        rg.blas_sizes(10, builder="ploc", radius=r)
    for r in (-1, 33):
        with pytest.raises(rg.RgError):
            rg.blas_sizes(10, builder="ploc", radius=r)
    o = rg.BuildOpts(4, 4, 3, 0)  # no such builder
    s = rg.Sizes()
    assert rg._lib.rg_blas_sizes(10, rg.ctypes.byref(o), rg.ctypes.byref(s)) == -1
    with pytest.raises(ValueError):
        rg.blas_sizes(10, builder="sah")


def test_render_sizes_validation():
    import paper_2001_09792_amd as rg
    s1 = rg.render_sizes(64, 64, 1, 0)
    s2 = rg.render_sizes(64, 64, 2, 0)
    assert s2 > s1 > 0
    assert rg.render_sizes(64, 64, 0, 1) > 0
    for args in ((0, 64, 1, 0), (64, 64, 9, 0), (64, 64, -1, 0), (64, 64, 1, 2)):
        with pytest.raises(rg.RgError):
            rg.render_sizes(*args)


def test_null_pointer_calls_are_rejected_on_the_host():
    import paper_2001_09792_amd as rg
    lib = rg._lib
    d = rg.BlasDesc()
    o = rg.BuildOpts(4, 4)
    # NULL vertices
    assert lib.rg_build_blas(None, 3, None, 1, None, ctypes.byref(o), None, 0, None, 0, None,
                             ctypes.byref(d)) == -1
    t = rg.TlasDesc()
    assert lib.rg_trace_closest(None, rg.Rays(), 1, rg.Hits(), None) == -1
    assert lib.rg_trace_any(ctypes.byref(t), rg.Rays(), 1, None, None, None) == -1
    assert lib.rg_trace_counts(None, rg.Rays(), 1, 0, None, None) == -1
    assert lib.rg_camera_rays(None, 4, 4, None, None) == -1
    assert lib.rg_render(None, None, 0, None, None, 4, 4, 1, 0, 0, None, None, 0, None, None) == -1
    # a top level over a singular matrix is rejected before any device work
    xf = (ctypes.c_float * 12)(*([0.0] * 12))
    bid = (ctypes.c_uint32 * 1)(0)
    im = (ctypes.c_uint32 * 1)(0)
    fake = rg.BlasDesc()
    fake.buf = 256
    fake.width = 4
    blas = (rg.BlasDesc * 1)(fake)
    assert lib.rg_build_tlas(blas, 1, xf, bid, im, 1, ctypes.byref(o), 256, 1 << 20, 256, 1 << 20, None,
                             ctypes.byref(t)) == -1
    # non-finite matrix entry
    vals = [1.0, 0, 0, 0, 0, 1.0, 0, 0, 0, 0, 1.0, float("nan")]
    xf2 = (ctypes.c_float * 12)(*vals)
    assert lib.rg_build_tlas(blas, 1, xf2, bid, im, 1, ctypes.byref(o), 256, 1 << 20, 256, 1 << 20, None,
                             ctypes.byref(t)) == -1
    # blas id out of range
    vals[11] = 0.0
    xf3 = (ctypes.c_float * 12)(*vals)
    bid2 = (ctypes.c_uint32 * 1)(1)
    assert lib.rg_build_tlas(blas, 1, xf3, bid2, im, 1, ctypes.byref(o), 256, 1 << 20, 256, 1 << 20, None,
                             ctypes.byref(t)) == -1
    # mixed widths
    fake.width = 8
    blas = (rg.BlasDesc * 1)(fake)
    assert lib.rg_build_tlas(blas, 1, xf3, bid, im, 1, ctypes.byref(o), 256, 1 << 20, 256, 1 << 20, None,
                             ctypes.byref(t)) == -1
    # refit: sizes from the descriptor, NULL arrays, another triangle count, short scratch
    fake.n_nodes, fake.n_tris = 100, 150
    need = ctypes.c_uint64()
    assert lib.rg_refit_sizes(ctypes.byref(fake), ctypes.byref(need)) == 0 and need.value >= 800
    assert lib.rg_refit_sizes(None, ctypes.byref(need)) == -1
    assert lib.rg_refit_blas(ctypes.byref(fake), None, 3, None, 150, None, 0, None) == -1
    assert lib.rg_refit_blas(ctypes.byref(fake), 256, 3, 256, 149, 256, 1 << 20, None) == -1
    assert lib.rg_refit_blas(ctypes.byref(fake), 256, 3, 256, 150, 256, 16, None) == -1   # depth 0
    fake.depth = 300      # deeper than the level table: needs scratch for the counters
    assert lib.rg_refit_blas(ctypes.byref(fake), 256, 3, 256, 150, 256, 16, None) == -2
    assert lib.rg_refit_blas(ctypes.byref(fake), 256, 3, 256, 150, None, 0, None) == -2
    other = rg.BlasDesc()
    other.buf, other.width, other.n_nodes, other.n_tris, other.depth = 256, 4, 10, 10, 3
    two = (rg.BlasDesc * 2)(fake, other)
    ptrs = (ctypes.c_void_p * 2)(256, 256)
    nv = (ctypes.c_int64 * 2)(3, 3)
    nt = (ctypes.c_int64 * 2)(150, 10)
    assert lib.rg_refit_blas_many(two, 2, ptrs, nv, ptrs, nt, None, 0, None) == -1    # mixed widths
    f3 = (ctypes.c_float * 3)()
    assert lib.rg_blas_state(None, f3, f3, ctypes.byref(need), None) == -1


def test_undersized_buffers_are_rejected():
    import paper_2001_09792_amd as rg
    lib = rg._lib
    d = rg.BlasDesc()
    o = rg.BuildOpts(4, 4)
    nb, ns = rg.blas_sizes(100)
    # pointers are never dereferenced because the size check fails first
    assert lib.rg_build_blas(256, 300, 256, 100, None, ctypes.byref(o), 256, nb - 1, 256, ns, None,
                             ctypes.byref(d)) == -2
    assert lib.rg_build_blas(256, 300, 256, 100, None, ctypes.byref(o), 256, nb, 256, ns - 1, None,
                             ctypes.byref(d)) == -2


def test_trace_tuning_scopes_host_only():
    """rg_trace_tuning keeps one launch-parameter set per family of calls and
    validates ranges (host state only, no GPU call)."""
    import pytest
    import paper_2001_09792_amd as rg
    saved = {s: rg.trace_tuning(scope=s) for s in rg.TUNE_SCOPES}
    try:
        assert saved["trace"]["leaf_batch"] == 12 and saved["trace"]["inst_batch"] == 6
        assert saved["frame"]["leaf_batch"] == 1 and saved["frame"]["inst_batch"] == 1
        rg.trace_tuning(refill=32, leaf_batch=4, scope="engine")
        assert rg.trace_tuning(scope="engine")["refill"] == 32
        assert rg.trace_tuning(scope="trace") == saved["trace"]      # other scopes untouched
        assert rg.trace_tuning(scope="frame") == saved["frame"]
        for bad in (dict(refill=0), dict(refill=65), dict(waves_per_cu=3), dict(lds_depth=7), dict(lds_depth=33),
                    dict(leaf_batch=0), dict(inst_batch=65)):
            with pytest.raises(rg.RgError):
                rg.trace_tuning(scope="trace", **bad)
        assert rg.trace_tuning(scope="trace") == saved["trace"]      # a rejected set changes nothing
        t = rg.TraceTune()
        assert rg._lib.rg_trace_tuning(3, None, ctypes.byref(t)) == -1  # unknown scope
    finally:
        for s, v in saved.items():
            rg.trace_tuning(scope=s, **v)


def test_trace_options_and_instance_flags_are_checked_on_the_host():
    """Unknown ray flags, a mask above 8 bits and unknown instance flag bits
    are rejected before any device work; valid options on zero rays are a
    no-op."""
    import paper_2001_09792_amd as rg
    lib = rg._lib
    t = rg.TlasDesc()
    t.buf, t.n_inst, t.width, t.depth = 256, 1, 4, 2
    for flags, mask, want in ((4, 0xFF, -1), (rg.RAY_CULL_BACK, 0x100, -1), (rg.RAY_CULL_FRONT, 0x0F, 0),
                              (rg.RAY_CULL_BACK | rg.RAY_CULL_FRONT, 0, 0)):
        o = rg.TraceOpts(flags, mask, None)
        assert lib.rg_trace_closest_ex(ctypes.byref(t), rg.Rays(), 0, rg.Hits(), ctypes.byref(o), None) == want
        assert lib.rg_trace_any_ex(ctypes.byref(t), rg.Rays(), 0, None, None, ctypes.byref(o), None) == want
    assert lib.rg_trace_closest_ex(None, rg.Rays(), 0, rg.Hits(), None, None) == -1
    xf = (ctypes.c_float * 12)(*[1.0, 0, 0, 0, 0, 1.0, 0, 0, 0, 0, 1.0, 0])
    bid = (ctypes.c_uint32 * 1)(0)
    im = (ctypes.c_uint32 * 1)(0)
    fl = (ctypes.c_uint32 * 1)(0xFF | (1 << 10))
    fake = rg.BlasDesc()
    fake.buf, fake.width = 256, 4
    blas = (rg.BlasDesc * 1)(fake)
    o = rg.BuildOpts(4, 4)
    assert lib.rg_build_tlas_ex(blas, 1, xf, bid, im, fl, 1, ctypes.byref(o), 256, 1 << 20, 256, 1 << 20, None,
                                ctypes.byref(t)) == -1


def test_post_process_arguments_are_checked_on_the_host():
    import paper_2001_09792_amd as rg
    lib = rg._lib
    need = ctypes.c_uint64()
    assert lib.rg_post_sizes(1920, 1080, ctypes.byref(need)) == 0 and need.value >= 16 * 1920 * 1080
    assert lib.rg_post_sizes(0, 10, ctypes.byref(need)) == -1
    assert lib.rg_post_sizes(1 << 16, 1 << 15, ctypes.byref(need)) == -1      # above 2^30 pixels
    lib.rg_post_sizes(64, 32, ctypes.byref(need))
    n = 64 * 32
    a, b, m, r, s = 1 << 20, 1 << 24, 1 << 26, 1 << 27, 1 << 28        # disjoint fake device addresses
    big = need.value
    assert lib.rg_roughness_blur(None, m, r, 4, 64, 32, 8, b, s, big, None) == -1
    assert lib.rg_roughness_blur(a, m, r, 0, 64, 32, 8, b, s, big, None) == -1            # no materials
    assert lib.rg_roughness_blur(a, m, r, 4, 64, 32, rg.RG_BLUR_RADIUS_MAX + 1, b, s, big, None) == -1
    assert lib.rg_roughness_blur(a, m, r, 4, 64, 32, -1, b, s, big, None) == -1
    assert lib.rg_roughness_blur(a, m, r, 4, 64, 32, 8, b, s, big - 1, None) == -2      # short scratch
    assert lib.rg_roughness_blur(a, m, r, 4, 64, 32, 8, a + 12 * n - 4, s, big, None) == -1   # in / out overlap
    assert lib.rg_roughness_blur(a, m, r, 4, 64, 32, 8, b, a + 8, big, None) == -1       # scratch over the input
    assert lib.rg_fxaa(a, 64, 32, a, s, big, None) == -1
    assert lib.rg_fxaa(a, 64, 32, b, s, 100, None) == -2
    assert lib.rg_fxaa(a, 64, 0, b, s, big, None) == -1
    assert lib.rg_fxaa(a, 64, 32, b, b - 12 * n + 256, big, None) == -1                 # luma scratch over the output


def test_opacity_mask_arguments_are_checked_on_the_host():
    import paper_2001_09792_amd as rg
    lib = rg._lib
    fake = rg.BlasDesc()
    assert lib.rg_blas_set_alpha(None, 256, 3, None) == -1
    assert lib.rg_blas_set_alpha(ctypes.byref(fake), 256, 3, None) == -1            # no buffer
    fake.buf = 256
    assert lib.rg_blas_set_alpha(ctypes.byref(fake), 512, rg.RG_ALPHA_LEVEL_MAX + 1, None) == -1
    assert lib.rg_blas_set_alpha(ctypes.byref(fake), 512, -1, None) == -1
    assert ctypes.sizeof(rg.BlasDesc) == 120


def test_treelet_builder_options():
    import paper_2001_09792_amd as rg
    lib = rg._lib
    s = rg.Sizes()
    for radius, want in ((0, 0), (1, 0), (8, 0), (9, -1), (-1, -1)):
        o = rg.BuildOpts(4, 4, 2, radius)
        assert lib.rg_blas_sizes(1000, ctypes.byref(o), ctypes.byref(s)) == want, radius
    o = rg.BuildOpts(4, 4, 3, 0)
    assert lib.rg_blas_sizes(1000, ctypes.byref(o), ctypes.byref(s)) == -1       # unknown builder
    lbvh, tr = rg.blas_sizes(5000, builder="lbvh"), rg.blas_sizes(5000, builder="treelet")
    assert tr[0] == lbvh[0] and tr[1] > lbvh[1]          # same output, more scratch


def test_morton_bits_option():
    """Key width: 0 / 21 (63-bit keys) or 10 (30-bit keys, at most 2^20
    primitives); anything else is rejected before any GPU work."""
    import paper_2001_09792_amd as rg
    lib, s = rg._lib, rg.Sizes()
    assert rg.blas_sizes(1000, morton_bits=10) == rg.blas_sizes(1000)
    assert rg.blas_sizes(1000, morton_bits=21) == rg.blas_sizes(1000)
    assert rg.blas_sizes(1 << 20, morton_bits=10)[0] > 0
    for bits, n in ((11, 1000), (32, 1000), (-1, 1000), (10, (1 << 20) + 1)):
        o = rg.BuildOpts(4, 4, 0, 0, bits)
        assert lib.rg_blas_sizes(n, ctypes.byref(o), ctypes.byref(s)) == -1, (bits, n)
        assert lib.rg_tlas_sizes(n, ctypes.byref(o), ctypes.byref(s)) == -1, (bits, n)


def test_async_build_arguments_are_checked_on_the_host():
    """rg_build_blas_async / rg_build_blas_finish reject what the host can
    see before enqueueing anything: a missing or misaligned ticket, a builder
    other than the linear one, a ticket holding no pending build."""
    import paper_2001_09792_amd as rg
    lib = rg._lib
    raw = ctypes.create_string_buffer(rg.BUILD_TICKET_BYTES + 32)
    t = (ctypes.addressof(raw) + 15) & ~15
    d = rg.BlasDesc()
    assert lib.rg_build_blas_finish(t, ctypes.byref(d)) == -1          # nothing pending
    assert lib.rg_build_blas_finish(None, ctypes.byref(d)) == -1
    assert lib.rg_build_blas_finish(t + 4, ctypes.byref(d)) == -1      # misaligned
    fake = 1 << 20  # never dereferenced: every call below fails its host checks
    nb, ns = rg.blas_sizes(1000)
    args = lambda o, ticket: (fake, 3000, fake, 1000, None, ctypes.byref(o), fake, nb, fake, ns, None, ticket)  # noqa: E731
    assert lib.rg_build_blas_async(*args(rg.BuildOpts(4, 4, 0, 0), None)) == -1
    assert lib.rg_build_blas_async(*args(rg.BuildOpts(4, 4, 0, 0), t + 8)) == -1
    assert lib.rg_build_blas_async(*args(rg.BuildOpts(4, 4, 1, 0), t)) == -4   # clustering: unsupported
    assert lib.rg_build_blas_async(*args(rg.BuildOpts(4, 4, 2, 0), t)) == -4   # treelets: unsupported
    assert lib.rg_build_blas_async(*args(rg.BuildOpts(3, 4, 0, 0), t)) == -1


def test_async_tlas_arguments_are_checked_on_the_host():
    import paper_2001_09792_amd as rg
    lib = rg._lib
    nb = ctypes.c_uint64()
    assert lib.rg_tlas_ticket_bytes(100, 4, 0, ctypes.byref(nb)) == 0 and nb.value > 100 * 48
    n1 = ctypes.c_uint64()
    assert lib.rg_tlas_ticket_bytes(100, 4, 1, ctypes.byref(n1)) == 0 and n1.value > nb.value
    assert lib.rg_tlas_ticket_bytes(0, 4, 0, ctypes.byref(nb)) == -1
    raw = ctypes.create_string_buffer(1 << 16)
    t = (ctypes.addressof(raw) + 255) & ~255
    d = rg.TlasDesc()
    assert lib.rg_build_tlas_finish(t, ctypes.byref(d)) == -1        # nothing pending
    assert lib.rg_build_tlas_finish(t + 16, ctypes.byref(d)) == -1   # misaligned
    blas = (rg.BlasDesc * 1)()
    xf = (ctypes.c_float * 12)(1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0)
    ids = (ctypes.c_uint32 * 1)(0)
    o = rg.BuildOpts(4, 1, 1, 0)  # clustering: unsupported asynchronously
    fake = 1 << 20
    assert lib.rg_build_tlas_async(blas, 1, xf, ids, ids, None, 1, ctypes.byref(o), fake, 1 << 20, fake, 1 << 20,
                                   None, t, 1 << 15) in (-1, -4)
    assert lib.rg_build_tlas_async(blas, 1, xf, ids, ids, None, 1, None, fake, 1 << 20, fake, 1 << 20, None,
                                   t + 8, 1 << 15) == -1
