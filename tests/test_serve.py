"""Serving host logic on the CPU: the admission pool (rg_pool_*, C++), the
frame reservation bound, the resident-scene cache and the FIFO request loop
driven through a simulated executor and clock.  No GPU calls."""
import math

import numpy as np
import pytest

import paper_2001_09792_amd as rg
import scenegen as sg
from paper_2001_09792_amd import serve

DIFFUSE_ONLY = rg.materials_array(sg.materials([(0, (0.5, 0.5, 0.5), 1.5), (1, (0.9, 0.9, 0.9), 1.5)]))
WITH_GLASS = rg.materials_array(sg.materials([(0, (0.5, 0.5, 0.5), 1.5), (2, (1, 1, 1), 1.5)]))


# ------------------------------------------------------------------ pool
def test_pool_reserve_release_coalesce():
    p = rg.Pool(1000, 100, 4)
    a = p.reserve(100, 30)
    b = p.reserve(100, 30)
    c = p.reserve(100, 30)
    assert [a, b, c] == [(0, 0), (1, 30), (2, 60)]
    assert p.reserve(100, 20) is None                 # 10 pixels left
    assert p.usage() == dict(rays=300, pixels=90, largest_free_pixels=10, jobs=3)
    p.release(1)                                      # hole [30, 60)
    assert p.reserve(10, 40) is None                  # no contiguous 40
    d = p.reserve(10, 25)
    assert d == (1, 30)                               # lowest slot, first fit
    p.release(0)
    p.release(1)
    p.release(2)
    assert p.usage() == dict(rays=0, pixels=0, largest_free_pixels=100, jobs=0)  # coalesced back
    assert p.reserve(1000, 100) == (0, 0)


def test_pool_limits_and_errors():
    p = rg.Pool(100, 100, 2)
    with pytest.raises(rg.RgError) as e:
        p.reserve(101, 1)                            # larger than the whole pool
    assert e.value.status == -2
    with pytest.raises(rg.RgError):
        p.reserve(1, 101)
    with pytest.raises(rg.RgError):
        p.reserve(0, 1)
    assert p.reserve(10, 10) is not None
    assert p.reserve(10, 10) is not None
    assert p.reserve(10, 10) is None                 # out of slots
    with pytest.raises(rg.RgError):
        p.release(5)
    p.release(0)
    with pytest.raises(rg.RgError):
        p.release(0)                                 # already free
    with pytest.raises(rg.RgError):
        rg.Pool(0, 10, 1)


def test_pool_random_against_model():
    rng = np.random.default_rng(11)
    R, P, J = 5000, 4000, 16
    p = rg.Pool(R, P, J)
    held = {}
    for _ in range(3000):
        if held and rng.random() < 0.45:
            slot = list(held)[rng.integers(len(held))]
            p.release(slot)
            del held[slot]
        else:
            rays, pix = int(rng.integers(1, 800)), int(rng.integers(1, 700))
            got = p.reserve(rays, pix)
            used_r = sum(h[0] for h in held.values())
            if got is None:
                # refused only for a real reason: rays, slots or no contiguous range
                free = _free_ranges(held, P)
                assert used_r + rays > R or len(held) == J or max([b - a for a, b in free] + [0]) < pix
                continue
            slot, off = got
            assert slot not in held and 0 <= off and off + pix <= P
            for (_, o2, n2) in held.values():
                assert off + pix <= o2 or o2 + n2 <= off   # no overlap
            held[slot] = (rays, off, pix)
        u = p.usage()
        assert u["rays"] == sum(h[0] for h in held.values()) <= R
        assert u["pixels"] == sum(h[2] for h in held.values()) <= P
        assert u["jobs"] == len(held)


def _free_ranges(held, P):
    used = sorted((o, o + n) for (_, o, n) in held.values())
    out, cur = [], 0
    for a, b in used:
        if a > cur:
            out.append((cur, a))
        cur = max(cur, b)
    if cur < P:
        out.append((cur, P))
    return out


def test_job_reservation_bound():
    # a glass hit spawns two children, so depth k holds up to pixels * 2^k
    assert rg.job_reservation(WITH_GLASS, 64, 32, 3) == (64 * 32 * 8, 64 * 32)
    assert rg.job_reservation(WITH_GLASS, 64, 32, 0) == (64 * 32, 64 * 32)
    # mirror / diffuse: at most one child per ray
    assert rg.job_reservation(DIFFUSE_ONLY, 64, 32, 4) == (64 * 32, 64 * 32)
    with pytest.raises(rg.RgError):
        rg.job_reservation(WITH_GLASS, 64, 32, rg.MAX_DEPTH + 1)


# --------------------------------------------------------- resident cache
def test_resident_cache_lru_and_pins():
    loads = []

    def loader(k):
        loads.append(k)
        return f"scene{k}", 10

    c = serve.ResidentCache(loader, budget_bytes=30)
    for k in (0, 1, 2):
        c.get(k)
        c.release(k)
    c.get(0)                      # 0 becomes most recent
    c.release(0)
    c.get(3)                      # evicts 1 (least recent)
    c.release(3)
    assert list(c.entries) == [2, 0, 3] and c.evictions == 1
    c.get(2)                      # pin 2 and 0
    c.get(0)
    c.get(4)                      # must evict 3, the only unpinned one
    assert set(c.entries) == {2, 0, 4}
    with pytest.raises(MemoryError):
        c.get(5)                  # everything pinned
    c.release(2)
    assert c.get(5) == "scene5"   # 2 evicted now
    assert loads == [0, 1, 2, 3, 4, 5, 5]
    s = c.stats()
    assert s["resident"] == 3 and s["bytes"] == 30 and s["hits"] == 3


# ------------------------------------------------------ the request loop
def _sim(reqs, max_rays, max_pixels, max_jobs=64, glass=True, cost=lambda n: 1e-4 + n * 1e-9, checks=None):
    pool = rg.Pool(max_rays, max_pixels, max_jobs)
    clock = serve.SimClock()
    mats = WITH_GLASS if glass else DIFFUSE_ONLY

    def reserve(r):
        return rg.job_reservation(mats, r.width, r.height, r.depth)

    def on_admit(r):
        u = pool.usage()
        assert u["rays"] <= max_rays and u["pixels"] <= max_pixels and u["jobs"] <= max_jobs
        if checks is not None:
            checks.append((clock.now(), u))

    ex = serve.SimExecutor(pool, clock, reserve, cost, on_admit)
    info = serve.serve(reqs, ex, clock)
    return ex, info, pool


def test_serve_fifo_budget_and_completion():
    reqs = serve.poisson_requests(400, 300.0, 64, seed=5)
    checks = []
    budget = 40_000_000
    ex, info, pool = _sim(reqs, budget, budget, checks=checks)
    # every request completes, after it arrived and was admitted
    assert all(math.isfinite(r.t_done) and r.t_done >= r.t_admit >= r.arrival for r in reqs)
    # FIFO: admission order is arrival order
    assert info["order"] == [r.rid for r in sorted(reqs, key=lambda r: (r.arrival, r.rid))]
    assert len(checks) == len(reqs)
    assert pool.usage() == dict(rays=0, pixels=0, largest_free_pixels=budget, jobs=0)
    # continuous batching: frames share passes
    assert ex.max_in_pass > 1


def test_tiny_budget_forces_queueing_without_starvation():
    # room for one 1920x1080 depth-4 frame with glass at a time (and a few small ones)
    big = 1920 * 1080 * 16
    reqs = serve.poisson_requests(120, 2000.0, 8, seed=7)
    ex, info, pool = _sim(reqs, big, big)
    assert all(math.isfinite(r.t_done) for r in reqs)
    waits = np.array([r.t_admit - r.arrival for r in reqs])
    assert (waits > 0).sum() > len(reqs) // 2          # most requests queued
    assert info["max_waiting"] > 10
    assert info["order"] == [r.rid for r in sorted(reqs, key=lambda r: (r.arrival, r.rid))]
    # the largest requests were served too (no starvation behind small ones)
    largest = [r for r in reqs if r.pixels == 1920 * 1080 and r.depth == 4]
    assert largest and all(math.isfinite(r.t_done) for r in largest)


def test_one_slot_serialises():
    reqs = serve.poisson_requests(30, math.inf, 4, seed=3)
    ex, info, pool = _sim(reqs, 1 << 31, 1 << 31, max_jobs=1)
    assert ex.max_in_pass == 1
    spans = sorted((r.t_admit, r.t_done) for r in reqs)
    for (a0, d0), (a1, d1) in zip(spans, spans[1:]):
        assert a1 >= d0                                 # one frame at a time


def test_request_that_never_fits_is_an_error():
    reqs = [serve.Request(0, 0, 1920, 1080, 4, 0.0)]
    with pytest.raises(rg.RgError):
        _sim(reqs, 1 << 20, 1 << 20)


def test_depth_mix_in_one_pass():
    # frames admitted a pass apart overlap at different recursion depths
    reqs = [serve.Request(k, 0, 256, 256, 4, k * 2e-4) for k in range(6)]
    pool = rg.Pool(1 << 30, 1 << 30, 8)
    clock = serve.SimClock()
    depths = []

    class Probe(serve.SimExecutor):
        def step(self):
            live = [f for f in self.frames.values() if f[2] >= self.passes]
            depths.append({self.passes - f[1] for f in live})
            return super().step()

    ex = Probe(pool, clock, lambda r: rg.job_reservation(WITH_GLASS, r.width, r.height, r.depth),
               lambda n: 2e-4, None)
    serve.serve(reqs, ex, clock, max_ahead=1)
    assert max(len(d) for d in depths) >= 3
    assert all(math.isfinite(r.t_done) for r in reqs)


def test_poisson_requests_statistics():
    reqs = serve.poisson_requests(20000, 50.0, 64, seed=5)
    gaps = np.diff([0.0] + [r.arrival for r in reqs])
    assert abs(gaps.mean() - 1 / 50.0) < 0.02 / 50 * 10
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05      # exponential: cv = 1
    assert {(r.width, r.height) for r in reqs} == set(serve.RESOLUTIONS)
    assert {r.depth for r in reqs} == {1, 2, 3, 4}
    assert min(r.scene for r in reqs) == 0 and max(r.scene for r in reqs) == 63


def test_summarize():
    reqs = [serve.Request(k, 0, 1, 1, 1, float(k), t_admit=float(k), t_done=float(k) + 0.01 * (k + 1))
            for k in range(100)]
    s = serve.summarize(reqs, rays=10**6)
    assert abs(s["p50_ms"] - np.percentile([0.01 * (k + 1) for k in range(100)], 50) * 1e3) < 1e-6
    assert abs(s["p99_ms"] - np.percentile([0.01 * (k + 1) for k in range(100)], 99) * 1e3) < 1e-6
