"""Serving loop: render requests of many scenes, admitted first come first
served against a device-memory budget, with continuous batching.

The paper's renderer keeps loaded resources for reuse (its resource manager,
section 2.2) and dispatches frames one after another.  Here:

  * ResidentCache keeps built top/bottom levels on the device, keyed by
    scene id, least recently used first out under a byte budget; entries in
    use by a frame in flight are pinned.
  * serve() is the request loop.  Requests arrive at given times (Poisson
    in the benchmarks); the head of the queue is admitted as soon as the
    executor has room for it (FIFO: no later request overtakes it, so none
    starves); the executor is kept one or two passes ahead of the device;
    completions are timestamped on a monotonic host clock.
  * EngineExecutor drives rg_engine_* (continuous batching: frames join and
    leave between passes, sharing every launch); PlainExecutor renders one
    frame at a time with rg_render (the queue-only baseline);
    SimExecutor replays the same admission accounting (rg_pool_*) on a
    simulated clock, for tests without a GPU.

Host logic only: every ray is traced by librg.so.
"""
from __future__ import annotations

import collections
import ctypes
import math
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, Hashable, List, Optional

import numpy as np

RESOLUTIONS = ((256, 256), (512, 512), (1280, 720), (1920, 1080))


@dataclass
class Request:
    rid: int
    scene: int
    width: int
    height: int
    depth: int
    arrival: float                 # seconds from the start of the run
    t_admit: float = math.nan
    t_done: float = math.nan

    @property
    def pixels(self) -> int:
        return self.width * self.height

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


def poisson_requests(n: int, rate: float, n_scenes: int, seed: int, resolutions=RESOLUTIONS,
                     depths=(1, 2, 3, 4), start: float = 0.0, rid0: int = 0) -> List[Request]:
    """n requests with exponential inter-arrival times of mean 1/rate (rate
    = inf: all at `start`); scene uniform over n_scenes, resolution and
    depth uniform over the given sets."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    gaps = np.zeros(n) if math.isinf(rate) else rng.exponential(1.0 / rate, n)
    t = start + np.cumsum(gaps)
    scene = rng.integers(0, n_scenes, n)
    res = rng.integers(0, len(resolutions), n)
    dep = rng.integers(0, len(depths), n)
    return [Request(rid0 + k, int(scene[k]), resolutions[res[k]][0], resolutions[res[k]][1], int(depths[dep[k]]),
                    float(t[k])) for k in range(n)]


# ------------------------------------------------------------------ clocks
class RealClock:
    def __init__(self):
        self.t0 = time.perf_counter()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def sleep_until(self, t: float):
        while True:
            d = t - self.now()
            if d <= 0:
                return
            time.sleep(min(d, 0.002))


class SimClock:
    def __init__(self):
        self.t = 0.0

    def now(self) -> float:
        return self.t

    def sleep_until(self, t: float):
        self.t = max(self.t, t)


# ------------------------------------------------------------ resident cache
class ResidentCache:
    """scene id -> resident object, loaded by loader(id) -> (obj, nbytes).
    Least recently used unpinned entries are evicted when the resident bytes
    would exceed budget_bytes (None: no limit).  get() pins, release()
    unpins; a pinned entry is never evicted."""

    def __init__(self, loader: Callable[[Hashable], tuple], budget_bytes: Optional[int] = None):
        self.loader = loader
        self.budget = budget_bytes
        self.entries: "collections.OrderedDict[Hashable, list]" = collections.OrderedDict()  # id -> [obj, n, pins]
        self.bytes = 0
        self.hits = self.misses = self.evictions = 0

    def _evict_for(self, need: int):
        if self.budget is None:
            return
        for key in list(self.entries.keys()):
            if self.bytes + need <= self.budget:
                return
            e = self.entries[key]
            if e[2] == 0:
                del self.entries[key]
                self.bytes -= e[1]
                self.evictions += 1

    def get(self, key: Hashable):
        e = self.entries.get(key)
        if e is not None:
            self.hits += 1
            self.entries.move_to_end(key)
        else:
            self.misses += 1
            obj, n = self.loader(key)
            self._evict_for(n)
            if self.budget is not None and self.bytes + n > self.budget:
                raise MemoryError(f"scene {key!r} ({n} bytes) does not fit the resident budget "
                                  f"({self.bytes} of {self.budget} bytes pinned)")
            e = [obj, n, 0]
            self.entries[key] = e
            self.bytes += n
        e[2] += 1
        return e[0]

    def release(self, key: Hashable):
        self.entries[key][2] -= 1

    def stats(self) -> dict:
        return dict(resident=len(self.entries), bytes=self.bytes, hits=self.hits, misses=self.misses,
                    evictions=self.evictions)


# --------------------------------------------------------------- executors
class SimExecutor:
    """The engine's admission and pass structure on a simulated device:
    reservations go through the real rg_pool; a pass over `bound` queue
    entries takes pass_cost(bound) simulated seconds.  reserve(req) ->
    (rays, pixels) gives a request's reservation."""

    def __init__(self, pool, clock: SimClock, reserve: Callable[[Request], tuple],
                 pass_cost: Callable[[int], float], on_admit: Optional[Callable] = None):
        self.pool, self.clock, self.reserve, self.cost = pool, clock, reserve, pass_cost
        self.on_admit = on_admit
        self.frames: Dict[int, tuple] = {}      # slot -> (rid, start, last, pixels, growth)
        self.passes = 0
        self.device_free = 0.0
        self.pending: collections.deque = collections.deque()  # (pass, end time)
        self.max_in_pass = 0

    def admit(self, req: Request) -> bool:
        rays, pix = self.reserve(req)
        got = self.pool.reserve(rays, pix)
        if got is None:
            return False
        slot, _ = got
        growth = 2 if rays > pix else 1
        self.frames[slot] = (req.rid, self.passes, self.passes + req.depth, pix, growth)
        if self.on_admit:
            self.on_admit(req)
        return True

    def step(self) -> bool:
        active = [f for f in self.frames.values() if f[2] >= self.passes]
        if not active:
            return False
        bound = sum(f[3] * (f[4] ** (self.passes - f[1])) for f in active)
        self.max_in_pass = max(self.max_in_pass, len(active))
        start = max(self.clock.now(), self.device_free)
        self.device_free = start + self.cost(bound)
        self.pending.append((self.passes, self.device_free))
        self.passes += 1
        return True

    def outstanding(self) -> int:
        return len(self.pending)

    def poll(self, wait: bool = False) -> List[int]:
        if wait and self.pending:
            self.clock.sleep_until(self.pending[0][1])
        out = []
        while self.pending and self.pending[0][1] <= self.clock.now():
            p, _ = self.pending.popleft()
            for slot in [s for s, f in self.frames.items() if f[2] == p]:
                out.append(self.frames.pop(slot)[0])
                self.pool.release(slot)
        return out


class EngineExecutor:
    """Continuous batching on the GPU through rg_engine_*.  scenes: a
    ResidentCache whose objects are (tlas, materials_array, camera, light)."""

    def __init__(self, engine, scenes: ResidentCache, keep_images: bool = False, device="cuda"):
        self.engine, self.scenes, self.keep, self.device = engine, scenes, keep_images, device
        self.live: Dict[int, tuple] = {}     # rid -> (request, image)
        self.images: Dict[int, object] = {}
        self._outstanding = 0

    def admit(self, req: Request) -> bool:
        import torch
        tl, ma, cam, light = self.scenes.get(req.scene)
        img = torch.empty((req.height, req.width, 3), dtype=torch.float32, device=self.device)
        ok = self.engine.admit(tl, ma, cam, light, req.width, req.height, req.depth, img, req.rid)
        if not ok:
            self.scenes.release(req.scene)
            return False
        self.live[req.rid] = (req, img)
        return True

    def step(self) -> bool:
        return self.engine.step()

    def outstanding(self) -> int:
        i = self.engine.info()
        return i["passes"] - i["passes_done"]

    def poll(self, wait: bool = False) -> List[int]:
        done = self.engine.poll(wait)
        for rid in done:
            req, img = self.live.pop(rid)
            self.scenes.release(req.scene)
            if self.keep:
                self.images[rid] = img
        return done


class PlainExecutor:
    """One frame at a time with rg_render (a queue and nothing more): the
    next request is admitted only when the device is idle."""

    def __init__(self, scenes: ResidentCache, max_pixels: int, max_depth: int = 4, keep_images: bool = False,
                 device="cuda"):
        import torch
        import paper_2001_09792_amd as rg
        self.rg, self.scenes, self.keep, self.device = rg, scenes, keep_images, device
        self.scratch = torch.empty(rg.render_sizes(max_pixels, 1, max_depth, 0), dtype=torch.uint8, device=device)
        self.cur = None            # (request, image, event) of the frame in flight
        self.queued = None
        self.images: Dict[int, object] = {}

    def admit(self, req: Request) -> bool:
        if self.cur is not None or self.queued is not None:
            return False
        self.queued = req
        return True

    def step(self) -> bool:
        import torch
        if self.queued is None:
            return False
        req, self.queued = self.queued, None
        tl, ma, cam, light = self.scenes.get(req.scene)
        img = torch.empty((req.height, req.width, 3), dtype=torch.float32, device=self.device)
        self.rg.render_into(tl, ma, cam, light, req.width, req.height, req.depth, img, self.scratch)
        ev = torch.cuda.Event()
        ev.record()
        self.cur = (req, img, ev)
        return True

    def outstanding(self) -> int:
        return 0 if self.cur is None else 1

    def poll(self, wait: bool = False) -> List[int]:
        if self.cur is None:
            return []
        req, img, ev = self.cur
        if wait:
            ev.synchronize()
        elif not ev.query():
            return []
        self.cur = None
        self.scenes.release(req.scene)
        if self.keep:
            self.images[req.rid] = img
        return [req.rid]


# ----------------------------------------------------------------- the loop
def serve(requests: List[Request], ex, clock, max_ahead: int = 2, on_step: Optional[Callable] = None) -> dict:
    """Runs requests (arrival times on `clock`) through executor `ex` until
    all are complete; fills t_admit / t_done.  FIFO admission: the head of
    the queue waits until it fits and nothing behind it goes first."""
    reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
    by_id = {r.rid: r for r in reqs}
    n, i, done = len(reqs), 0, 0
    waiting: collections.deque = collections.deque()
    order: List[int] = []
    max_waiting = 0
    while done < n:
        now = clock.now()
        while i < n and reqs[i].arrival <= now:
            waiting.append(reqs[i])
            i += 1
        max_waiting = max(max_waiting, len(waiting))
        while waiting and ex.admit(waiting[0]):
            r = waiting.popleft()
            r.t_admit = now
            order.append(r.rid)
        stepped = ex.outstanding() < max_ahead and ex.step()
        if stepped and on_step:
            on_step()
        finished = ex.poll(False)
        if not finished and not stepped:
            if ex.outstanding() > 0:
                finished = ex.poll(True)
            elif i < n:
                clock.sleep_until(reqs[i].arrival)
            elif waiting:
                raise RuntimeError(f"request {waiting[0].rid} cannot be admitted on an idle executor")
        t = clock.now()
        for rid in finished:
            by_id[rid].t_done = t
            done += 1
    return dict(order=order, max_waiting=max_waiting)


def summarize(reqs: List[Request], rays: Optional[int] = None) -> dict:
    lat = np.array([r.latency for r in reqs])
    t0 = min(r.arrival for r in reqs)
    t1 = max(r.t_done for r in reqs)
    out = dict(requests=len(reqs), p50_ms=float(np.percentile(lat, 50) * 1e3),
               p99_ms=float(np.percentile(lat, 99) * 1e3), mean_ms=float(lat.mean() * 1e3),
               span_s=float(t1 - t0), req_per_s=float(len(reqs) / max(t1 - t0, 1e-9)))
    if rays is not None:
        out["mrays_s"] = rays / max(t1 - t0, 1e-9) / 1e6
    return out
