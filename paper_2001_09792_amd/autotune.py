"""Autotuner for the traversal: hierarchy builder, node width, leaf size, LDS
stack depth, refill threshold, resident waves per CU and leaf / instance
batching, chosen by measurement.

The best setting depends on the workload's size (rays per launch, triangles,
coherence), so results are cached per GPU architecture, workload kind and
size bucket in a JSON file ($RG_TUNE_CACHE, default
~/.cache/raygun_mi/tune.json).  The search is a coordinate descent: starting
from the defaults, each parameter in turn takes the value that measured best
with the others held, for `passes` rounds.  Builder, width and leaf size are
build-time choices: the caller's `measure` rebuilds when they change.
"""
from __future__ import annotations

import json
import math
import os
import time
from typing import Callable, Dict, Optional

DEFAULT = dict(builder="lbvh", width=4, leaf=1, refill=8, waves_per_cu=16, lds_depth=16, leaf_batch=12,
               inst_batch=6)
BUILD_KEYS = ("builder", "width", "leaf")
SPACE = dict(builder=("lbvh", "ploc", "treelet"), width=(2, 4, 8), leaf=(1, 2, 4), lds_depth=(8, 16, 24), refill=(4, 8, 16, 32),
             waves_per_cu=(12, 16, 24), leaf_batch=(1, 8, 12, 16, 24), inst_batch=(1, 4, 6, 8, 12))
LAUNCH_KEYS = ("refill", "waves_per_cu", "lds_depth", "leaf_batch", "inst_batch")


def bucket(n_rays: int, n_tris: int) -> str:
    """Size bucket: rays and unique triangles, each to the nearest power of 4."""
    r = int(round(math.log(max(n_rays, 1), 4)))
    t = int(round(math.log(max(n_tris, 1), 4)))
    return f"rays4^{r}-tris4^{t}"


def arch() -> str:
    import torch
    return str(torch.cuda.get_device_properties(0).gcnArchName).split(":")[0]


class TuneCache:
    def __init__(self, path: Optional[str] = None):
        self.path = path or os.environ.get("RG_TUNE_CACHE") or os.path.join(
            os.path.expanduser("~"), ".cache", "raygun_mi", "tune.json")

    def _load(self) -> dict:
        try:
            with open(self.path) as f:
                return json.load(f)
        except (OSError, ValueError):
            return {}

    def get(self, arch_name: str, kind: str, bkt: str) -> Optional[dict]:
        return self._load().get(arch_name, {}).get(kind, {}).get(bkt)

    def put(self, arch_name: str, kind: str, bkt: str, entry: dict) -> None:
        data = self._load()
        data.setdefault(arch_name, {}).setdefault(kind, {})[bkt] = entry
        os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def search(measure: Callable[[Dict[str, int]], float], space: Dict[str, tuple] = SPACE,
           start: Optional[Dict[str, int]] = None, passes: int = 2, log=None):
    """Coordinate descent maximising measure(config).  Returns (best config,
    best score, list of (config, score) trials); each config is measured once."""
    cfg = dict(DEFAULT if start is None else start)
    seen = {}

    def score(c):
        key = tuple(sorted(c.items()))
        if key not in seen:
            seen[key] = measure(dict(c))
            if log:
                log(f"  {c} -> {seen[key]:.1f}")
        return seen[key]

    best = score(cfg)
    for _ in range(passes):
        improved = False
        for k, values in space.items():
            for v in values:
                if v == cfg[k]:
                    continue
                c = dict(cfg)
                c[k] = v
                s = score(c)
                if s > best:
                    best, cfg, improved = s, c, True
        if not improved:
            break
    trials = [(dict(k), v) for k, v in seen.items()]
    return cfg, best, trials


def apply_launch(cfg: Dict[str, int], scope: str = "trace") -> dict:
    """Sets the launch parameters of a configuration for one family of calls
    ("trace", "frame" or "engine"); returns them."""
    import paper_2001_09792_amd as rg
    return rg.trace_tuning(scope=scope, **{k: cfg[k] for k in LAUNCH_KEYS if k in cfg})


def tuned(kind: str, n_rays: int, n_tris: int, measure: Callable[[Dict[str, int]], float],
          cache: Optional[TuneCache] = None, space: Dict[str, tuple] = SPACE, log=None,
          start: Optional[Dict[str, int]] = None) -> dict:
    """The cached configuration for this workload bucket, or a fresh search
    (stored in the cache).  Returns {config, score, bucket, cached, seconds}."""
    cache = cache or TuneCache()
    a = arch()
    bkt = bucket(n_rays, n_tris)
    hit = cache.get(a, kind, bkt)
    if hit is not None:
        return dict(config=hit["config"], score=hit["score"], bucket=bkt, cached=True, seconds=0.0)
    t0 = time.perf_counter()
    cfg, best, trials = search(measure, space, start=start, log=log)
    dt = time.perf_counter() - t0
    cache.put(a, kind, bkt, dict(config=cfg, score=best, trials=len(trials), seconds=dt))
    return dict(config=cfg, score=best, bucket=bkt, cached=False, seconds=dt)
