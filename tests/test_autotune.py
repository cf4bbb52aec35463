"""The autotuner's search and cache (host logic, no GPU)."""
import numpy as np

from paper_2001_09792_amd import autotune as at


def test_bucket():
    assert at.bucket(4 ** 10, 4 ** 12) == "rays4^10-tris4^12"
    assert at.bucket(1, 1) == "rays4^0-tris4^0"


def test_search_finds_separable_optimum():
    target = dict(builder="ploc", width=8, leaf=1, lds_depth=24, refill=16, waves_per_cu=12, leaf_batch=16,
                  inst_batch=8)

    def measure(c):
        return 100.0 - sum(abs(at.SPACE[k].index(c[k]) - at.SPACE[k].index(target[k])) for k in c)

    cfg, best, trials = at.search(measure)
    assert cfg == target and best == 100.0
    # every configuration is measured once
    keys = [tuple(sorted(c.items())) for c, _ in trials]
    assert len(keys) == len(set(keys))


def test_search_keeps_default_when_flat():
    cfg, best, trials = at.search(lambda c: 1.0)
    assert cfg == at.DEFAULT


def test_cache_round_trip(tmp_path):
    cache = at.TuneCache(str(tmp_path / "t.json"))
    assert cache.get("gfx950", "trace", "b") is None
    cache.put("gfx950", "trace", "b", dict(config=at.DEFAULT, score=3.0))
    cache.put("gfx950", "batch", "c", dict(config=at.DEFAULT, score=4.0))
    assert cache.get("gfx950", "trace", "b")["score"] == 3.0
    assert cache.get("gfx950", "batch", "c")["score"] == 4.0
    assert cache.get("gfx942", "trace", "b") is None


def test_search_noisy_measure_is_deterministic_per_config():
    rng = np.random.default_rng(0)
    table = {}

    def measure(c):
        key = tuple(sorted(c.items()))
        if key not in table:
            table[key] = float(rng.uniform(0, 1))
        return table[key]

    cfg, best, trials = at.search(measure)
    assert best == max(v for _, v in trials)
