"""Host logic of the autotuner: the fastest candidate is chosen, stored in
the JSON cache under the shape key and read back without timing again."""
import json

from paper_2511_01927_amd import autotune


def test_tune_picks_fastest_and_caches(tmp_path):
    calls = []
    cost = {1: 0.004, 2: 0.001, 3: 0.003}

    def solve(variant):
        import time
        calls.append(variant)
        time.sleep(cost[variant])

    path = str(tmp_path / "tune.json")
    key = autotune.shape_key(1000, 31, 9.0, 256, "fp64", "band")
    best = autotune.tune(solve, key, [{"variant": v} for v in (1, 2, 3)], cache_path=path, repeats=2)
    assert best == {"variant": 2}
    assert len(calls) == 9
    with open(path) as f:
        cache = json.load(f)
    assert cache[key]["opts"] == {"variant": 2} and len(cache[key]["candidates"]) == 3
    calls.clear()
    again = autotune.tune(solve, key, [{"variant": v} for v in (1, 2, 3)], cache_path=path)
    assert again == {"variant": 2} and calls == []


def test_shape_key_distinguishes_precision_and_size():
    a = autotune.shape_key(1000, 31, 9.0, 256, "fp64", "band")
    assert a != autotune.shape_key(1000, 31, 9.0, 256, "mixed", "band")
    assert a != autotune.shape_key(1001, 31, 9.0, 256, "fp64", "band")
