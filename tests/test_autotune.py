"""Host logic of the autotuner (no GPU): workload shape keys, the cache file,
and the coordinate-descent search on a synthetic cost function."""
import json

import pytest

from paper_2508_20735_amd import autotune as T


def test_batch_shape_buckets():
    s = T.batch_shape([64, 100, 5000, 65536], [2, 8, 3, 5], "minimise")
    assert s == "batch-minimise|count2^2|states2^16|median2^11|kmax8"
    assert T.batch_shape([1], [1], "equivalent") == "batch-equivalent|count2^0|states2^0|median2^0|kmax1"


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "tuning.json")
    assert T.lookup("shape-a", path, device="gpuX|256cu") is None
    T.save_entry("shape-a", {"chunk": 8, "batch_lds_states": 2048}, 1.5, path, device="gpuX|256cu")
    T.save_entry("shape-b", {"chunk": 4}, 2.0, path, device="gpuX|256cu")
    T.save_entry("shape-a", {"chunk": 16}, 1.2, path, device="gpuY|80cu")
    assert T.lookup("shape-a", path, device="gpuX|256cu") == {"chunk": 8, "batch_lds_states": 2048}
    assert T.lookup("shape-a", path, device="gpuY|80cu") == {"chunk": 16}
    data = json.load(open(path))
    assert data["gpuX|256cu"]["shape-b"]["device_ms"] == 2.0
    # a damaged cache reads as empty
    open(path, "w").write("{not json")
    assert T.load_cache(path) == {}


def test_search_coordinate_descent(monkeypatch):
    state = {"a": 1, "b": 10}
    monkeypatch.setattr(T.B, "get_tuning", lambda: dict(state))
    monkeypatch.setattr(T.B, "set_tuning", lambda **kw: state.update(kw))
    # cost: a best at 3, b best at 30 (separable), plus call counting
    calls = []

    def run():
        calls.append(dict(state))
        return abs(state["a"] - 3) + abs(state["b"] - 30) / 10 + 1.0

    best, ms = T.search(run, {"a": [1, 2, 3, 4], "b": [10, 20, 30]}, reps=1)
    assert best == {"a": 3, "b": 30} and ms == pytest.approx(1.0)
    assert state == best  # left set
    # every candidate timed after a warm-up run (2 runs each), the start too
    assert len(calls) == 2 * (1 + 3 + 2)
