"""Host logic of the tuner (no GPU): the workload signature, the coordinate
descent over result-neutral knobs, and the persisted cache file."""
import json
import os

import pytest

tune = pytest.importorskip("paper_2510_19301_amd.tune")


def test_signature_buckets_lengths_and_separates_workloads():
    a = tune.signature("gfx950", 1024, "dense", "flash", 0, [500, 4000, 8000])
    b = tune.signature("gfx950", 1024, "dense", "flash", 0, [600, 3000, 7000])   # same buckets
    c = tune.signature("gfx950", 1024, "dense", "flash", 0, [600, 3000, 9000])   # longer tail
    d = tune.signature("gfx950", 1024, "dense", "beam", 64, [500, 4000, 8000])
    e = tune.signature("gfx942", 1024, "dense", "flash", 0, [500, 4000, 8000])
    assert a == b and len({a, c, d, e}) == 4
    assert "tmed4096" in a and "tmax8192" in a and "n4" in a


def test_search_space_per_method_and_model():
    s = dict(tune.search_space("flash", 1024, "dense", (4, 16)))
    assert s["P"] == [4, 16] and "leaves" in s and "engine" not in s and s["step"] == ["auto", "items", "tiles"]
    s = dict(tune.search_space("vanilla", 128, "dense", (4,)))
    assert "P" not in s and s["engine"] == [False, True] and "leaves" not in s
    s = dict(tune.search_space("beam", 1024, "csr", (4,)))
    assert s == {}


def test_coordinate_descent_finds_separable_optimum_once_per_candidate():
    costs = {"P": {4: 5.0, 16: 2.0, 64: 3.0}, "rows": {"auto": 1.0, "wide": 4.0, "local": 0.5},
             "step": {"auto": 1.0, "items": 0.7, "tiles": 2.0}, "leaves": {True: 0.0, False: 1.0}}
    calls = []

    def evaluate(cfg):
        calls.append(cfg)
        return sum(costs[k][cfg[k]] for k in costs)

    space = tune.search_space("flash", 1024, "dense", (4, 16, 64))
    best, seen = tune.coordinate_descent(evaluate, space, dict(tune.DEFAULT, P=4))
    assert best["P"] == 16 and best["rows"] == "local" and best["step"] == "items" and best["leaves"] is True
    assert len(calls) == len(seen) == len({json.dumps(c, sort_keys=True) for c in calls})


def test_cache_roundtrip_and_atomic_update(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    assert tune.load_cache(path) == {}
    tune.store(path, "k1", {"config": {"P": 64}, "timings": {"x": 1.0}})
    tune.store(path, "k2", {"config": {"P": 16}, "timings": {}})
    data = tune.load_cache(path)
    assert data["k1"]["config"]["P"] == 64 and data["k2"]["config"]["P"] == 16
    assert [f for f in os.listdir(tmp_path / "sub") if f.startswith(".tune.")] == []
    with open(path, "w") as f:
        f.write("not json")
    assert tune.load_cache(path) == {}


def test_cache_path_from_environment(monkeypatch, tmp_path):
    monkeypatch.setenv("FV_TUNE_CACHE", str(tmp_path / "t.json"))
    assert tune.cache_path() == str(tmp_path / "t.json")
