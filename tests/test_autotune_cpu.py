"""Host logic of the autotuner: the search, the graph-class key, the cache."""
import json

import pytest

pytest.importorskip("torch")

from paper_1509_08267_amd import autotune  # noqa: E402


def test_coordinate_descent_finds_separable_optimum():
    # time = sum of independent per-knob costs: coordinate descent is exact
    cost = {"lanes": {2: 3.0, 4: 1.0, 8: 2.0}, "medium_degree": {0: 2.0, 64: 0.5},
            "heavy_degree": {1024: 1.0, 4096: 0.2}, "blocks_per_cu": {4: 0.3, 8: 0.1}}
    seen = []

    def measure(s):
        seen.append(dict(s))
        return sum(cost[k][s[k]] for k in cost)

    start = {"lanes": 2, "medium_degree": 0, "heavy_degree": 1024, "blocks_per_cu": 4}
    cands = {k: list(v) for k, v in cost.items()}
    best, t, table = autotune.coordinate_descent(autotune.KNOBS, cands, measure, start)
    assert best == {"lanes": 4, "medium_degree": 64, "heavy_degree": 4096, "blocks_per_cu": 8}
    assert t == pytest.approx(1.0 + 0.5 + 0.2 + 0.1)
    # the start is measured once, and no setting is measured twice
    keys = [tuple(sorted(s.items())) for s in seen]
    assert len(keys) == len(set(keys)) == len(table)
    assert table[0][0] == start


def test_coordinate_descent_keeps_start_when_nothing_is_faster():
    best, t, _ = autotune.coordinate_descent(
        ["lanes"], {"lanes": [2, 4, 8]}, lambda s: 1.0 if s["lanes"] == 16 else 2.0, {"lanes": 16})
    assert best == {"lanes": 16} and t == 1.0


def test_coordinate_descent_stops_on_budget():
    # an exhausted budget reads as an infinite time: the best so far is kept
    calls = []

    def measure(s):
        calls.append(s)
        return 5.0 if len(calls) == 1 else float("inf")

    best, t, _ = autotune.coordinate_descent(["lanes"], {"lanes": [2, 4]}, measure, {"lanes": 8})
    assert best == {"lanes": 8} and t == 5.0


def test_graph_class_key():
    a = autotune.graph_class(1 << 20, 1 << 25, 62, False, "push")
    assert a == "rp32-n20-avg5-max5-push"
    assert autotune.graph_class(1 << 20, 1 << 25, 62, True, "push") != a
    assert autotune.graph_class(1 << 20, 1 << 25, 62, False, "pull") != a
    # same buckets, same class
    assert autotune.graph_class(1_100_000, 1_100_000 * 33, 60, False, "push") == a
    assert autotune.graph_class(0, 0, 0, False, "push") == "rp32-n0-avg0-max0-push"


def test_cache_round_trip(tmp_path):
    path = tmp_path / "sub" / "tune.json"
    c = autotune.Cache(str(path))
    assert c.get("dev", "cls") is None
    c.put("dev", "cls", {"lanes": 4}, 1e-3)
    c.put("dev", "cls2", {"lanes": 8}, 2e-3)
    d = autotune.Cache(str(path))
    assert d.get("dev", "cls") == {"setting": {"lanes": 4}, "seconds": 1e-3}
    assert json.loads(path.read_text())["dev"]["cls2"]["setting"] == {"lanes": 8}


def test_shipped_table_is_a_read_only_fallback(tmp_path):
    shipped = tmp_path / "shipped.json"
    shipped.write_text(json.dumps({"dev": {"cls": {"setting": {"lanes": 16}, "seconds": 5e-4}}}))
    c = autotune.Cache(str(tmp_path / "user.json"), shipped=str(shipped))
    assert c.get("dev", "cls")["setting"] == {"lanes": 16}       # from the shipped table
    assert c.get("dev", "other") is None
    c.put("dev", "cls", {"lanes": 4}, 1e-3)                      # the user's entry wins
    assert autotune.Cache(str(tmp_path / "user.json"), shipped=str(shipped)).get(
        "dev", "cls")["setting"] == {"lanes": 4}
    assert json.loads(shipped.read_text())["dev"]["cls"]["setting"] == {"lanes": 16}
    assert autotune.Cache(str(tmp_path / "none.json"), shipped=None).get("dev", "cls") is None


def test_cache_path_from_environment(monkeypatch, tmp_path):
    monkeypatch.setenv("GC_AUTOTUNE_CACHE", str(tmp_path / "x.json"))
    assert autotune.default_cache_path() == str(tmp_path / "x.json")
