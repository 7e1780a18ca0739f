"""Host logic of the launch-shape autotuner (no GPU needed)."""
import json

from paper_2302_13529_amd import autotune
from paper_2302_13529_amd import graphgen as gg


def test_descent_finds_the_minimum_of_a_separable_cost():
    grid = {"a": [1, 2, 3, 4, 5], "b": [10, 20, 30], "c": [0, 1]}
    calls = []

    def cost(cfg):
        calls.append(cfg)
        return (cfg["a"] - 4) ** 2 + abs(cfg["b"] - 10) + (1 - cfg["c"]) * 0.5

    best, c, table = autotune._descend(grid, {"a": 3, "b": 20, "c": 0}, cost)
    assert best == {"a": 4, "b": 10, "c": 1} and c == 0
    # every configuration is timed at most once
    keys = [tuple(sorted(x.items())) for x in calls]
    assert len(keys) == len(set(keys)) == len(table)


def test_descent_keeps_the_start_when_nothing_is_better():
    best, c, table = autotune._descend({"a": [1, 2, 3]}, {"a": 2}, lambda cfg: 0.0)
    assert best == {"a": 2} and len(table) == 3


def test_signatures_bucket_similar_workloads_together():
    a = gg.batched_instances(count=4, seed=3)
    assert autotune.batch_signature(a) == autotune.batch_signature(a)
    assert autotune.batch_signature(a).startswith("batch/c2/")
    assert autotune.graph_signature(1 << 20, 8 << 20, 10, 1000) == "graph/n20/d3/s3/t10"
    assert autotune.graph_signature(1 << 20, 8 << 20, 10, 1000) == \
        autotune.graph_signature((1 << 20) + 5, 8 << 20, 11, 1100)


def test_cache_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "tuned.json"
    monkeypatch.setenv("IMIN_TUNE_CACHE", str(path))
    autotune.save("gfx950/batch/x", {"launch": {"waves_per_cu": 16}})
    autotune.save("gfx950/batch/y", {"launch": {"waves_per_cu": 8}})
    table = json.loads(path.read_text())
    assert set(table) == {"gfx950/batch/x", "gfx950/batch/y"}
    assert autotune.load_cache()["gfx950/batch/x"]["launch"]["waves_per_cu"] == 16
