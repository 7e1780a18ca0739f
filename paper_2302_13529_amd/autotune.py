"""Launch-shape autotuner for the decrease kernels.

Launch shapes change speed only, never results (every count is an exact integer sum), so a
tuner may simply time candidates on the workload and keep the fastest. Two searches:

* ``tune_batch(problems)`` -- the wavefront-level kernels of the batched greedy call: waves
  per compute unit of the one-sample-per-wave kernel, its frontier-chunk quad limit, the run
  length of the guided sample schedule, and the workgroups per compute unit of the kernel
  that packs several samples per wave (or that kernel off) (``imin_launch``). The probe is
  the first greedy round of every instance.
* ``tune_graph(graph, seeds, theta)`` -- a plain graph: wave kernel on or off, its launch
  shape, and the workgroup kernel's slot count. The probe is one decrease call.

Both use coordinate descent over small candidate grids (one parameter at a time, repeated
until nothing improves), timing the kernels with the library's own HIP events
(``kernel_ms``), best of ``repeats`` runs. Results are cached as JSON, keyed by the GPU
architecture and a workload signature: a read-only table shipped with the package
(``tuned.json``) and a user cache (``$IMIN_TUNE_CACHE``, else ``~/.cache/imin/tuned.json``)
that tuning writes.
"""
from __future__ import annotations

import json
import math
import os
import statistics

from . import binding

HERE = os.path.dirname(os.path.abspath(__file__))
SHIPPED = os.path.join(HERE, "tuned.json")

BATCH_GRID = {
    "waves_per_cu": [8, 12, 16, 20, 24, 32],
    "quad_limit": [256, 1024, 2048, 8192],
    "pick_div": [1, 2, 4, 8],
    "pack_per_cu": [-1, 1, 2, 3, 4],
}
GRAPH_GRID = {
    "small": [0, 1],
    "waves_per_cu": [8, 16, 20, 32],
    "quad_limit": [512, 2048, 8192],
    "slots": [256, 512, 768],
}


def user_cache_path() -> str:
    return os.environ.get("IMIN_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "imin", "tuned.json"))


def _read(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def load_cache() -> dict:
    """Shipped table overlaid with the user cache."""
    table = _read(SHIPPED)
    table.update(_read(user_cache_path()))
    return table


def save(key: str, entry: dict) -> None:
    path = user_cache_path()
    table = _read(path)
    table[key] = entry
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def gpu_arch() -> str:
    import torch
    props = torch.cuda.get_device_properties(0)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def _bucket(x: float) -> int:
    """Power-of-two bucket, so similar workloads share an entry."""
    return int(round(math.log2(max(x, 1.0))))


def batch_signature(instances) -> str:
    """instances: objects with n, m, seeds, theta (graphgen.Instance)."""
    ns = [t.n for t in instances]
    deg = statistics.mean(t.m / max(t.n, 1) for t in instances)
    seeds = statistics.mean(len(t.seeds) for t in instances)
    theta = statistics.mean(t.theta for t in instances)
    return (f"batch/c{_bucket(len(instances))}/n{_bucket(statistics.median(ns))}"
            f"/d{_bucket(deg)}/s{_bucket(seeds)}/t{_bucket(theta)}")


def graph_signature(n: int, m: int, n_seeds: int, theta: int) -> str:
    return f"graph/n{_bucket(n)}/d{_bucket(m / max(n, 1))}/s{_bucket(n_seeds)}/t{_bucket(theta)}"


def _descend(grid: dict, start: dict, cost, max_passes: int = 3):
    """Coordinate descent: returns (best config, best cost, every (config, cost) timed)."""
    seen = {}

    def timed(cfg):
        k = tuple(sorted(cfg.items()))
        if k not in seen:
            seen[k] = cost(dict(cfg))
        return seen[k]

    best = dict(start)
    best_cost = timed(best)
    for _ in range(max_passes):
        improved = False
        for name, values in grid.items():
            for v in values:
                if v == best[name]:
                    continue
                cand = dict(best)
                cand[name] = v
                c = timed(cand)
                if c < best_cost:
                    best, best_cost, improved = cand, c, True
        if not improved:
            break
    return best, best_cost, [(dict(k), c) for k, c in seen.items()]


def tune_batch(problems, *, rounds: int = 1, repeats: int = 2, grid: dict | None = None):
    """problems: (handle, seeds, b, theta, seed) tuples as for imin_greedy_batch. Returns
    (best imin_launch fields, best kernel ms of the probe, table of all timings)."""
    grid = grid or BATCH_GRID
    probe = [(h, s, min(int(b), rounds), th, sd) for h, s, b, th, sd in problems]

    def cost(cfg):
        best = math.inf
        for _ in range(repeats):
            res = binding.imin_greedy_batch(probe, binding.IMIN_AG, cfg)
            best = min(best, res[0][1]["kernel_ms"])
        return best

    start = {k: v[len(v) // 2] for k, v in grid.items()}
    return _descend(grid, start, cost)


def tune_graph(graph, seeds, theta: int, *, repeats: int = 2, grid: dict | None = None):
    """graph: binding.Graph. Returns (best config, best kernel ms, table). The graph keeps
    the automatic policy afterwards; apply a result with ``apply_graph``."""
    grid = grid or GRAPH_GRID

    def cost(cfg):
        apply_graph(graph, cfg)
        best = math.inf
        for _ in range(repeats):
            _, st = graph.decrease(seeds, None, theta, 0)
            best = min(best, st["kernel_ms"])
        return best

    start = {k: v[len(v) // 2] for k, v in grid.items()}
    out = _descend(grid, start, cost)
    graph.set_small(-1)
    graph.set_launch(0, 0)
    return out


def apply_graph(graph, cfg: dict) -> None:
    graph.set_small(int(cfg["small"]), {k: cfg[k] for k in ("waves_per_cu", "quad_limit")
                                        if k in cfg})
    graph.set_launch(int(cfg.get("slots", 0)), 0)


def tuned_batch_launch(instances, problems=None, tune_if_missing: bool = False):
    """The cached launch shape for a batch like ``instances`` on this GPU; tunes (and caches)
    it with ``problems`` when there is none and ``tune_if_missing``; else None (defaults)."""
    key = f"{gpu_arch()}/{batch_signature(instances)}"
    entry = load_cache().get(key)
    if entry is None and tune_if_missing and problems is not None:
        best, ms, table = tune_batch(problems)
        entry = {"launch": best, "probe_kernel_ms": ms, "timed": len(table)}
        save(key, entry)
    return key, (entry or {}).get("launch")
