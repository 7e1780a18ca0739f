"""Evaluation harness: the effectiveness experiments of arXiv 2302.13529 on synthetic graphs.

* ``rand_blockers`` / ``outdegree_blockers`` -- the two heuristic baselines of Section VI-A
  ("Algorithms"): RA picks b blockers uniformly at random among the non-seed vertices, OD
  the b non-seed vertices of largest out-degree (ties to the smaller id).
* ``compare`` -- the experiment behind Table VII (Section VI-B, "Comparison with
  Heuristics"): seeds fixed, budgets varied, and the expected spread left by the blockers
  of RA, OD, AdvancedGreedy and GreedyReplace, each estimated by Monte-Carlo simulation
  (10^5 rounds in the paper; here live-edge samples, which Lemma 1 shows are equivalent)
  with a key independent of the keys used to choose the blockers.
* ``theta_sweep`` -- Section VI-B, "Varying the Number of Sampled Graphs": GreedyReplace
  with theta in {10^3, 10^4, 10^5}, its spread and running time.

Every estimate runs on the GPU through the library (``imin_greedy``, ``imin_spread``). The
datasets of Table IV are not available here; the graphs come from ``graphgen``.

Command line: ``python -m paper_2302_13529_amd.evaluate --workload rmat17 --budgets 20 40``
prints one JSON object per measured row.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import binding, graphgen as gg

EVAL_KEY = 0x5EED_0000_0000  # Philox key base of the spread estimates, apart from selection


def rand_blockers(n: int, seeds, b: int, rng_seed: int) -> np.ndarray:
    """RA: b distinct non-seed vertices, uniformly at random (seeded)."""
    seeds = set(int(s) for s in seeds)
    pool = np.array([v for v in range(n) if v not in seeds], dtype=np.int32)
    rng = np.random.default_rng(rng_seed)
    k = min(b, pool.shape[0])
    return np.sort(rng.choice(pool, size=k, replace=False)).astype(np.int32)


def outdegree_blockers(row_ptr, seeds, b: int) -> np.ndarray:
    """OD: the b non-seed vertices with the largest out-degree, ties to the smaller id."""
    deg = np.diff(np.asarray(row_ptr, dtype=np.int64))
    order = np.lexsort((np.arange(deg.shape[0]), -deg))
    seeds = set(int(s) for s in seeds)
    out = [int(v) for v in order if int(v) not in seeds][:b]
    return np.asarray(out, dtype=np.int32)


def blocked_mask(n: int, blockers) -> np.ndarray:
    m = np.zeros(n, dtype=np.uint8)
    m[np.asarray(blockers, dtype=np.int64)] = 1
    return m


def spread(graph: binding.Graph, seeds, blockers, rounds: int, key: int = EVAL_KEY):
    """Expected spread left by `blockers`, from `rounds` live-edge samples drawn in calls of
    at most 2^20 samples (each call its own key). Returns (estimate, per-call estimates)."""
    per = []
    done = 0
    while done < rounds:
        t = min(rounds - done, 1 << 20)
        s, _ = graph.spread(seeds, blocked_mask(graph.n, blockers), t, key + len(per))
        per.append((s, t))
        done += t
    return sum(s * t for s, t in per) / rounds, per


def compare(inst: gg.Instance, budgets, theta: int, mc_rounds: int, rng_seed: int = 0):
    """Rows of the Table VII experiment for one seed set: spread left by RA, OD, AG, GR."""
    g = binding.Graph(inst.row_ptr, inst.col, inst.prob)
    rows = []
    base, _ = spread(g, inst.seeds, [], mc_rounds)
    for b in budgets:
        row = {"workload": inst.name, "b": int(b), "theta": int(theta), "mc_rounds": mc_rounds,
               "no_blockers": base}
        choices = {
            "RA": rand_blockers(inst.n, inst.seeds, b, rng_seed),
            "OD": outdegree_blockers(inst.row_ptr, inst.seeds, b),
        }
        for name, mode in (("AG", binding.IMIN_AG), ("GR", binding.IMIN_GR)):
            t0 = time.perf_counter()
            B, st = g.greedy(inst.seeds, b, theta, inst.seed, mode)
            row[f"{name}_seconds"] = time.perf_counter() - t0
            choices[name] = B
        for name, B in choices.items():
            row[name], _ = spread(g, inst.seeds, B, mc_rounds)
        rows.append(row)
    g.close()
    return rows


def theta_sweep(inst: gg.Instance, b: int, thetas, mc_rounds: int, mode=binding.IMIN_GR):
    """GreedyReplace (default) at several theta: spread of its blockers and its time."""
    g = binding.Graph(inst.row_ptr, inst.col, inst.prob)
    rows = []
    for theta in thetas:
        t0 = time.perf_counter()
        B, st = g.greedy(inst.seeds, b, theta, inst.seed, mode)
        dt = time.perf_counter() - t0
        s, _ = spread(g, inst.seeds, B, mc_rounds)
        rows.append({"workload": inst.name, "b": int(b), "theta": int(theta),
                     "mode": "GR" if mode == binding.IMIN_GR else "AG", "spread": s,
                     "seconds": dt, "samples": st["samples"], "blockers": [int(x) for x in B]})
    g.close()
    return rows


def _workload(name: str) -> gg.Instance:
    return {"tiny": gg.tiny_plain, "rmat17": gg.rmat_plain, "rmat22": gg.large_plain}[name]()


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--workload", default="rmat17", choices=["tiny", "rmat17", "rmat22"])
    ap.add_argument("--budgets", type=int, nargs="+", default=[20, 40, 60, 80, 100])
    ap.add_argument("--theta", type=int, default=10000)
    ap.add_argument("--mc-rounds", type=int, default=100000)
    ap.add_argument("--sweep", type=int, nargs="*", default=[],
                    help="theta values for the sweep (GR at the first budget)")
    args = ap.parse_args(argv)
    inst = _workload(args.workload)
    for row in compare(inst, args.budgets, args.theta, args.mc_rounds):
        print(json.dumps(row), flush=True)
    if args.sweep:
        for row in theta_sweep(inst, args.budgets[0], args.sweep, args.mc_rounds):
            print(json.dumps(row), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
