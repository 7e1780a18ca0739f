"""Write the oracle's results at the five benchmark configurations as text fixtures.

Every value written here comes from ``oracle/`` (the plain CPU oracle, its threaded
variant spreading each Algorithm 2 call's samples over host threads) applied to the seeded
synthetic inputs of ``paper_2302_13529_amd.graphgen``; nothing is read from the GPU
library. The GPU tests compare the library's results against these files bit-exactly.

    python tests/golden/make_config_goldens.py c3 c5 c4 c2ag c2gr [--threads 8]

Configurations (blocker choice by Algorithm 3 / Algorithm 4, budgets per the benchmark):
  c2ag  AdvancedGreedy on the 2^17-vertex R-MAT graph, top-10 seeds, theta 10^4, b 100
  c2gr  GreedyReplace on the same input
  c3    AdvancedGreedy on each of the 256 Chung-Lu instances, theta 2000, b 20
  c4    the 2^22-vertex R-MAT graph, top-100 seeds: Algorithm 2 at theta 2048 (key 0, no
        blockers; the counts as a SHA-256 digest), and AdvancedGreedy rounds 0 and 1 at
        theta 10^4
  c5    a seeded subset of 20 of the 2000 served queries on the 2^20-vertex R-MAT graph,
        each by AdvancedGreedy at its full seed set, budget and theta
"""
from __future__ import annotations

import argparse
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as orc  # noqa: E402
from paper_2302_13529_amd import graphgen as gg  # noqa: E402

C5_SUBSET_SEED = 2000
C5_SUBSET_SIZE = 20


def c5_subset(count: int = 2000):
    """The indices of the served queries checked against the oracle (sorted)."""
    rng = np.random.default_rng(C5_SUBSET_SEED)
    return sorted(int(i) for i in rng.choice(count, size=C5_SUBSET_SIZE, replace=False))


def stats_line(st: dict) -> str:
    return " ".join(f"{k}={st[k]}" for k in ("samples", "reached", "edges_scanned", "live_edges"))


def d_digest(D: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(D, dtype="<u8").tobytes()).hexdigest()


def write(name: str, header: list, lines: list) -> None:
    path = os.path.join(HERE, name)
    with open(path + ".tmp", "w") as f:
        for h in header:
            f.write(f"# {h}\n")
        f.write("# written by tests/golden/make_config_goldens.py (calls only oracle/)\n")
        for line in lines:
            f.write(line + "\n")
    os.replace(path + ".tmp", path)
    print(f"wrote {path}", flush=True)


def greedy_lines(inst, b, theta, seed, mode, threads):
    B, calls, st = orc.greedy(inst.n, inst.row_ptr, inst.col, inst.prob, inst.seeds, b, theta,
                              seed, mode, threads=threads)
    return [f"blockers {' '.join(str(int(x)) for x in B)}", f"calls {calls}",
            f"stats {stats_line(st)}"]


def make_c2(mode: int, threads: int) -> None:
    inst = gg.rmat_plain()
    name = "AdvancedGreedy (Algorithm 3)" if mode == orc.AG else "GreedyReplace (Algorithm 4)"
    lines = greedy_lines(inst, inst.b, inst.theta, inst.seed, mode, threads)
    write("config_c2_" + ("ag" if mode == orc.AG else "gr") + ".txt",
          [f"{name} on {inst.name}: n={inst.n} m={inst.m}, top-10 out-degree seeds, "
           f"theta={inst.theta}, b={inst.b}, Philox seed {inst.seed}"], lines)


def make_c3(threads: int) -> None:
    insts = gg.batched_instances()
    lines = []
    for i, t in enumerate(insts):
        B, calls, st = orc.greedy(t.n, t.row_ptr, t.col, t.prob, t.seeds, t.b, t.theta, t.seed,
                                  orc.AG, threads=threads)
        lines.append(f"inst {i} blockers {' '.join(str(int(x)) for x in B)} | {stats_line(st)}")
    write("config_c3.txt", ["AdvancedGreedy (Algorithm 3) on each of the 256 batched Chung-Lu "
                            "instances (TR), theta=2000, b=20, instance i with Philox seed i"],
          lines)


def make_c4(threads: int) -> None:
    inst = gg.large_plain()
    D, st = orc.decrease(inst.n, inst.row_ptr, inst.col, inst.prob, inst.seeds, None, 2048, 0,
                         threads=threads)
    top = np.argsort(-D.astype(np.int64), kind="stable")[:10]
    lines = [f"decrease2048 sha256 {d_digest(D)}", f"decrease2048 stats {stats_line(st)}",
             "decrease2048 top " + " ".join(f"{int(v)}:{int(D[v])}" for v in top)]
    lines += ["greedy2 " + x for x in greedy_lines(inst, 2, inst.theta, inst.seed, orc.AG,
                                                    threads)]
    write("config_c4.txt", [f"{inst.name}: n={inst.n} m={inst.m}, top-100 out-degree seeds",
                            "decrease2048: Algorithm 2 with theta=2048, key 0, no blockers; "
                            "sha256 of the counts as little-endian uint64[n]",
                            "greedy2: AdvancedGreedy rounds 0 and 1 at theta=10000, seed 0"],
          lines)


def make_c5(threads: int) -> None:
    inst = gg.served_graph()
    qs = gg.served_queries(inst.n)
    lines = []
    for i in c5_subset(len(qs)):
        q = qs[i]
        t0 = time.time()
        B, calls, st = orc.greedy(inst.n, inst.row_ptr, inst.col, inst.prob, q["seeds"], q["b"],
                                  q["theta"], q["seed"], orc.AG, threads=threads)
        lines.append(f"query {i} blockers {' '.join(str(int(x)) for x in B)} | {stats_line(st)}")
        print(f"query {i}: |S|={len(q['seeds'])} b={q['b']} theta={q['theta']} "
              f"{time.time() - t0:.1f} s", flush=True)
    write("config_c5.txt", [f"AdvancedGreedy (Algorithm 3) for {C5_SUBSET_SIZE} of the "
                            f"{len(qs)} served queries on {inst.name} (n={inst.n} m={inst.m}), "
                            f"chosen by numpy default_rng({C5_SUBSET_SEED}), each at its full "
                            "seed set, budget and theta, Philox seed = query index"], lines)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("configs", nargs="+", choices=["c2ag", "c2gr", "c3", "c4", "c5"])
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    for c in args.configs:
        t0 = time.time()
        if c == "c2ag":
            make_c2(orc.AG, args.threads)
        elif c == "c2gr":
            make_c2(orc.GR, args.threads)
        elif c == "c3":
            make_c3(args.threads)
        elif c == "c4":
            make_c4(args.threads)
        else:
            make_c5(args.threads)
        print(f"{c}: {time.time() - t0:.0f} s", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
