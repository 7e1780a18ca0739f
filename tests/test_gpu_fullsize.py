"""The batched and served forms at their full input sizes.

C3: all 256 Chung-Lu instances in one batched call (theta = 2000, two rounds here), every
instance against its plain call and a seeded subset against the checker. C5: the
1M-vertex R-MAT graph with a mix of queries in the server, each against the checker.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2302_13529_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[case] {msg}", flush=True)


def test_batch_of_256_full_size(gpu):
    case("generating the 256 batched instances")
    insts = gg.batched_instances()
    graphs = [gpu.Graph(t.row_ptr, t.col, t.prob) for t in insts]
    probs = [(g.handle, t.seeds, 2, t.theta, t.seed) for g, t in zip(graphs, insts)]
    case("batched AG over 256 instances, theta 2000, 2 rounds")
    res = gpu.imin_greedy_batch(probs)
    assert sum(st["samples"] for _, st in res) == 256 * 2 * 2000
    rng = np.random.default_rng(256)
    check = set(int(i) for i in rng.choice(256, size=12, replace=False))
    for i, (g, t) in enumerate(zip(graphs, insts)):
        B, st = res[i]
        Bp, sp = g.greedy(t.seeds, 2, t.theta, t.seed, gpu.IMIN_AG)
        assert list(B) == list(Bp), i
        assert st["reached"] == sp["reached"] and st["live_edges"] == sp["live_edges"], i
        if i in check:
            case(f"instance {i} (n={t.n}) against the checker")
            Bo, _, so = orc.greedy(t.n, t.row_ptr, t.col, t.prob, t.seeds, 2, t.theta, t.seed, 0)
            assert list(B) == list(Bo) and st["reached"] == so["reached"], i
    for g in graphs:
        g.close()


def test_served_graph_full_size(gpu):
    case("generating the served graph (2^20 vertices, 8M edges)")
    inst = gg.served_graph()
    qs = gg.served_queries(inst.n, count=20, seed=6)
    # the first queries of the mix, with budgets and samples cut so the checker keeps up
    mix = [dict(seeds=q["seeds"], b=min(q["b"], 3), theta=min(q["theta"], 500), seed=q["seed"])
           for q in qs[:8]]
    g = gpu.Graph(inst.row_ptr, inst.col, inst.prob)
    srv = gpu.Server(g, hbm_budget=4 << 30, max_active=5, max_theta=500)
    tickets = [srv.submit(q["seeds"], q["b"], q["theta"], q["seed"]) for q in mix]
    case("server: 8 queries, at most 5 at a time")
    while srv.step() != (0, 0):
        pass
    for q, tk in zip(mix, tickets):
        B, st = srv.result(tk, q["b"])
        Bo, _, so = orc.greedy(inst.n, inst.row_ptr, inst.col, inst.prob, q["seeds"], q["b"],
                               q["theta"], q["seed"], 0)
        assert list(B) == list(Bo) and st["reached"] == so["reached"]
        assert st["edges_scanned"] == so["edges_scanned"]
    srv.close()
    g.close()


def test_rmat17_full_theta_round(gpu):
    """C2 at full size: one Algorithm 2 call with theta = 10^4 on the 131k-vertex R-MAT graph,
    every count against the checker (about a minute of checker time)."""
    t = gg.rmat_plain()
    g = gpu.Graph(t.row_ptr, t.col, t.prob)
    case("rmat17 decrease, theta 10^4")
    D, st = g.decrease(t.seeds, None, t.theta, 0)
    Do, so = orc.decrease(t.n, t.row_ptr, t.col, t.prob, t.seeds, None, t.theta, 0)
    assert np.array_equal(D, Do)
    for k in ("samples", "reached", "edges_scanned", "live_edges"):
        assert st[k] == so[k], k
    # the first greedy round blocks the argmax of these counts (ties to the smaller id)
    B, _ = g.greedy(t.seeds, 1, t.theta, 0, gpu.IMIN_AG)
    cand = np.ones(t.n, bool)
    cand[t.seeds] = False
    best = int(np.flatnonzero(cand)[np.argmax(Do[cand])])
    assert int(B[0]) == best
    g.close()
