"""The served form and the 2^17-vertex R-MAT graph at their full input sizes, against the
oracle run live (the stored full-budget results are in test_gpu_configs.py).

C5: the 1M-vertex R-MAT graph with a mix of queries in the server, each against the
oracle. C2: one Algorithm 2 call at theta = 10^4, every count against the oracle.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2302_13529_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[case] {msg}", flush=True)


def test_served_graph_full_size(gpu):
    case("generating the served graph (2^20 vertices, 8M edges)")
    inst = gg.served_graph()
    qs = gg.served_queries(inst.n, count=20, seed=6)
    # the first queries of the mix, with budgets and samples cut so the oracle keeps up
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
    every count against the oracle (about a minute of oracle time)."""
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
