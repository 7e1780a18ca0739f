"""Blocker sets and counters at the five benchmark configurations, against the oracle.

The expected values are the oracle's own full runs at each configuration's stated sizes
and budgets (tests/golden/config_*.txt, written by make_config_goldens.py from oracle/
alone): the library must reproduce every blocker, in order, and every work counter
bit-exactly.

* 2^17-vertex R-MAT, theta 10^4, b 100: AdvancedGreedy (Algorithm 3) and GreedyReplace
  (Algorithm 4) in full.
* 256 Chung-Lu instances, theta 2000, b 20: all 20 rounds of every instance in one batched
  call, and every instance's plain call.
* 2^22-vertex R-MAT: Algorithm 2 at theta 2048 (a SHA-256 digest of all 4M counts), and
  AdvancedGreedy rounds 0 and 1 at theta 10^4.
* 2^20-vertex R-MAT served: a seeded subset of 20 queries at their full seeds, budget and
  theta, run together in the server.
"""
import hashlib

import numpy as np
import pytest

from paper_2302_13529_amd import graphgen as gg
from tests import helpers as H

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[case] {msg}", flush=True)


def _stats(st):
    return {k: st[k] for k in ("samples", "reached", "edges_scanned", "live_edges")}


@pytest.mark.parametrize("mode_name", ["ag", "gr"])
def test_rmat17_greedy_b100_theta1e4(gpu, mode_name):
    want = H.read_config_golden(f"config_c2_{mode_name}.txt")
    t = H.cached("rmat17", gg.rmat_plain)
    mode = gpu.IMIN_AG if mode_name == "ag" else gpu.IMIN_GR
    g = gpu.Graph(t.row_ptr, t.col, t.prob)
    case(f"rmat17 {mode_name.upper()} b={t.b} theta={t.theta}")
    B, st = g.greedy(t.seeds, t.b, t.theta, t.seed, mode)
    g.close()
    assert [int(x) for x in B] == want["blockers"]
    assert _stats(st) == want["stats"]
    assert st["samples"] == want["calls"] * t.theta


def test_batch256_all_rounds(gpu):
    want = H.read_config_golden("config_c3.txt")
    insts = H.cached("batch256", gg.batched_instances)
    graphs = [gpu.Graph(t.row_ptr, t.col, t.prob) for t in insts]
    probs = [(g.handle, t.seeds, t.b, t.theta, t.seed) for g, t in zip(graphs, insts)]
    case("batched AG over 256 instances, theta 2000, b 20")
    res = gpu.imin_greedy_batch(probs)
    for i, (B, st) in enumerate(res):
        wB, wst = want[("inst", i)]
        assert [int(x) for x in B] == wB, i
        assert _stats(st) == wst, i
    case("the same 256 instances, one plain call each")
    for i, (g, t) in enumerate(zip(graphs, insts)):
        B, st = g.greedy(t.seeds, t.b, t.theta, t.seed, gpu.IMIN_AG)
        wB, wst = want[("inst", i)]
        assert [int(x) for x in B] == wB and _stats(st) == wst, i
    for g in graphs:
        g.close()


def test_rmat22_theta2048_counts_and_two_rounds(gpu):
    want = H.read_config_golden("config_c4.txt")
    t = H.cached("rmat22", gg.large_plain)
    case("rmat22 graph upload")
    g = gpu.Graph(t.row_ptr, t.col, t.prob)
    case("rmat22 decrease, theta 2048, key 0")
    D, st = g.decrease(t.seeds, None, 2048, 0)
    d = want["decrease2048"]
    top = [(v, int(D[v])) for v, _ in d["top"]]
    assert top == d["top"]
    assert _stats(st) == d["stats"]
    assert hashlib.sha256(np.ascontiguousarray(D, dtype="<u8").tobytes()).hexdigest() == d["sha256"]
    case("rmat22 AG rounds 0 and 1, theta 10^4")
    B, st = g.greedy(t.seeds, 2, t.theta, t.seed, gpu.IMIN_AG)
    g.close()
    w = want["greedy2"]
    assert [int(x) for x in B] == w["blockers"]
    assert _stats(st) == w["stats"]


def test_served_subset_full_budgets(gpu):
    want = H.read_config_golden("config_c5.txt")
    t = H.cached("rmat20", gg.served_graph)
    qs = gg.served_queries(t.n)
    idx = sorted(i for kind, i in want if kind == "query")
    assert len(idx) == 20
    g = gpu.Graph(t.row_ptr, t.col, t.prob)
    srv = gpu.Server(g, hbm_budget=8 << 30, max_active=12, max_theta=10000)
    # the 20 checked queries arrive interleaved with their neighbours in the mix
    mix = sorted(set(idx) | {i + 1 for i in idx if i + 1 < len(qs)})
    tickets = {i: srv.submit(qs[i]["seeds"], qs[i]["b"], qs[i]["theta"], qs[i]["seed"])
               for i in mix}
    case(f"server: {len(mix)} queries of the served mix, at most 12 at a time")
    steps = 0
    while srv.step() != (0, 0):
        steps += 1
    for i in idx:
        B, st = srv.result(tickets[i], qs[i]["b"])
        wB, wst = want[("query", i)]
        assert [int(x) for x in B] == wB, i
        assert _stats(st) == wst, i
    srv.close()
    g.close()


def test_rmat17_greedy_replace_batched_and_served(gpu):
    """GreedyReplace at b = 100, theta = 10^4 on the 2^17-vertex R-MAT graph through the
    batched call (a batch with a second, smaller instance) and through the server, against
    the oracle's full run."""
    want = H.read_config_golden("config_c2_gr.txt")
    t = H.cached("rmat17", gg.rmat_plain)
    g = gpu.Graph(t.row_ptr, t.col, t.prob)
    tiny = gg.tiny_plain()
    g2 = gpu.Graph(tiny.row_ptr, tiny.col, tiny.prob)
    case("rmat17 GR b=100 theta=10^4 in a batch of two")
    res = gpu.imin_greedy_batch([(g.handle, t.seeds, t.b, t.theta, t.seed),
                                 (g2.handle, tiny.seeds, 3, 500, 2)], gpu.IMIN_GR)
    B, st = res[0]
    assert [int(x) for x in B] == want["blockers"]
    assert _stats(st) == want["stats"]
    case("rmat17 GR b=100 theta=10^4 in the server, beside an AG query")
    srv = gpu.Server(g, hbm_budget=2 << 30, max_active=4, max_theta=10000)
    tk = srv.submit(t.seeds, t.b, t.theta, t.seed, mode=gpu.IMIN_GR)
    tk2 = srv.submit(t.seeds[:3], 5, 2000, 9)
    while srv.step() != (0, 0):
        pass
    B, st = srv.result(tk, t.b)
    assert [int(x) for x in B] == want["blockers"]
    assert _stats(st) == want["stats"]
    B2, _ = srv.result(tk2, 5)
    B2p, _ = g.greedy(t.seeds[:3], 5, 2000, 9, gpu.IMIN_AG)
    assert list(B2) == list(B2p)
    srv.close()
    g.close()
    g2.close()
