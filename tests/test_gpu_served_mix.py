"""The full 2,000-query served mix on the 2^20-vertex R-MAT graph: every query's blockers and
work counters are the same in two different mixes (all submitted at once with up to 256
admitted, and in reverse order with up to 48 admitted), and equal a plain imin_greedy call
alone for a seeded subset of 200 queries (the seeded 20-query subset is checked against the
oracle's full runs in test_gpu_configs.py)."""
import numpy as np
import pytest

from paper_2302_13529_amd import graphgen as gg
from tests import helpers as H

pytestmark = pytest.mark.gpu

KEYS = ("samples", "reached", "edges_scanned", "live_edges")


def case(msg):
    print(f"[case] {msg}", flush=True)


def _serve(gpu, g, qs, order, max_active):
    srv = gpu.Server(g, hbm_budget=16 << 30, max_active=max_active, max_theta=10000)
    tickets = {i: srv.submit(qs[i]["seeds"], qs[i]["b"], qs[i]["theta"], qs[i]["seed"])
               for i in order}
    steps = 0
    while srv.step() != (0, 0):
        steps += 1
        if steps % 200 == 0:
            case(f"  step {steps}")
    out = {i: srv.result(t, qs[i]["b"]) for i, t in tickets.items()}
    srv.close()
    return out


@pytest.mark.timeout(900)
def test_full_served_mix_alone_and_in_two_mixes(gpu):
    t = H.cached("rmat20", gg.served_graph)
    qs = gg.served_queries(t.n)
    g = gpu.Graph(t.row_ptr, t.col, t.prob)
    case("2000 queries submitted at once, up to 256 admitted")
    a = _serve(gpu, g, qs, range(len(qs)), 256)
    case("2000 queries in reverse order, up to 48 admitted")
    b = _serve(gpu, g, qs, reversed(range(len(qs))), 48)
    for i in range(len(qs)):
        assert list(a[i][0]) == list(b[i][0]), i
        assert {k: a[i][1][k] for k in KEYS} == {k: b[i][1][k] for k in KEYS}, i
    rng = np.random.default_rng(2001)
    subset = sorted(int(i) for i in rng.choice(len(qs), size=200, replace=False))
    case("200 of them alone, one plain call each")
    for i in subset:
        q = qs[i]
        B, st = g.greedy(q["seeds"], q["b"], q["theta"], q["seed"], gpu.IMIN_AG)
        assert list(B) == list(a[i][0]), i
        assert {k: st[k] for k in KEYS} == {k: a[i][1][k] for k in KEYS}, i
    g.close()
