"""imin_spread (reachability-only sampling) and the evaluation harness on the GPU.

The reached-vertex sum is an integer, so it must equal the oracle's exactly; the spread
estimate is then checked against exact expected spreads from world enumeration.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2302_13529_amd import evaluate as ev
from paper_2302_13529_amd import graphgen as gg
from tests import helpers as H

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[case] {msg}", flush=True)


def test_spread_counts_equal_the_oracle_and_the_decrease_call(gpu):
    t = gg.tiny_plain()
    g = gpu.Graph(t.row_ptr, t.col, t.prob)
    rng = np.random.default_rng(3)
    blocked = np.zeros(t.n, np.uint8)
    pick = [v for v in rng.choice(t.n, 40, replace=False) if v not in t.seeds]
    blocked[pick] = 1
    for blk in (None, blocked):
        for enable in (-1, 0, 1):
            g.set_small(enable)
            case(f"tiny spread, blocked={blk is not None}, wave kernel {enable}")
            s, st = g.spread(t.seeds, blk, 3000, 17)
            _, so = orc.decrease(t.n, t.row_ptr, t.col, t.prob, t.seeds, blk, 3000, 17)
            assert st["reached"] == so["reached"] and st["samples"] == 3000
            assert st["edges_scanned"] == so["edges_scanned"]
            assert s == len(set(t.seeds.tolist())) + so["reached"] / 3000
            _, sd = g.decrease(t.seeds, blk, 3000, 17)
            assert sd["reached"] == st["reached"]
    g.close()


def test_spread_large_samples_and_handover(gpu):
    rp, c, p = H.csr_from_edges(300, [(i, i + 1, 1.0) for i in range(299)])
    g = gpu.Graph(rp, c, p)
    case("path 300, spread")
    s, st = g.spread([0], None, 100, 0)
    assert s == 300.0 and st["reached"] == 299 * 100
    g.close()


def test_spread_matches_exact_enumeration(gpu):
    rng = np.random.default_rng(11)
    for k in range(4):
        n = int(rng.integers(5, 12))
        rp, c, p = H.random_graph(rng, n, int(rng.integers(n, 3 * n)), probs=(0.2, 0.5, 0.8, 1.0))
        unc = int(np.sum((p > 0) & (p < 1)))
        if unc > 18:
            continue
        seeds = [int(rng.integers(0, n))]
        blocked = np.zeros(n, np.uint8)
        for v in rng.choice(n, size=n // 4, replace=False):
            if v not in seeds:
                blocked[v] = 1
        E, E2 = H.spread_moments(n, rp, c, p, seeds, blocked)
        g = gpu.Graph(rp, c, p)
        theta = 200000
        case(f"random graph {k}: n={n}, exact spread {E:.4f}")
        s, _ = g.spread(seeds, blocked, theta, 1000 + k)
        assert H.within_sigmas(s, E, E2, theta), (s, E)
        g.close()


def test_toy_spread_is_the_printed_value(gpu):
    n, row_ptr, col, prob, seeds, lines = H.toy_from_golden()
    g = gpu.Graph(row_ptr, col, prob)
    E, E2 = H.spread_moments(n, row_ptr, col, prob, seeds)
    s, _ = g.spread(seeds, None, 400000, 5)
    assert H.within_sigmas(s, E, E2, 400000)
    assert abs(E - 7.66) < 1e-6
    g.close()


def test_harness_orders_the_heuristics(gpu):
    """Table VII's qualitative result on a small synthetic graph: the greedy blockers leave
    a smaller spread than random ones."""
    t = gg.tiny_plain()
    case("tiny: RA / OD / AG / GR at b = 10, 20")
    rows = ev.compare(t, [10, 20], theta=2000, mc_rounds=20000)
    for r in rows:
        assert r["AG"] < r["RA"] and r["GR"] < r["RA"] and r["AG"] < r["no_blockers"]
        assert set(r) >= {"RA", "OD", "AG", "GR", "AG_seconds", "GR_seconds"}
    case("tiny: theta sweep")
    sweep = ev.theta_sweep(t, 10, [100, 1000], 20000)
    assert [r["theta"] for r in sweep] == [100, 1000]
    assert all(r["samples"] >= r["theta"] for r in sweep)
