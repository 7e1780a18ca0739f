"""More pins of the oracle: its work counters, its linear-threshold interval bounds, and its
threaded variant.

* Work counters (Algorithm 2's loop over sampled graphs): with every probability 0 or 1
  each sample is the same graph, so per sample the edges scanned are the out-edges of the
  seeds and of every reached vertex, the live edges are the certain ones among them whose
  target is neither a seed nor blocked (Definition 2), and the counters are theta times
  that. The expected values come from a plain breadth-first search written here.
* Linear-threshold bounds (Section V-E): the interval upper ends min(2^24, ceil(2^24 *
  (w_1 + ... + w_k))) of each vertex's in-edges, against exact rational arithmetic on the
  fp32 weights; the weights are chosen so that a running sum kept in fp32 would give
  different bounds, and so a fp32 slip cannot pass. The choice made from a 24-bit draw R is
  pinned at an interval edge (R equal to a bound is outside that interval).
* Threaded variant: Algorithm 2's samples are independent, so spreading them over host
  threads must give bit-identical counts, counters and greedy choices.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as orc
from tests import helpers as H


def _certain_graph(rng, n, m):
    return H.random_graph(rng, n, m, probs=(0.0, 1.0, 1.0), allow_loops=True, allow_dups=True)


def _expected_counters(n, row_ptr, col, prob, seeds, blocked):
    """(reached non-seeds, edges scanned, live edges) of the one deterministic sample."""
    removed = np.zeros(n, bool) if blocked is None else np.asarray(blocked, bool)
    live = np.asarray(prob) >= 1.0
    r = H.reach(n, row_ptr, col, live, seeds, removed)
    is_seed = np.zeros(n, bool)
    is_seed[list(seeds)] = True
    scanned = live_n = 0
    for u in range(n):
        if not r[u]:
            continue
        for e in range(row_ptr[u], row_ptr[u + 1]):
            scanned += 1
            v = col[e]
            if live[e] and not is_seed[v] and not removed[v]:
                live_n += 1
    return int(r.sum() - is_seed.sum()), scanned, live_n


@pytest.mark.parametrize("trial", range(30))
def test_work_counters_closed_form_on_certain_graphs(trial):
    rng = np.random.default_rng(900 + trial)
    n = int(rng.integers(2, 40))
    m = int(rng.integers(0, 4 * n))
    row_ptr, col, prob = _certain_graph(rng, n, m)
    k = int(rng.integers(1, min(n, 5) + 1))
    seeds = [int(x) for x in rng.choice(n, size=k, replace=False)]
    seeds = seeds + seeds[:1]  # a repeated seed counts once
    blocked = None
    if trial % 3 == 1:
        blocked = (rng.random(n) < 0.2).astype(np.uint8)
        blocked[seeds] = 0
    theta = int(rng.integers(1, 9))
    reached, scanned, live = _expected_counters(n, row_ptr, col, prob, set(seeds), blocked)
    _, st = orc.decrease(n, row_ptr, col, prob, seeds, blocked, theta, trial)
    assert st["samples"] == theta
    assert st["reached"] == theta * reached
    assert st["edges_scanned"] == theta * scanned
    assert st["live_edges"] == theta * live


def test_work_counters_closed_form_linear_threshold():
    """LT with weights in {0, 1}: a vertex keeps its weight-1 in-edge in every sample."""
    rng = np.random.default_rng(77)
    for trial in range(20):
        n = int(rng.integers(3, 30))
        edges = []
        for v in range(n):
            k = int(rng.integers(0, 4))
            srcs = rng.integers(0, n, size=k)
            one = int(rng.integers(-1, k)) if k else -1  # at most one certain in-edge
            for i, u in enumerate(srcs):
                edges.append((int(u), v, 1.0 if i == one else 0.0))
        row_ptr, col, w = H.csr_from_edges(n, edges)
        seeds = [int(x) for x in rng.choice(n, size=2, replace=False)]
        reached, scanned, live = _expected_counters(n, row_ptr, col, w, set(seeds), None)
        _, st = orc.decrease(n, row_ptr, col, w, seeds, None, 3, trial, model=orc.LT)
        assert (st["reached"], st["edges_scanned"], st["live_edges"]) == \
            (3 * reached, 3 * scanned, 3 * live)


def _lt_graph(rng, n, max_in):
    """Random in-edges with non-dyadic fp32 weights that sum to at most 1 per vertex."""
    edges = []
    for v in range(n):
        k = int(rng.integers(1, max_in + 1))
        raw = rng.random(k) + 0.05
        scale = rng.uniform(0.5, 1.0) / raw.sum()
        for u, x in zip(rng.integers(0, n, size=k), raw * scale):
            edges.append((int(u), v, float(np.float32(x))))
    return H.csr_from_edges(n, edges)


def _exact_bounds(weights):
    out, s = [], Fraction(0)
    for x in weights:
        s += Fraction(float(x))
        b = -((-s * 2**24).numerator // (s * 2**24).denominator)  # ceil
        out.append(min(2**24, b))
    return out


def _fp32_bounds(weights):
    out, s = [], np.float32(0)
    for x in weights:
        s = np.float32(s + np.float32(x))
        out.append(min(2**24, int(np.ceil(np.float64(s) * 2**24))))
    return out


def test_lt_bounds_match_exact_rationals():
    rng = np.random.default_rng(31)
    n = 300
    row_ptr, col, w = _lt_graph(rng, n, 7)
    differs = 0
    for u in range(n):
        ins = [e for e in range(len(col)) if col[e] == u]  # ascending edge id
        ws = [w[e] for e in ins]
        got = [int(x) for x in orc.lt_bounds(n, row_ptr, col, w, u)]
        assert got == _exact_bounds(ws), u
        differs += got != _fp32_bounds(ws)
    # a running sum kept in fp32 would have failed on these weights
    assert differs > 0


def test_lt_choice_follows_exact_intervals():
    """The choice of u in sample j is the in-edge whose [bound_{k-1}, bound_k) holds R, with R
    from the pinned Philox word (u & 3) at counter (u >> 2, j, 1, 0)."""
    rng = np.random.default_rng(32)
    n = 64
    row_ptr, col, w = _lt_graph(rng, n, 5)
    key = 0x1234_5678_9ABC
    for u in range(n):
        ins = [e for e in range(len(col)) if col[e] == u]
        bounds = _exact_bounds([w[e] for e in ins])
        for j in range(40):
            R = int(orc.philox((u >> 2, j, 1, 0), (key & 0xFFFFFFFF, key >> 32))[u & 3]) >> 8
            want, lo = -1, 0
            for e, hi in zip(ins, bounds):
                if lo <= R < hi:
                    want = e
                    break
                lo = hi
            assert orc.lt_trigger(n, row_ptr, col, w, key, j, u) == want, (u, j)


def test_lt_choice_at_an_interval_edge():
    """A weight whose bound equals R leaves R outside; one fp32 ulp more takes it in."""
    key, j, u = 5, 3, 1
    R = int(orc.philox((u >> 2, j, 1, 0), (key, 0))[u & 3]) >> 8
    row_ptr, col, _ = H.csr_from_edges(2, [(0, 1, 0.0)])
    exact = np.float32(R / 2**24)  # exactly representable: R < 2^24
    above = np.nextafter(exact, np.float32(1))
    assert orc.lt_trigger(2, row_ptr, col, np.array([exact], np.float32), key, j, u) == -1
    assert orc.lt_trigger(2, row_ptr, col, np.array([above], np.float32), key, j, u) == 0


def _random_problem(rng, model):
    n = int(rng.integers(5, 60))
    if model == orc.LT:
        row_ptr, col, p = _lt_graph(rng, n, 4)
    else:
        row_ptr, col, p = H.random_graph(rng, n, int(rng.integers(n, 5 * n)),
                                         probs=(0.1, 0.3, 0.5, 0.9, 1.0))
    seeds = [int(x) for x in rng.choice(n, size=int(rng.integers(1, 4)), replace=False)]
    blocked = (rng.random(n) < 0.1).astype(np.uint8)
    blocked[seeds] = 0
    return n, row_ptr, col, p, seeds, blocked


@pytest.mark.parametrize("model", [orc.IC, orc.LT])
def test_threaded_decrease_equals_single_thread(model):
    rng = np.random.default_rng(41 + model)
    for trial in range(12):
        n, row_ptr, col, p, seeds, blocked = _random_problem(rng, model)
        theta = [1, 2, 7, 37, 200, 513][trial % 6]
        threads = [2, 3, 8, 16][trial % 4]
        key = int(rng.integers(0, 2**63))
        D1, s1 = orc.decrease(n, row_ptr, col, p, seeds, blocked, theta, key, model=model)
        Dt, st = orc.decrease(n, row_ptr, col, p, seeds, blocked, theta, key, model=model,
                              threads=threads)
        assert np.array_equal(D1, Dt) and s1 == st, (trial, theta, threads)


@pytest.mark.parametrize("mode", [orc.AG, orc.GR])
def test_threaded_greedy_equals_single_thread(mode):
    rng = np.random.default_rng(51 + mode)
    for trial in range(8):
        n, row_ptr, col, p, seeds, _ = _random_problem(rng, orc.IC)
        b = int(rng.integers(0, 6))
        theta = int(rng.integers(1, 120))
        one = orc.greedy(n, row_ptr, col, p, seeds, b, theta, trial, mode)
        many = orc.greedy(n, row_ptr, col, p, seeds, b, theta, trial, mode, threads=5)
        assert list(one[0]) == list(many[0]) and one[1:] == many[1:], trial


def test_threaded_decrease_on_a_larger_graph():
    """Several samples per thread on a 2,000-vertex power-law graph (TR probabilities)."""
    from paper_2302_13529_amd import graphgen as gg
    rng = np.random.default_rng(61)
    n = 2000
    src, dst = gg.chung_lu_edges(n, 16000, 2.5, rng)
    row_ptr, col = gg.to_csr(n, src, dst)
    p = gg.tr_probs(col.shape[0], rng) * np.float32(5)
    seeds = gg.uniform_seeds(n, 20, rng)
    D1, s1 = orc.decrease(n, row_ptr, col, p, seeds, None, 300, 9)
    D8, s8 = orc.decrease(n, row_ptr, col, p, seeds, None, 300, 9, threads=8)
    assert s1["reached"] > 300 and np.array_equal(D1, D8) and s1 == s8
