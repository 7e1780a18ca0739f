"""Pins of the oracle's linear-threshold (triggering-model) sampling, Section V-E.

Under LT a vertex keeps at most one in-edge per sample (its triggering set), chosen with
probability equal to the edge's weight. Pinned here against: closed forms that tell LT from
IC apart, exact enumeration of all triggering-set worlds on small graphs (Lemma 1,
Theorem 4), choice frequencies for dyadic weights, vertex-deletion brute force on
reconstructed samples (Theorem 6), and the one-live-in-edge invariant.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as orc
from tests import helpers as H


def _in_edges(n, row_ptr, col):
    ins = [[] for _ in range(n)]
    for u in range(n):
        for e in range(row_ptr[u], row_ptr[u + 1]):
            ins[col[e]].append(e)
    return ins


def _lt_options(n, row_ptr, col, w):
    """Per vertex: list of (chosen in-edge or -1, probability) with dyadic-exact weights."""
    ins = _in_edges(n, row_ptr, col)
    opts = []
    for v in range(n):
        o = [(e, float(w[e])) for e in ins[v]]
        rest = 1.0 - sum(p for _, p in o)
        if rest > 1e-12:
            o.append((-1, rest))
        opts.append(o)
    return opts


def _exact_lt(n, row_ptr, col, w, seeds, blocked=None):
    """E[spread] and E[spread^2] and per-vertex decrease, by enumerating every LT world."""
    removed = np.zeros(n, bool) if blocked is None else np.asarray(blocked, bool)
    opts = _lt_options(n, row_ptr, col, w)
    E = E2 = 0.0
    dec = np.zeros(n)
    for choice in itertools.product(*opts):
        prob = math.prod(p for _, p in choice)
        if prob == 0.0:
            continue
        live = np.zeros(len(col), bool)
        for e, _ in choice:
            if e >= 0:
                live[e] = True
        r = H.reach(n, row_ptr, col, live, seeds, removed)
        size = int(r.sum())
        E += prob * size
        E2 += prob * size * size
        for u in range(n):
            if r[u] and u not in seeds and not removed[u]:
                rem = removed.copy()
                rem[u] = True
                dec[u] += prob * (size - int(H.reach(n, row_ptr, col, live, seeds, rem).sum()))
    return E, E2, dec


def test_two_seeds_into_one_vertex_add_their_weights():
    # s1 -> u (0.25), s2 -> u (0.5): LT activates u with probability 0.75 (IC: 0.625)
    rp, c, w = H.csr_from_edges(3, [(0, 2, 0.25), (1, 2, 0.5)])
    theta = 40000
    _, st = orc.decrease(3, rp, c, w, [0, 1], None, theta, 3, model=orc.LT)
    p = st["reached"] / theta
    se = math.sqrt(0.75 * 0.25 / theta)
    assert abs(p - 0.75) < 4 * se
    _, st_ic = orc.decrease(3, rp, c, w, [0, 1], None, theta, 3, model=orc.IC)
    assert abs(st_ic["reached"] / theta - 0.625) < 4 * math.sqrt(0.625 * 0.375 / theta)


def test_choice_frequencies_follow_dyadic_weights():
    # vertex 3 has in-edges of weight 1/8, 1/4, 1/2 (and 1/8 chance of none)
    rp, c, w = H.csr_from_edges(4, [(0, 3, 0.125), (1, 3, 0.25), (2, 3, 0.5)])
    counts = {}
    trials = 20000
    for j in range(trials):
        e = orc.lt_trigger(4, rp, c, w, 77, j, 3)
        counts[e] = counts.get(e, 0) + 1
    want = {0: 0.125, 1: 0.25, 2: 0.5, -1: 0.125}
    assert set(counts) <= set(want)
    for e, p in want.items():
        assert abs(counts.get(e, 0) / trials - p) < 4 * math.sqrt(p * (1 - p) / trials)
    # a vertex without in-edges never chooses one
    assert orc.lt_trigger(4, rp, c, w, 77, 5, 0) == -1


def test_weights_above_one_are_rejected():
    rp, c, w = H.csr_from_edges(3, [(0, 2, 0.75), (1, 2, 0.5)])
    with pytest.raises(orc.OracleError):
        orc.decrease(3, rp, c, w, [0], None, 10, 0, model=orc.LT)
    # the same weights are a valid IC input
    orc.decrease(3, rp, c, w, [0], None, 10, 0, model=orc.IC)


def _random_lt_graph(rng, n, m):
    """Random graph with dyadic LT weights summing to at most 1 per target."""
    edges = []
    for _ in range(m):
        u, v = int(rng.integers(0, n)), int(rng.integers(0, n))
        edges.append((u, v))
    ins = {}
    for u, v in edges:
        ins.setdefault(v, []).append(u)
    out = []
    for v, srcs in ins.items():
        k = len(srcs)
        # weights 2^-a that sum to at most 1
        for i, u in enumerate(srcs):
            out.append((u, v, 2.0 ** -(1 + (i % 3)) / max(1, (k + 2) // 3)))
    return H.csr_from_edges(n, out)


def test_estimator_matches_exact_lt_worlds():
    rng = np.random.default_rng(21)
    done = 0
    for k in range(40):
        n = int(rng.integers(3, 8))
        rp, c, w = _random_lt_graph(rng, n, int(rng.integers(n, 2 * n + 2)))
        opts = _lt_options(n, rp, c, w)
        if math.prod(len(o) for o in opts) > 4000:
            continue
        seeds = [int(rng.integers(0, n))]
        E, E2, dec = _exact_lt(n, rp, c, w, seeds)
        theta = 20000
        D, st = orc.decrease(n, rp, c, w, seeds, None, theta, 100 + k, model=orc.LT)
        est = len(seeds) + st["reached"] / theta
        assert H.within_sigmas(est, E, E2, theta), (k, est, E)
        # every reached vertex has exactly one live in-edge from the reached part
        assert st["live_edges"] == st["reached"]
        # decrease estimates within a generous bound of the exact decrease
        for u in range(n):
            if u in seeds:
                continue
            var_bound = (n ** 2) / 4.0
            assert abs(D[u] / theta - dec[u]) <= 4 * math.sqrt(var_bound / theta) + 1e-9
        done += 1
    assert done >= 10


def test_lt_samples_satisfy_theorem_6_by_deletion():
    rng = np.random.default_rng(8)
    for k in range(20):
        n = int(rng.integers(4, 25))
        rp, c, w = _random_lt_graph(rng, n, int(rng.integers(n, 3 * n)))
        seeds = list(map(int, rng.choice(n, size=int(rng.integers(1, 3)), replace=False)))
        key, j = 5 + k, k
        r, cs, idom = orc.sample(n, rp, c, w, seeds, None, key, j, model=orc.LT)
        # rebuild the sample's live edges from the triggering choices alone
        live = np.zeros(len(c), bool)
        for v in range(n):
            e = orc.lt_trigger(n, rp, c, w, key, j, v)
            if e >= 0:
                live[e] = True
        removed = np.zeros(n, bool)
        full = H.reach(n, rp, c, live, seeds, removed)
        assert r == int(full.sum()) - len(seeds)
        for u in range(n):
            if u in seeds:
                continue
            if not full[u]:
                assert cs[u] == 0
                continue
            rem = removed.copy()
            rem[u] = True
            assert cs[u] == int(full.sum()) - int(H.reach(n, rp, c, live, seeds, rem).sum())


def test_lt_greedy_blocks_the_only_bridge():
    # 0 -> 1 (w 1) -> {2..9} (w 1 each): blocking 1 removes everything
    edges = [(0, 1, 1.0)] + [(1, v, 1.0) for v in range(2, 10)]
    rp, c, w = H.csr_from_edges(10, edges)
    for mode in (orc.AG, orc.GR):
        B, calls, st = orc.greedy(10, rp, c, w, [0], 1, 200, 0, mode, model=orc.LT)
        assert list(B) == [1]
