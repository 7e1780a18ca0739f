"""Greedy drivers of the oracle against brute force on deterministic graphs (p in {0, 1}).

With every probability 0 or 1 each sample is the same graph, so D[u] = theta * (size of
u's dominator subtree) exactly, and AdvancedGreedy / GreedyReplace (Algorithms 3, 4) must
equal the same loops run on exact spreads (Theorem 4 with zero variance).
"""
import networkx as nx
import numpy as np
import pytest

from oracle import oracle as orc
from tests import helpers as H


def _det_graph(rng, n, m):
    return H.random_graph(rng, n, m, probs=(0.0, 1.0, 1.0))


def _exact_spread(n, row_ptr, col, prob, seeds, blocked):
    live = np.asarray(prob) >= 1.0
    return int(H.reach(n, row_ptr, col, live, seeds, blocked).sum())


def _brute_ag(n, row_ptr, col, prob, seeds, b):
    blocked = np.zeros(n, dtype=bool)
    B = []
    is_seed = np.zeros(n, bool)
    is_seed[seeds] = True
    for _ in range(min(b, n - int(is_seed.sum()))):
        base = _exact_spread(n, row_ptr, col, prob, seeds, blocked)
        best, bx = -1, -1
        for u in range(n):
            if is_seed[u] or blocked[u]:
                continue
            b2 = blocked.copy()
            b2[u] = True
            d = base - _exact_spread(n, row_ptr, col, prob, seeds, b2)
            if d > best:
                best, bx = d, u
        blocked[bx] = True
        B.append(bx)
    return B


def _brute_gr(n, row_ptr, col, prob, seeds, b):
    is_seed = np.zeros(n, bool)
    is_seed[seeds] = True
    cand = sorted({int(col[e]) for s in set(seeds) for e in range(row_ptr[s], row_ptr[s + 1])
                   if not is_seed[col[e]]})
    blocked = np.zeros(n, dtype=bool)

    def dec(u):
        b2 = blocked.copy()
        b2[u] = True
        return (_exact_spread(n, row_ptr, col, prob, seeds, blocked)
                - _exact_spread(n, row_ptr, col, prob, seeds, b2))

    B = []
    for _ in range(min(len(cand), b)):
        best, bx = -1, -1
        for u in cand:
            d = dec(u)
            if d > best:
                best, bx = d, u
        cand.remove(bx)
        blocked[bx] = True
        B.append(bx)
    for u in list(reversed(B)):
        slot = B.index(u)
        blocked[u] = False
        best, bx = -1, -1
        for v in range(n):
            if is_seed[v] or blocked[v]:
                continue
            d = dec(v)
            if d > best:
                best, bx = d, v
        B[slot] = bx
        blocked[bx] = True
        if bx == u:
            break
    return B


def test_deterministic_counts_are_theta_times_subtree():
    rng = np.random.default_rng(21)
    for trial in range(40):
        n = int(rng.integers(2, 30))
        row_ptr, col, prob = _det_graph(rng, n, int(rng.integers(0, 3 * n)))
        seeds = list(rng.choice(n, size=int(rng.integers(1, 3)), replace=False))
        theta = 7
        D, st = orc.decrease(n, row_ptr, col, prob, seeds, None, theta, trial)
        G = nx.DiGraph()
        G.add_node("r")
        for u in range(n):
            for e in range(row_ptr[u], row_ptr[u + 1]):
                v = int(col[e])
                if prob[e] >= 1.0 and v not in seeds:
                    G.add_edge("r" if u in seeds else u, v)
        reached = nx.descendants(G, "r")
        idom = nx.immediate_dominators(G, "r")
        size = {v: 1 for v in reached}
        # accumulate subtree sizes from the deepest dominator-tree vertices up
        depth = {}
        for v in reached:
            d, x = 0, v
            while x != "r":
                x = idom[x]
                d += 1
            depth[v] = d
        for v in sorted(reached, key=lambda x: -depth[x]):
            if idom[v] != "r":
                size[idom[v]] += size[v]
        for v in range(n):
            assert D[v] == theta * size.get(v, 0)
        assert st["reached"] == theta * len(reached)


@pytest.mark.parametrize("mode", [orc.AG, orc.GR])
def test_greedy_equals_brute_force_on_deterministic_graphs(mode):
    rng = np.random.default_rng(100 + mode)
    for trial in range(30):
        n = int(rng.integers(2, 18))
        row_ptr, col, prob = _det_graph(rng, n, int(rng.integers(1, 3 * n)))
        seeds = list(map(int, rng.choice(n, size=int(rng.integers(1, 3)), replace=False)))
        b = int(rng.integers(0, 6))
        B, calls, st = orc.greedy(n, row_ptr, col, prob, seeds, b, 3, 9, mode)
        want = (_brute_ag if mode == orc.AG else _brute_gr)(n, row_ptr, col, prob, seeds, b)
        assert list(B) == want, (trial, list(B), want)


def test_dks_construction_all_edges_certain():
    """Theorem 1's reduction uses p = 1 everywhere: spreads are deterministic reach counts.

    Seed s points to every vertex of one layer, each of which points to the vertices of
    a second layer given by the edges of an undirected graph; blocking k first-layer
    vertices removes exactly the second-layer vertices all of whose parents are blocked.
    """
    rng = np.random.default_rng(8)
    k = 6
    und = [(a, b) for a in range(k) for b in range(a + 1, k) if rng.random() < 0.5]
    n = 1 + k + len(und)
    edges = [(0, 1 + a, 1.0) for a in range(k)]
    for i, (a, b) in enumerate(und):
        edges += [(1 + a, 1 + k + i, 1.0), (1 + b, 1 + k + i, 1.0)]
    row_ptr, col, prob = H.csr_from_edges(n, edges)
    D, st = orc.decrease(n, row_ptr, col, prob, [0], None, 5, 0)
    for a in range(k):
        assert D[1 + a] == 5  # a first-layer vertex dominates only itself
    for i in range(len(und)):
        assert D[1 + k + i] == 5
    # blocking both endpoints of an undirected edge cuts its second-layer vertex
    if und:
        a, b = und[0]
        blk = np.zeros(n, np.uint8)
        blk[1 + a] = 1
        D2, st2 = orc.decrease(n, row_ptr, col, prob, [0], blk, 5, 0)
        assert D2[1 + b] == 5 * (1 + sum(1 for (x, y) in und if a in (x, y) and b in (x, y)))
