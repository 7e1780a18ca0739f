"""Test-only brute force: reachability, exact enumeration of live-edge worlds, small graphs.

Everything here is written from the definitions (IC model and blockers, Section III;
random sampled graphs, Definition 4; Lemma 1, Corollary 1, Theorem 4, Theorem 6) and
shares nothing with the oracle or the library.
"""
from __future__ import annotations

import itertools
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def csr_from_edges(n, edges):
    """edges: list of (u, v, p). Returns row_ptr, col, prob sorted by (u, v) (stable)."""
    order = sorted(range(len(edges)), key=lambda i: (edges[i][0], edges[i][1], i))
    col = np.array([edges[i][1] for i in order], dtype=np.int32)
    prob = np.array([edges[i][2] for i in order], dtype=np.float32)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    for u, _, _ in edges:
        row_ptr[u + 1] += 1
    row_ptr = np.cumsum(row_ptr).astype(np.int32)
    return row_ptr, col, prob


def reach(n, row_ptr, col, live, seeds, removed):
    """Vertices reached from the seeds over live edges, never entering `removed`.

    Seeds are active at time 0 (Section III-A); removed vertices never activate
    (Definition 2). Returns a boolean array (seeds included).
    """
    seen = np.zeros(n, dtype=bool)
    stack = []
    for s in seeds:
        if not seen[s]:
            seen[s] = True
            stack.append(s)
    while stack:
        u = stack.pop()
        for e in range(row_ptr[u], row_ptr[u + 1]):
            v = col[e]
            if live[e] and not seen[v] and not removed[v]:
                seen[v] = True
                stack.append(v)
    return seen


def effective_p(prob):
    """Probability the 24-bit coin realises: ceil(p * 2^24) / 2^24 (p in [0, 1])."""
    p = np.asarray(prob, dtype=np.float64)
    t = np.ceil(p * 2.0**24)
    t[p >= 1.0] = 2.0**24
    t[p <= 0.0] = 0.0
    return t / 2.0**24


def enumerate_worlds(n, row_ptr, col, prob, seeds, blocked=None, use_effective=True):
    """Exact expected spread and per-vertex decrease by enumerating every live-edge world.

    Returns (E, dec, dec2) where E = E(S, G[V \\ B]) (seeds counted, Definition 3),
    dec[u] = E[sigma^{->u}] = decrease from blocking u (Theorem 4), and dec2[u] its second
    moment (for standard errors of a sample mean).
    """
    p = effective_p(prob) if use_effective else np.asarray(prob, dtype=np.float64)
    m = len(col)
    removed0 = np.zeros(n, dtype=bool)
    if blocked is not None:
        removed0 |= np.asarray(blocked, dtype=bool)
    unc = [e for e in range(m) if 0.0 < p[e] < 1.0]
    if len(unc) > 20:
        raise ValueError("too many uncertain edges to enumerate")
    base = p >= 1.0
    E = 0.0
    dec = np.zeros(n)
    dec2 = np.zeros(n)
    is_seed = np.zeros(n, dtype=bool)
    is_seed[list(seeds)] = True
    for bits in itertools.product([0, 1], repeat=len(unc)):
        live = base.copy()
        w = 1.0
        for e, b in zip(unc, bits):
            live[e] = bool(b)
            w *= p[e] if b else 1.0 - p[e]
        if w == 0.0:
            continue
        r = reach(n, row_ptr, col, live, seeds, removed0)
        size = int(r.sum())
        E += w * size
        for u in range(n):
            if is_seed[u] or removed0[u] or not r[u]:
                continue
            rem = removed0.copy()
            rem[u] = True
            c = size - int(reach(n, row_ptr, col, live, seeds, rem).sum())
            dec[u] += w * c
            dec2[u] += w * c * c
    return E, dec, dec2


def read_golden(name):
    """Parse a golden fixture of 'key values' lines (# comments)."""
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                out.append(line.split())
    return out


def toy_from_golden():
    lines = read_golden("toy_fig1.txt")
    edges = [(int(a) - 1, int(b) - 1, float(p)) for k, a, b, p in
             (l for l in lines if l[0] == "edge")]
    seeds = [int(l[1]) - 1 for l in lines if l[0] == "seed"]
    row_ptr, col, prob = csr_from_edges(9, edges)
    return 9, row_ptr, col, prob, seeds, lines


def random_graph(rng, n, m, probs=(0.3, 0.6, 1.0), allow_loops=True, allow_dups=True):
    edges = []
    while len(edges) < m:
        u = int(rng.integers(0, n))
        v = int(rng.integers(0, n))
        if u == v and not allow_loops:
            continue
        if not allow_dups and any(a == u and b == v for a, b, _ in edges):
            continue
        edges.append((u, v, float(rng.choice(probs))))
    return csr_from_edges(n, edges)


def within_sigmas(est, mean, second, theta, k=4.0, floor=1e-12):
    """|est - mean| <= k standard errors of a theta-sample mean (variance from moments)."""
    var = max(second - mean * mean, 0.0)
    se = math.sqrt(var / theta)
    return abs(est - mean) <= k * se + floor


def spread_moments(n, row_ptr, col, prob, seeds, blocked=None):
    """Exact first and second moments of the number of active vertices (seeds counted) by
    enumerating every live-edge world (at most 20 uncertain edges)."""
    p = effective_p(prob)
    removed = np.zeros(n, dtype=bool) if blocked is None else np.asarray(blocked, dtype=bool)
    unc = [e for e in range(len(col)) if 0.0 < p[e] < 1.0]
    if len(unc) > 20:
        raise ValueError("too many uncertain edges to enumerate")
    base = p >= 1.0
    E = E2 = 0.0
    for bits in itertools.product([0, 1], repeat=len(unc)):
        live = base.copy()
        w = 1.0
        for e, b in zip(unc, bits):
            live[e] = bool(b)
            w *= p[e] if b else 1.0 - p[e]
        if w == 0.0:
            continue
        size = int(reach(n, row_ptr, col, live, seeds, removed).sum())
        E += w * size
        E2 += w * size * size
    return E, E2


_INSTANCE_CACHE = {}


def cached(name, make):
    """A generated workload, kept for the rest of the test session (generation is seeded,
    so every caller sees the same arrays)."""
    if name not in _INSTANCE_CACHE:
        _INSTANCE_CACHE[name] = make()
    return _INSTANCE_CACHE[name]


def read_config_golden(name):
    """Parse a tests/golden/config_*.txt file written by make_config_goldens.py.

    Returns a dict: 'blockers' -> list, 'calls' -> int, 'stats' -> dict, plus per-item
    entries keyed (kind, index) -> (blockers, stats) for 'inst' / 'query' lines, and
    'decrease2048 ...' / 'greedy2 ...' lines under their first word.
    """
    out = {}

    def stats_of(words):
        return {k: int(v) for k, v in (w.split("=") for w in words)}

    for words in read_golden(name):
        head = words[0]
        if head in ("inst", "query"):
            bar = words.index("|")
            out[(head, int(words[1]))] = ([int(x) for x in words[3:bar]],
                                          stats_of(words[bar + 1:]))
        elif head in ("decrease2048", "greedy2"):
            sub = out.setdefault(head, {})
            kind = words[1]
            if kind == "blockers":
                sub[kind] = [int(x) for x in words[2:]]
            elif kind == "calls":
                sub[kind] = int(words[2])
            elif kind == "stats":
                sub[kind] = stats_of(words[2:])
            elif kind == "sha256":
                sub[kind] = words[2]
            elif kind == "top":
                sub[kind] = [tuple(int(y) for y in x.split(":")) for x in words[2:]]
        elif head == "blockers":
            out["blockers"] = [int(x) for x in words[1:]]
        elif head == "calls":
            out["calls"] = int(words[1])
        elif head == "stats":
            out["stats"] = stats_of(words[1:])
    return out
