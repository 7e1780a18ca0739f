"""Seeded synthetic inputs: directed graphs, edge probabilities and seed sets.

The paper evaluates on SNAP social graphs (Table IV) under the trivalency (TR) and
weighted-cascade (WC) probability models (Section VI-A, "Propagation Models").
Those datasets are not shipped here, so every workload is a synthetic power-law graph
of comparable shape, generated from a fixed seed:

* directed Chung-Lu graphs whose out- and in-weights follow w_i = (i+1)^(-1/(gamma-1))
  under independent random permutations;
* R-MAT graphs with quadrant probabilities (a, b, c, d), relabelled by a random
  permutation so that vertex id carries no degree information.

This module holds none of the blocking method's arithmetic. It produces only the
inputs both the library and the oracle consume: CSR arrays (int32), float32 edge
probabilities and seed lists. Edges inside a CSR row are sorted by target id; the
edge id of an edge is its CSR position.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Instance", "chung_lu_edges", "rmat_edges", "to_csr", "wc_probs", "tr_probs",
    "uniform_seeds", "top_out_degree_seeds", "tiny_plain", "rmat_plain", "batched_instances",
    "large_plain", "served_graph", "served_queries", "toy_fig1", "CONFIGS",
]


@dataclasses.dataclass
class Instance:
    """One influence-minimisation input: graph G, probabilities p, seeds S, theta, b."""
    name: str
    n: int
    row_ptr: np.ndarray  # int32[n+1]
    col: np.ndarray      # int32[m]
    prob: np.ndarray     # float32[m]
    seeds: np.ndarray    # int32[|S|]
    theta: int
    b: int
    seed: int = 0        # Philox seed of the sampling stream

    @property
    def m(self) -> int:
        return int(self.col.shape[0])


def _dedup_in_draw_order(src: np.ndarray, dst: np.ndarray, n: int, limit: int | None):
    """Drop self-loops and repeated (src, dst) pairs, keeping first draws in order."""
    keep = src != dst
    src, dst = src[keep], dst[keep]
    key = src.astype(np.int64) * n + dst.astype(np.int64)
    _, first = np.unique(key, return_index=True)
    first.sort()
    if limit is not None:
        first = first[:limit]
    return src[first], dst[first]


def chung_lu_edges(n: int, m_target: int, gamma: float, rng: np.random.Generator):
    """Directed Chung-Lu: draw m_target (u, v) pairs with u ~ w_out and v ~ w_in.

    Self-loops and duplicates are removed afterwards, so the edge count is at most
    m_target.
    """
    w = (np.arange(1, n + 1, dtype=np.float64)) ** (-1.0 / (gamma - 1.0))
    w_out = w[rng.permutation(n)]
    w_in = w[rng.permutation(n)]
    src = rng.choice(n, size=m_target, p=w_out / w_out.sum()).astype(np.int32)
    dst = rng.choice(n, size=m_target, p=w_in / w_in.sum()).astype(np.int32)
    return _dedup_in_draw_order(src, dst, n, None)


def _rmat_draw(scale: int, count: int, abcd, rng: np.random.Generator):
    a, b, c, _ = abcd
    src = np.zeros(count, dtype=np.int32)
    dst = np.zeros(count, dtype=np.int32)
    r = np.empty(count, dtype=np.float32)
    for _level in range(scale):
        rng.random(count, dtype=np.float32, out=r)
        sbit = r >= np.float32(a + b)
        dbit = ((r >= np.float32(a)) & (r < np.float32(a + b))) | (r >= np.float32(a + b + c))
        src <<= 1
        src |= sbit
        dst <<= 1
        dst |= dbit
    return src, dst


def rmat_edges(scale: int, m_unique: int, rng: np.random.Generator,
               abcd=(0.57, 0.19, 0.19, 0.05)):
    """R-MAT edges: distinct non-loop pairs drawn until m_unique exist (a uniform subset of
    them is kept if a batch overshoots), then relabelled by a random permutation."""
    n = 1 << scale
    keys = np.zeros(0, dtype=np.int64)
    while keys.size < m_unique:
        need = m_unique - keys.size
        s, d = _rmat_draw(scale, int(need * 1.2) + 1024, abcd, rng)
        k = (s.astype(np.int64) << scale) | d
        keys = np.unique(np.concatenate([keys, k[s != d]]))
    if keys.size > m_unique:
        keep = np.sort(rng.choice(keys.size, m_unique, replace=False))
        keys = keys[keep]
    perm = rng.permutation(n).astype(np.int32)
    return perm[keys >> scale], perm[keys & (n - 1)]


def to_csr(n: int, src: np.ndarray, dst: np.ndarray):
    """CSR with rows sorted by target id; returns (row_ptr int32[n+1], col int32[m])."""
    key = src.astype(np.int64) * n + dst.astype(np.int64)
    key.sort()
    col = (key % n).astype(np.int32)
    counts = np.bincount((key // n).astype(np.int64), minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    assert row_ptr[-1] < 2**31
    return row_ptr.astype(np.int32), col


def wc_probs(n: int, col: np.ndarray) -> np.ndarray:
    """Weighted cascade: p(u, v) = 1 / d_in(v), computed as an fp32 division."""
    indeg = np.bincount(col, minlength=n).astype(np.float32)
    return (np.float32(1.0) / indeg[col]).astype(np.float32)


def tr_probs(m: int, rng: np.random.Generator) -> np.ndarray:
    """Trivalency: each edge independently takes 0.1, 0.01 or 0.001 (fp32)."""
    vals = np.array([0.1, 0.01, 0.001], dtype=np.float32)
    return vals[rng.integers(0, 3, size=m)]


def uniform_seeds(n: int, k: int, rng: np.random.Generator) -> np.ndarray:
    return np.sort(rng.choice(n, size=k, replace=False)).astype(np.int32)


def top_out_degree_seeds(row_ptr: np.ndarray, k: int) -> np.ndarray:
    """The k vertices of largest out-degree; equal degrees go to the smaller id."""
    deg = np.diff(row_ptr.astype(np.int64))
    order = np.lexsort((np.arange(deg.shape[0]), -deg))
    return np.sort(order[:k]).astype(np.int32)


# ----------------------------------------------------------------------------------------
# Workloads. Sizes follow the paper's datasets (Table IV) in shape; seeds of the
# generators are fixed per workload so every run sees identical inputs.
# ----------------------------------------------------------------------------------------

def tiny_plain(seed: int = 1) -> Instance:
    """Chung-Lu n=1000, ~5000 edges, gamma 2.5, WC, 10 uniform seeds, theta=1000, b=10."""
    rng = np.random.default_rng(seed)
    n = 1000
    src, dst = chung_lu_edges(n, 5000, 2.5, rng)
    row_ptr, col = to_csr(n, src, dst)
    return Instance("chunglu_n1k_wc", n, row_ptr, col, wc_probs(n, col),
                    uniform_seeds(n, 10, rng), theta=1000, b=10, seed=0)


def rmat_plain(seed: int = 2) -> Instance:
    """R-MAT scale 17, 1M unique edges, WC, top-10 out-degree seeds, theta=1e4, b=100."""
    rng = np.random.default_rng(seed)
    scale = 17
    src, dst = rmat_edges(scale, 1_000_000, rng)
    n = 1 << scale
    row_ptr, col = to_csr(n, src, dst)
    return Instance("rmat17_m1M_wc", n, row_ptr, col, wc_probs(n, col),
                    top_out_degree_seeds(row_ptr, 10), theta=10_000, b=100, seed=0)


def large_plain(seed: int = 4) -> Instance:
    """R-MAT scale 22, 35M unique edges, WC, top-100 out-degree seeds, theta=1e4, b=100."""
    rng = np.random.default_rng(seed)
    scale = 22
    src, dst = rmat_edges(scale, 35_000_000, rng)
    n = 1 << scale
    row_ptr, col = to_csr(n, src, dst)
    return Instance("rmat22_m35M_wc", n, row_ptr, col, wc_probs(n, col),
                    top_out_degree_seeds(row_ptr, 100), theta=10_000, b=100, seed=0)


def batched_instances(count: int = 256, seed: int = 3):
    """Chung-Lu instances: n log-uniform in [1e3, 2e5], mean degree U[4, 16], TR, 1-50 seeds."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(2e5)))))
        davg = rng.uniform(4.0, 16.0)
        src, dst = chung_lu_edges(n, int(round(n * davg)), 2.5, rng)
        row_ptr, col = to_csr(n, src, dst)
        k = int(rng.integers(1, 51))
        out.append(Instance(f"chunglu_batch{i}", n, row_ptr, col, tr_probs(col.shape[0], rng),
                            uniform_seeds(n, k, rng), theta=2000, b=20, seed=i))
    return out


def served_graph(seed: int = 5) -> Instance:
    """R-MAT scale 20, 8M unique edges, WC; queries supply seeds, theta and b."""
    rng = np.random.default_rng(seed)
    scale = 20
    src, dst = rmat_edges(scale, 8_000_000, rng)
    n = 1 << scale
    row_ptr, col = to_csr(n, src, dst)
    return Instance("rmat20_m8M_wc", n, row_ptr, col, wc_probs(n, col),
                    np.zeros(0, np.int32), theta=0, b=0, seed=0)


def served_queries(n: int, count: int = 2000, seed: int = 6):
    """Query mix: |S| log-uniform in [1, 100], b uniform in [10, 200], theta in {1k, 5k, 10k}."""
    rng = np.random.default_rng(seed)
    qs = []
    for i in range(count):
        k = int(round(math.exp(rng.uniform(0.0, math.log(100.0)))))
        qs.append(dict(seeds=uniform_seeds(n, k, rng), b=int(rng.integers(10, 201)),
                       theta=int(rng.choice([1000, 5000, 10000])), seed=i))
    return qs


def toy_fig1() -> Instance:
    """A nine-vertex graph consistent with every value printed for the paper's toy example.

    Vertices v1..v9 are ids 0..8; the seed is v1. All edges have p = 1 except
    p(v5,v8) = 0.5, p(v9,v8) = 0.2 and p(v8,v7) = 0.1 (Example 1, Example 3).
    """
    edges = [(1, 2, 1.0), (1, 4, 1.0), (2, 5, 1.0), (4, 5, 1.0), (5, 3, 1.0), (5, 6, 1.0),
             (5, 9, 1.0), (5, 8, 0.5), (9, 8, 0.2), (8, 7, 0.1)]
    src = np.array([u - 1 for u, _, _ in edges], dtype=np.int32)
    dst = np.array([v - 1 for _, v, _ in edges], dtype=np.int32)
    p = np.array([w for _, _, w in edges], dtype=np.float32)
    order = np.lexsort((dst, src))
    n = 9
    row_ptr, col = to_csr(n, src, dst)
    return Instance("toy_fig1", n, row_ptr, col, p[order], np.array([0], np.int32),
                    theta=100_000, b=2, seed=0)


CONFIGS = {
    "tiny": tiny_plain,
    "rmat17": rmat_plain,
    "rmat22": large_plain,
}
