"""Pins of the CPU oracle against facts that do not come from the oracle itself.

* Philox4x32-10: published known-answer vectors and torch's independent header-only engine.
* Coin rule: the integer threshold test equals the float test U < p for every 24-bit U.
* Dominators: networkx (Cooper-Harvey-Kennedy) and vertex-deletion brute force (Theorem 6).
* Estimator: exact enumeration of all live-edge worlds (Lemma 1, Corollary 1, Theorem 4)
  within 4 standard errors; the paper's toy-graph numbers (Examples 1 and 3, Theorem 2).
* Exact per-sample identity of Corollary 1 with shared coins.
"""
import os
import shutil
import subprocess

import networkx as nx
import numpy as np
import pytest

from oracle import oracle as orc
from tests import helpers as H

# ---------------------------------------------------------------- Philox

# Known-answer vectors of the Random123 distribution for Philox4x32-10
# (counter words, key words) -> output words.
KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    assert tuple(int(x) for x in orc.philox(ctr, key)) == want


_TORCH_PROBE = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
int main() {
  unsigned c0, c1, c2, c3, k0, k1;
  while (scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    at::Philox4_32 eng(((uint64_t)k1 << 32) | k0, ((uint64_t)c3 << 32) | c2,
                       ((uint64_t)c1 << 32) | c0);
    unsigned a = eng(), b = eng(), c = eng(), d = eng();
    printf("%08x %08x %08x %08x\n", a, b, c, d);
  }
}
"""


def test_philox_matches_torch_engine(tmp_path):
    """torch's at::Philox4_32 maps (seed, subsequence, offset) to key / counter words."""
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if not shutil.which("g++") or not os.path.exists(os.path.join(inc, "ATen/core/PhiloxRNGEngine.h")):
        pytest.skip("g++ or torch headers unavailable")
    src = tmp_path / "probe.cpp"
    exe = tmp_path / "probe"
    src.write_text(_TORCH_PROBE)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I", inc, "-o", str(exe), str(src)])
    rng = np.random.default_rng(7)
    cases = rng.integers(0, 2**32, size=(2000, 6), dtype=np.uint64)
    cases[:100, 2:4] = 0  # the counter layout the method uses: (e >> 2, j, 0, 0)
    inp = "\n".join(" ".join(f"{int(x):x}" for x in row) for row in cases) + "\n"
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True)
    got = [tuple(int(w, 16) for w in line.split()) for line in out.stdout.strip().split("\n")]
    for row, g in zip(cases, got):
        want = tuple(int(x) for x in orc.philox(row[:4], row[4:]))
        assert g == want


# ---------------------------------------------------------------- coin rule

@pytest.mark.parametrize("p", [0.0, 1.0, 0.5, 0.1, 0.01, 0.001, 1 / 3, 1 / 7, 2.0**-24,
                               2.0**-25, 1e-9, 0.9999999, float(np.nextafter(np.float32(1), 0)),
                               float(np.float32(1) / np.float32(59174))])
def test_threshold_equals_float_test(p):
    """(u24 < ceil(p 2^24)) == (u24 * 2^-24 < p) for every 24-bit u24 (Definition 4)."""
    p32 = np.float32(p)
    thr = orc.threshold(float(p32))
    u = np.arange(2**24, dtype=np.int64)
    float_test = (u.astype(np.float64) * 2.0**-24) < np.float64(p32)
    assert np.array_equal(u < thr, float_test)


def test_edge_live_uses_word_of_quad():
    """Coin of edge e in sample j: word e & 3 of Philox at counter (e >> 2, j, 0, 0)."""
    key = 0x0123456789ABCDEF
    for e in range(0, 40):
        for j in (0, 1, 77):
            w = orc.philox([e >> 2, j, 0, 0], [key & 0xFFFFFFFF, key >> 32])[e & 3]
            for p in (0.25, 0.5, 0.75):
                assert orc.edge_live(key, j, e, p) == (int(w) >> 8 < orc.threshold(p))


# ---------------------------------------------------------------- one sampled graph

def _materialise(n, row_ptr, col, prob, key, j):
    return np.array([orc.edge_live(key, j, e, float(prob[e])) for e in range(len(col))],
                    dtype=bool)


def _rand_instance(rng):
    n = int(rng.integers(2, 26))
    m = int(rng.integers(0, 4 * n))
    row_ptr, col, prob = H.random_graph(rng, n, m)
    k = int(rng.integers(1, min(3, n) + 1))
    seeds = rng.choice(n, size=k, replace=False).astype(np.int32)
    blocked = np.zeros(n, dtype=np.uint8)
    for v in rng.choice(n, size=int(rng.integers(0, max(1, n // 4) + 1)), replace=False):
        if v not in seeds:
            blocked[v] = 1
    return n, row_ptr, col, prob, seeds, blocked


def test_dominators_match_networkx_and_deletion():
    rng = np.random.default_rng(11)
    checked = 0
    for trial in range(120):
        n, row_ptr, col, prob, seeds, blocked = _rand_instance(rng)
        for j in range(3):
            key = int(rng.integers(0, 2**63))
            r, c, idom = orc.sample(n, row_ptr, col, prob, seeds, blocked, key, j)
            live = _materialise(n, row_ptr, col, prob, key, j)
            # merged seed: a root 'r' with an edge to v iff some seed->v edge is live
            G = nx.DiGraph()
            G.add_node("r")
            is_seed = np.zeros(n, bool)
            is_seed[seeds] = True
            for u in range(n):
                for e in range(row_ptr[u], row_ptr[u + 1]):
                    v = int(col[e])
                    if not live[e] or is_seed[v] or blocked[v]:
                        continue
                    G.add_edge("r" if is_seed[u] else u, v)
            reached = nx.descendants(G, "r")
            assert r == len(reached)
            nx_idom = nx.immediate_dominators(G, "r")
            for v in range(n):
                if v in reached:
                    want = -1 if nx_idom[v] == "r" else nx_idom[v]
                    assert idom[v] == want
                else:
                    assert idom[v] == -2 and c[v] == 0
            # Theorem 6: c[u] = |reach| - |reach without u|, by deletion
            base = H.reach(n, row_ptr, col, live, seeds, blocked.astype(bool))
            for u in reached:
                rem = blocked.astype(bool).copy()
                rem[u] = True
                lost = int(base.sum()) - int(H.reach(n, row_ptr, col, live, seeds, rem).sum())
                assert c[u] == lost
            checked += 1
    assert checked == 360


def test_special_cases_tree_and_dag():
    """Out-tree: the dominator tree is the tree. DAG: idom(v) = NCA of its predecessors."""
    # complete binary out-tree on 15 vertices, all p = 1
    edges = [(i, 2 * i + 1, 1.0) for i in range(7)] + [(i, 2 * i + 2, 1.0) for i in range(7)]
    row_ptr, col, prob = H.csr_from_edges(15, edges)
    r, c, idom = orc.sample(15, row_ptr, col, prob, [0], None, 5, 0)
    assert r == 14
    for v in range(1, 15):
        assert idom[v] == (-1 if (v - 1) // 2 == 0 else (v - 1) // 2)
    sub = np.ones(15, dtype=int)
    for v in range(14, 0, -1):
        sub[(v - 1) // 2] += sub[v]
    assert list(c[1:]) == list(sub[1:])
    # diamond DAG 0->1, 0->2, 1->3, 2->3, 3->4: idom(3) = 0 (root), idom(4) = 3
    row_ptr, col, prob = H.csr_from_edges(5, [(0, 1, 1), (0, 2, 1), (1, 3, 1), (2, 3, 1), (3, 4, 1)])
    r, c, idom = orc.sample(5, row_ptr, col, prob, [0], None, 0, 0)
    assert list(idom[1:]) == [-1, -1, -1, 3] and list(c[1:]) == [1, 1, 2, 1]


# ---------------------------------------------------------------- estimator

def test_estimator_matches_exact_enumeration():
    """Lemma 1 / Theorem 4: the sample means converge to the exact enumerated values."""
    rng = np.random.default_rng(5)
    theta = 20000
    for trial in range(6):
        n = int(rng.integers(4, 8))
        row_ptr, col, prob = H.random_graph(rng, n, int(rng.integers(n, 2 * n + 2)),
                                            probs=(0.2, 0.5, 0.9, 1.0))
        unc = int(((prob > 0) & (prob < 1)).sum())
        if unc > 11:
            continue
        seeds = [int(rng.integers(0, n))]
        E, dec, dec2 = H.enumerate_worlds(n, row_ptr, col, prob, seeds)
        D, st = orc.decrease(n, row_ptr, col, prob, seeds, None, theta, 1000 + trial)
        for u in range(n):
            if u in seeds:
                assert D[u] == 0
                continue
            assert H.within_sigmas(D[u] / theta, dec[u], dec2[u], theta), (trial, u)
        # spread = |S| + mean reached; its variance bounded via enumeration of sigma
        est = len(seeds) + st["reached"] / theta
        assert abs(est - E) < 4 * np.sqrt(n * n / theta)


def test_toy_graph_paper_values():
    """Examples 1 and 3, Theorem 2's proof and Table III, with the v7/v8 erratum fixed."""
    n, row_ptr, col, prob, seeds, lines = H.toy_from_golden()
    E, dec, dec2 = H.enumerate_worlds(n, row_ptr, col, prob, seeds, use_effective=False)
    want_E = [float(l[1]) for l in lines if l[0] == "spread"][0]
    assert abs(E - want_E) < 1e-6  # p is stored in fp32
    for l in lines:
        if l[0] == "decrease":
            assert abs(dec[int(l[1]) - 1] - float(l[2])) < 1e-6, l
        if l[0] == "blocked_spread":
            k = l.index(":")
            blk = np.zeros(n, dtype=np.uint8)
            for v in l[1:k]:
                blk[int(v) - 1] = 1
            Eb, _, _ = H.enumerate_worlds(n, row_ptr, col, prob, seeds, blk, use_effective=False)
            assert abs(Eb - float(l[k + 1])) < 1e-6, l
    # Monte-Carlo estimate of the oracle within 4 standard errors of the exact values
    theta = 100_000
    Ee, dec_e, dec2_e = H.enumerate_worlds(n, row_ptr, col, prob, seeds)
    D, st = orc.decrease(n, row_ptr, col, prob, seeds, None, theta, 0)
    for u in range(1, n):
        assert H.within_sigmas(D[u] / theta, dec_e[u], dec2_e[u], theta), u
    # greedy drivers reproduce Table III / Example 4
    for l in lines:
        if l[0] == "greedy":
            mode = orc.AG if l[1] == "AG" else orc.GR
            b = int(l[2])
            want = [int(v) - 1 for v in l[4:]]
            B, calls, _ = orc.greedy(n, row_ptr, col, prob, seeds, b, 20000, 0, mode)
            assert list(B) == want, l


def test_corollary1_identity_with_shared_coins():
    """Per sample, blocking u removes exactly c_j[u] vertices: with the same key,
    sum_j |R_j(B + u)| = sum_j |R_j(B)| - D_B[u] (Corollary 1, Theorem 6)."""
    rng = np.random.default_rng(3)
    for trial in range(25):
        n, row_ptr, col, prob, seeds, blocked = _rand_instance(rng)
        key = int(rng.integers(0, 2**63))
        theta = 64
        D, st = orc.decrease(n, row_ptr, col, prob, seeds, blocked, theta, key)
        for u in range(n):
            if u in seeds or blocked[u]:
                assert D[u] == 0
                continue
            b2 = blocked.copy()
            b2[u] = 1
            _, st2 = orc.decrease(n, row_ptr, col, prob, seeds, b2, theta, key)
            assert st2["reached"] == st["reached"] - int(D[u])


def test_oracle_rejects_bad_input():
    row_ptr, col, prob = H.csr_from_edges(3, [(0, 1, 0.5), (1, 2, 0.5)])
    with pytest.raises(orc.OracleError):
        orc.decrease(3, row_ptr, col, prob, [0], np.array([1, 0, 0], np.uint8), 10, 0)
    with pytest.raises(orc.OracleError):
        orc.decrease(3, row_ptr, col, prob, [5], None, 10, 0)
    with pytest.raises(orc.OracleError):
        orc.decrease(3, row_ptr, col, np.array([0.5, np.nan], np.float32), [0], None, 10, 0)
    with pytest.raises(orc.OracleError):
        orc.decrease(3, row_ptr, col, prob, [0], None, 0, 0)
