"""Host side of the evaluation harness: the RA and OD baselines (Section VI-A)."""
import numpy as np

from paper_2302_13529_amd import evaluate as ev
from tests import helpers as H


def test_rand_blockers_are_distinct_non_seeds_and_seeded():
    seeds = [3, 7, 11]
    a = ev.rand_blockers(50, seeds, 10, 1)
    b = ev.rand_blockers(50, seeds, 10, 1)
    c = ev.rand_blockers(50, seeds, 10, 2)
    assert list(a) == list(b) and list(a) != list(c)
    assert len(set(a.tolist())) == 10 and not set(a.tolist()) & set(seeds)
    assert all(0 <= v < 50 for v in a)
    # budget beyond the non-seed vertices: all of them
    assert sorted(ev.rand_blockers(5, [0], 10, 0).tolist()) == [1, 2, 3, 4]


def test_outdegree_blockers_follow_degree_then_id():
    rng = np.random.default_rng(5)
    for _ in range(20):
        n = int(rng.integers(2, 40))
        rp, c, p = H.random_graph(rng, n, int(rng.integers(0, 4 * n)))
        seeds = list(map(int, rng.choice(n, size=int(rng.integers(1, 4)), replace=False)))
        b = int(rng.integers(0, n))
        got = ev.outdegree_blockers(rp, seeds, b).tolist()
        deg = np.diff(rp)
        want = sorted((v for v in range(n) if v not in seeds), key=lambda v: (-deg[v], v))[:b]
        assert got == want


def test_outdegree_blockers_skip_seeds_even_with_the_largest_degree():
    rp, c, p = H.csr_from_edges(4, [(0, 1, 1.0), (0, 2, 1.0), (0, 3, 1.0), (2, 3, 1.0)])
    assert ev.outdegree_blockers(rp, [0], 2).tolist() == [2, 1]


def test_blocked_mask():
    m = ev.blocked_mask(6, [1, 4])
    assert m.dtype == np.uint8 and m.tolist() == [0, 1, 0, 0, 1, 0]
