"""The seeded synthetic inputs match the recipes the benchmark configurations state (sizes,
probability models, seed rules, query mix), and are reproducible: the stored oracle
results under tests/golden were made from exactly these inputs."""
import numpy as np

from paper_2302_13529_amd import graphgen as gg


def _check_csr(t):
    rp, col = t.row_ptr, t.col
    assert rp.dtype == np.int32 and col.dtype == np.int32 and t.prob.dtype == np.float32
    assert rp[0] == 0 and rp[-1] == col.shape[0] and np.all(np.diff(rp) >= 0)
    assert col.min() >= 0 and col.max() < t.n
    src = np.repeat(np.arange(t.n), np.diff(rp))
    assert not np.any(src == col), "self-loops"
    key = src.astype(np.int64) * t.n + col
    assert np.all(np.diff(key) > 0), "rows sorted by target, no repeated edges"
    return src


def _check_wc(t):
    indeg = np.bincount(t.col, minlength=t.n).astype(np.float32)
    assert np.array_equal(t.prob, np.float32(1.0) / indeg[t.col])


def _check_top_seeds(t, k):
    deg = np.diff(t.row_ptr.astype(np.int64))
    assert t.seeds.shape[0] == k and np.all(np.diff(t.seeds) > 0)
    worst = deg[t.seeds].min()
    others = np.setdiff1d(np.arange(t.n), t.seeds)
    # no other vertex has a larger degree, and ties went to the smaller id
    assert deg[others].max() <= worst
    tied = others[deg[others] == worst]
    assert tied.size == 0 or tied.min() > t.seeds[deg[t.seeds] == worst].max()


def test_tiny_recipe_and_reproducible():
    t = gg.tiny_plain()
    assert (t.n, t.m, t.theta, t.b, t.seed) == (1000, 4797, 1000, 10, 0)
    _check_csr(t)
    _check_wc(t)
    assert t.seeds.shape[0] == 10 and np.unique(t.seeds).shape[0] == 10
    t2 = gg.tiny_plain()
    assert np.array_equal(t.col, t2.col) and np.array_equal(t.seeds, t2.seeds)


def test_rmat17_recipe():
    t = gg.rmat_plain()
    assert (t.n, t.m, t.theta, t.b) == (1 << 17, 1_000_000, 10_000, 100)
    _check_csr(t)
    _check_wc(t)
    _check_top_seeds(t, 10)


def test_batched_recipe():
    insts = gg.batched_instances()
    assert len(insts) == 256
    ns = np.array([t.n for t in insts])
    assert ns.min() >= 1000 and ns.max() <= 200_000
    # log-uniform sizes: both ends of the range are populated
    assert (ns < 5000).sum() > 20 and (ns > 50_000).sum() > 20
    for t in insts[:32]:
        _check_csr(t)
        assert set(np.unique(t.prob).tolist()) <= {np.float32(0.1), np.float32(0.01),
                                                   np.float32(0.001)}
        assert 1 <= t.seeds.shape[0] <= 50 and np.unique(t.seeds).shape[0] == t.seeds.shape[0]
        assert (t.theta, t.b) == (2000, 20)
        davg = t.m / t.n
        assert 2.0 <= davg <= 16.0  # U[4, 16] drawn, minus loops and repeats


def test_served_recipe():
    g = gg.served_graph()
    assert (g.n, g.m) == (1 << 20, 8_000_000)
    _check_csr(g)
    _check_wc(g)
    qs = gg.served_queries(g.n)
    assert len(qs) == 2000
    ks = np.array([len(q["seeds"]) for q in qs])
    bs = np.array([q["b"] for q in qs])
    assert ks.min() >= 1 and ks.max() <= 100
    assert bs.min() >= 10 and bs.max() <= 200
    assert {q["theta"] for q in qs} == {1000, 5000, 10000}
    assert [q["seed"] for q in qs] == list(range(2000))
    for q in qs[:200]:
        s = q["seeds"]
        assert np.all(np.diff(s) > 0) and s.min() >= 0 and s.max() < g.n
