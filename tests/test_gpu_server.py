"""The query server: every query's result equals imin_greedy alone, whatever else shares
its steps; admission respects the memory budget; errors leave the server usable."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2302_13529_amd import graphgen as gg
from paper_2302_13529_amd import serve
from tests import helpers as H

pytestmark = pytest.mark.gpu


def case(msg):
    print(f"[case] {msg}", flush=True)


def _queries(n, count, seed, theta=(100, 300, 1000), bmax=12, smax=8):
    rng = np.random.default_rng(seed)
    qs = []
    for i in range(count):
        k = int(rng.integers(1, smax + 1))
        qs.append(dict(seeds=rng.choice(n, size=k, replace=False).astype(np.int32),
                       b=int(rng.integers(0, bmax + 1)), theta=int(rng.choice(theta)),
                       seed=int(rng.integers(0, 2**40))))
    return qs


@pytest.fixture(scope="module")
def rmat17():
    return gg.rmat_plain()


def test_server_results_equal_single_calls(gpu):
    t = gg.tiny_plain()
    g = gpu.Graph(t.row_ptr, t.col, t.prob)
    qs = _queries(t.n, 40, 1)
    srv = gpu.Server(g, max_active=7, max_theta=1000)
    case("tiny: 40 queries, at most 7 at a time, staggered arrivals")
    arrivals = np.linspace(0.0, 0.05, len(qs))  # later queries join running ones
    res, lat, span, steps = serve.run(srv, qs, arrivals)
    assert np.all(lat >= 0) and steps >= max(q["b"] for q in qs)
    for i, q in enumerate(qs):
        B, st = res[i]
        Bp, sp = g.greedy(q["seeds"], q["b"], q["theta"], q["seed"], gpu.IMIN_AG)
        assert list(B) == list(Bp), i
        for k in ("samples", "reached", "edges_scanned", "live_edges"):
            assert st[k] == sp[k], (i, k)
    # a few against the oracle too
    for i in range(0, 40, 9):
        q = qs[i]
        Bo, calls, so = orc.greedy(t.n, t.row_ptr, t.col, t.prob, q["seeds"], q["b"], q["theta"],
                                   q["seed"], 0)
        assert list(res[i][0]) == list(Bo)
    srv.close()
    g.close()


def test_server_hands_over_large_samples(gpu):
    rp, c, p = H.csr_from_edges(300, [(i, i + 1, 1.0) for i in range(299)])
    g = gpu.Graph(rp, c, p)
    srv = gpu.Server(g, max_active=4, max_theta=200)
    qs = [dict(seeds=[0], b=3, theta=50, seed=1), dict(seeds=[100], b=2, theta=80, seed=2),
          dict(seeds=[5, 250], b=4, theta=20, seed=3)]
    case("path 300: samples larger than the wave kernel keeps")
    res, _, _, _ = serve.run(srv, qs)
    for q, (B, st) in zip(qs, res):
        Bp, sp = g.greedy(q["seeds"], q["b"], q["theta"], q["seed"], gpu.IMIN_AG)
        assert list(B) == list(Bp) and st["reached"] == sp["reached"]
    srv.close()
    g.close()


def test_admission_by_footprint(gpu, rmat17):
    t = rmat17
    g = gpu.Graph(t.row_ptr, t.col, t.prob)
    probe = gpu.Server(g, hbm_budget=1 << 30, max_active=4, max_theta=500)
    per = probe.query_bytes(3, 5)
    probe.close()
    budget = 3 * per + per // 2  # room for three queries, not four
    srv = gpu.Server(g, hbm_budget=budget, max_active=64, max_theta=500)
    qs = _queries(t.n, 9, 4, theta=(50, 100), bmax=5, smax=3)
    for q in qs:
        q["seeds"] = q["seeds"][:3]
    for q in qs:
        srv.submit(q["seeds"], q["b"], q["theta"], q["seed"])
    case("rmat17: budget for three queries")
    seen = []
    while True:
        a, qd = srv.step()
        seen.append(a)
        if a == 0 and qd == 0:
            break
    assert max(seen) <= 3
    done = srv.completed()
    assert len(done) == 9
    for tk, q in zip(sorted(done), qs):
        B, st = srv.result(tk, 5)
        Bp, _ = g.greedy(q["seeds"], q["b"], q["theta"], q["seed"], gpu.IMIN_AG)
        assert list(B) == list(Bp)
    srv.close()
    g.close()


def test_server_errors(gpu):
    t = gg.tiny_plain()
    g = gpu.Graph(t.row_ptr, t.col, t.prob)
    srv = gpu.Server(g, hbm_budget=1 << 24, max_active=2, max_theta=100)
    with pytest.raises(gpu.IminError) as e:
        srv.submit([t.n], 2, 10, 0)
    assert e.value.status == gpu.IMIN_EINVAL
    with pytest.raises(gpu.IminError) as e:
        srv.submit([0], 2, 101, 0)
    assert e.value.status == gpu.IMIN_ERANGE
    with pytest.raises(gpu.IminError) as e:
        srv.submit([0], -1, 10, 0)
    assert e.value.status == gpu.IMIN_EINVAL
    small = gpu.Server(g, hbm_budget=4096, max_active=2, max_theta=100)
    with pytest.raises(gpu.IminError) as e:
        small.submit([0], 2, 10, 0)  # can never fit
    assert e.value.status == gpu.IMIN_ERANGE
    small.close()
    tk = srv.submit([0, 1], 3, 50, 9)
    assert srv.result(tk, 3) is None  # not run yet
    with pytest.raises(gpu.IminError):
        srv.result(tk + 100, 3)
    while srv.step() != (0, 0):
        pass
    with pytest.raises(gpu.IminError) as e:
        srv.result(tk, 1)  # capacity too small; the result stays
    assert e.value.status == gpu.IMIN_ERANGE
    B, st = srv.result(tk, 3)
    assert list(B) == list(g.greedy([0, 1], 3, 50, 9, gpu.IMIN_AG)[0])
    with pytest.raises(gpu.IminError):
        srv.result(tk, 3)  # taken already
    srv.close()
    g.close()


def test_server_degenerate_queries(gpu):
    t = gg.tiny_plain()
    g = gpu.Graph(t.row_ptr, t.col, t.prob)
    srv = gpu.Server(g, max_active=4, max_theta=100)
    qs = [dict(seeds=[3], b=0, theta=10, seed=0),                 # nothing to do
          dict(seeds=list(range(t.n)), b=5, theta=10, seed=1),    # every vertex a seed
          dict(seeds=[7, 7, 7], b=2, theta=1, seed=2),            # duplicate seeds, one sample
          dict(seeds=[11], b=3, theta=100, seed=3)]
    case("server: degenerate queries")
    res, _, _, _ = serve.run(srv, qs)
    for q, (B, st) in zip(qs, res):
        Bp, sp = g.greedy(q["seeds"], q["b"], q["theta"], q["seed"], gpu.IMIN_AG)
        assert list(B) == list(Bp) and st["reached"] == sp["reached"]
        assert st["samples"] == sp["samples"]
    assert len(res[0][0]) == 0 and len(res[1][0]) == 0
    srv.close()
    g.close()


def test_server_greedy_replace_mixed_with_advanced_greedy(gpu):
    """GreedyReplace queries (Algorithm 4) in the server beside AdvancedGreedy ones: each
    equals imin_greedy alone with its mode, and a few equal the oracle."""
    t = gg.tiny_plain()
    g = gpu.Graph(t.row_ptr, t.col, t.prob)
    qs = _queries(t.n, 30, 4, bmax=8)
    for i, q in enumerate(qs):
        q["mode"] = gpu.IMIN_GR if i % 2 == 0 else gpu.IMIN_AG
    srv = gpu.Server(g, max_active=6, max_theta=1000)
    case("tiny: 30 queries, GR and AG alternating, at most 6 at a time")
    arrivals = np.linspace(0.0, 0.03, len(qs))
    res, lat, span, steps = serve.run(srv, qs, arrivals)
    for i, q in enumerate(qs):
        B, st = res[i]
        Bp, sp = g.greedy(q["seeds"], q["b"], q["theta"], q["seed"], q["mode"])
        assert list(B) == list(Bp), i
        for k in ("samples", "reached", "edges_scanned", "live_edges"):
            assert st[k] == sp[k], (i, k)
    for i in range(0, 30, 7):
        q = qs[i]
        Bo, calls, so = orc.greedy(t.n, t.row_ptr, t.col, t.prob, q["seeds"], q["b"], q["theta"],
                                   q["seed"], q["mode"])
        assert list(res[i][0]) == list(Bo), i
        assert res[i][1]["samples"] == calls * q["theta"], i
    with pytest.raises(gpu.IminError) as e:
        srv.submit(t.seeds, 2, 100, 0, mode=7)
    assert e.value.status == gpu.IMIN_EINVAL
    srv.close()
    g.close()
