"""The entry point that allocates nothing (imin_decrease_noalloc), through the C ABI, against
imin_decrease on the same graph and arguments: the counts into a caller-owned device buffer
must equal the plain call's bit for bit, with identical work counters, on two calls in a
row (the second on a smaller input, reusing the same static scratch), with blocked vertices
and duplicate seeds, interleaved with plain calls that leave thresholds masked, under the
linear-threshold model, and with the errors of a graph too large for the scratch."""
import numpy as np
import pytest

from paper_2302_13529_amd import graphgen as gg
from tests import helpers as H

pytestmark = pytest.mark.gpu

KEYS = ("samples", "reached", "edges_scanned", "live_edges")


def case(msg):
    print(f"[case] {msg}", flush=True)


def _noalloc(gpu, g, n, seeds, blocked, theta, seed):
    import torch
    out = torch.full((n,), -1, dtype=torch.int64, device="cuda")
    st = gpu.imin_decrease_noalloc(g.handle, n, seeds, blocked, theta, seed, out.data_ptr())
    torch.cuda.synchronize()
    return out.cpu().numpy().view(np.uint64), st


def _check(gpu, g, n, seeds, blocked, theta, seed, label):
    case(label)
    D, st = _noalloc(gpu, g, n, seeds, blocked, theta, seed)
    Dp, sp = g.decrease(seeds, blocked, theta, seed)
    assert np.array_equal(D, Dp), label
    assert {k: st[k] for k in KEYS} == {k: sp[k] for k in KEYS}, label
    return D


def test_noalloc_equals_decrease_two_calls_second_smaller(gpu):
    big = H.cached("rmat17", gg.rmat_plain)
    small = gg.tiny_plain()
    gb = gpu.Graph(big.row_ptr, big.col, big.prob)
    gs = gpu.Graph(small.row_ptr, small.col, small.prob)
    _check(gpu, gb, big.n, big.seeds, None, 3000, 7, "rmat17, theta 3000")
    _check(gpu, gs, small.n, small.seeds, None, 500, 3, "tiny after rmat17, theta 500")
    # blocked vertices, repeated seeds, a plain call's masks left in place before it
    blk = np.zeros(small.n, np.uint8)
    blk[[5, 17, 400]] = 1
    blk[small.seeds] = 0
    gs.greedy(small.seeds[:3], 2, 100, 1, gpu.IMIN_AG)
    seeds = list(small.seeds) + list(small.seeds[:2])
    _check(gpu, gs, small.n, seeds, blk, 777, 11, "tiny, blocked, repeated seeds")
    # the plain calls after it see the graph's thresholds as created
    D, st = gs.decrease(small.seeds, None, 500, 3)
    D2, st2 = _noalloc(gpu, gs, small.n, small.seeds, None, 500, 3)
    assert np.array_equal(D, D2)
    gb.close()
    gs.close()


def test_noalloc_hand_over_and_spill_paths(gpu):
    """Samples that outgrow the wave kernel, and a dense graph whose samples overflow the
    slots' extra-edge lists into the spill slots."""
    rp, c, p = H.csr_from_edges(300, [(i, i + 1, 1.0) for i in range(299)])
    g = gpu.Graph(rp, c, p)
    _check(gpu, g, 300, [0], None, 40, 0, "path 300")
    g.close()
    k = 120
    rng = np.random.default_rng(1)
    edges = [(u, v, 1.0) for u in range(k) for v in range(k) if u != v and rng.random() < 0.7]
    rp, c, p = H.csr_from_edges(k, edges)
    g = gpu.Graph(rp, c, p)
    g.set_launch(0, 64)  # a small extra-edge capacity for the plain call as well
    _check(gpu, g, k, [0], None, 30, 5, "dense 120")
    g.close()


def test_noalloc_linear_threshold(gpu):
    """A linear-threshold graph: its samples take the triggering model's kernel paths
    (vertex-keyed choices, no kept row ranges), through the wave kernel and the workgroup
    kernel, with blocked vertices."""
    t = gg.tiny_plain()
    g = gpu.Graph(t.row_ptr, t.col, t.prob, model=gpu.IMIN_LT)
    _check(gpu, g, t.n, t.seeds, None, 600, 9, "LT tiny, theta 600")
    blk = np.zeros(t.n, np.uint8)
    blk[[3, 29, 511]] = 1
    blk[t.seeds] = 0
    _check(gpu, g, t.n, t.seeds, blk, 300, 4, "LT tiny, blocked, theta 300")
    g.close()


def test_noalloc_rejects_what_does_not_fit(gpu):
    import torch
    t = H.cached("rmat22", gg.large_plain)
    g = gpu.Graph(t.row_ptr, t.col, t.prob)
    out = torch.zeros(t.n, dtype=torch.int64, device="cuda")
    case("rmat22 is larger than the scratch")
    with pytest.raises(gpu.IminError) as e:
        gpu.imin_decrease_noalloc(g.handle, t.n, t.seeds, None, 100, 0, out.data_ptr())
    assert e.value.status == gpu.IMIN_ERANGE
    with pytest.raises(gpu.IminError) as e:
        gpu.imin_decrease_noalloc(g.handle, t.n, [t.n], None, 100, 0, out.data_ptr())
    assert e.value.status == gpu.IMIN_EINVAL
    with pytest.raises(gpu.IminError) as e:
        gpu.imin_decrease_noalloc(g.handle, t.n, t.seeds, None, 100, 0, 0)
    assert e.value.status == gpu.IMIN_EINVAL
    g.close()
