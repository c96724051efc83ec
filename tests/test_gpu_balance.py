"""Pair balancing of large whole-GPU rounds (a round of at least 8 chunks of 1024
bucket rows: members g and g ^ 1 claim each other's remaining chunks).  Graphs whose
rounds hold most vertices at once, with default and odd workgroup counts (the last
member then has no partner), weights 1 and 2, and zero weights (a balanced round
followed by the single-vertex fallback): dist and pred against the oracle bit for
bit, rows relaxed equal to the oracle's."""
import numpy as np
import pytest

import oracle
from tests.graphs import random_dense

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GRID = 4


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_03667_amd as m
    m.lib()
    return m


def check(sp, W, src, workgroups, tag):
    Wt = torch.from_numpy(np.ascontiguousarray(W)).cuda()
    print("balance case", tag, "n", W.shape[0], "src", src, "workgroups", workgroups, flush=True)
    d, p = sp.solve(Wt, src, flags=GRID, workgroups=workgroups, balance=1)
    status, stats = sp.sssp_last_status()
    dr, pr, relaxed = oracle.dijkstra(W, src)
    assert status & 3 == 0, (tag, status)
    d, p = d.cpu().numpy(), p.cpu().numpy()
    bad = np.nonzero((d != dr) | (p != pr))[0]
    assert bad.size == 0, (tag, bad[:5].tolist(), d[bad[:5]].tolist(), dr[bad[:5]].tolist(),
                           p[bad[:5]].tolist(), pr[bad[:5]].tolist())
    assert stats[1] == relaxed, (tag, stats, relaxed)
    return stats


def test_rounds_of_most_vertices(sp):
    rng = np.random.default_rng(3100)
    W = random_dense(rng, 9000, 0.97, 1, 1)  # the solve's second round holds ~8700 vertices (9 chunks)
    for wg in (0, 64, 7, 255):
        stats = check(sp, W, int(rng.integers(0, 9000)), wg, ("unit", wg))
        assert stats[0] <= 4
    W = random_dense(rng, 12000, 0.9, 1, 2, directed=True)
    for wg in (0, 33):
        check(sp, W, 5, wg, ("one-two", wg))


def test_balanced_rounds_with_zero_weights(sp):
    rng = np.random.default_rng(3101)
    W = random_dense(rng, 9000, 0.95, 0, 1, zero_prob=0.2)
    for wg in (0, 9):
        stats = check(sp, W, 11, wg, ("zero", wg))
        assert stats[2] > 0  # single-vertex fallbacks happened


def test_large_buckets_many_sources(sp):
    rng = np.random.default_rng(3102)
    W = random_dense(rng, 14000, 0.7, 1, 2)  # the distance-2 round holds ~9000 vertices
    Wt = torch.from_numpy(W).cuda()
    for src in (0, 13999, 7777):
        print("balance case many-sources", src, flush=True)
        d, p = sp.solve(Wt, src, flags=GRID, balance=1)
        status, stats = sp.sssp_last_status()
        dr, pr, relaxed = oracle.dijkstra(W, src)
        assert status & 3 == 0
        assert np.array_equal(d.cpu().numpy(), dr) and np.array_equal(p.cpu().numpy(), pr), src
        assert stats[1] == relaxed
