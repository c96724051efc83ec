"""Pins for the label-correcting oracle (the paper's CUDA method, Algorithms 3
and 4, as synchronous sweeps over changed vertices) and for the closed-form pred
that the label-correcting kernels use, including the condition under which it
equals Algorithm 1's pred when zero weights are present."""
import numpy as np

import oracle
from tests.graphs import INF, brute_force_dist, from_edges, lexmin_tight_pred, random_dense


def test_dist_matches_dijkstra_and_bellman_ford():
    rng = np.random.default_rng(600)
    for trial in range(200):
        n = int(rng.integers(1, 48))
        W = random_dense(rng, n, float(rng.choice([0.05, 0.2, 0.6])), 0 if trial % 3 == 0 else 1,
                         int(rng.choice([3, 50, 1000])), directed=bool(trial % 2))
        src = int(rng.integers(0, n))
        d, sweeps, rows = oracle.label_correcting(W, src)
        assert np.array_equal(d, oracle.dijkstra(W, src)[0])
        bf = oracle.bellman_ford(W, src)
        assert np.array_equal(np.where(bf >= INF, INF, bf).astype(np.int32), d)
        assert sweeps >= 1 and rows >= sweeps


def test_dist_matches_brute_force_on_tiny_graphs():
    rng = np.random.default_rng(601)
    for _ in range(300):
        n = int(rng.integers(1, 7))
        W = random_dense(rng, n, 0.5, 0, 5, directed=True)
        src = int(rng.integers(0, n))
        assert np.array_equal(oracle.label_correcting(W, src)[0], brute_force_dist(W, src))


def test_sweep_and_row_counts_closed_forms():
    # directed path 0 -> 1 -> ... -> k-1: one new vertex per sweep, the last sweep changes nothing
    for k in (1, 2, 5, 17):
        W = from_edges(k, [(i, i + 1, 1) for i in range(k - 1)], directed=True)
        d, sweeps, rows = oracle.label_correcting(W, 0)
        assert list(d) == list(range(k)) and sweeps == k and rows == k
    # star around the source: its row, then the leaves' rows (which change nothing)
    W = from_edges(9, [(0, i, 3) for i in range(1, 9)])
    assert oracle.label_correcting(W, 0)[1:] == (2, 9)
    # complete graph with equal weights: two sweeps, every row once
    W = np.full((12, 12), 7, np.int32)
    np.fill_diagonal(W, 0)
    assert oracle.label_correcting(W, 4)[1:] == (2, 12)
    # 0->1 (10), 0->2 (1), 2->1 (1): vertex 1 improves in the second sweep, and
    # its row is relaxed again in a third
    W = from_edges(3, [(0, 1, 10), (0, 2, 1), (2, 1, 1)], directed=True)
    d, sweeps, rows = oracle.label_correcting(W, 0)
    assert list(d) == [0, 2, 1] and sweeps == 3 and rows == 4
    # isolated source
    W = from_edges(5, [(1, 2, 1)])
    d, sweeps, rows = oracle.label_correcting(W, 0)
    assert list(d) == [0, INF, INF, INF, INF] and (sweeps, rows) == (1, 1)


def tight_zero_edge(W, dist):
    """Is there an edge u -> v, u != v, of weight 0 with dist[u] == dist[v] < inf?"""
    n = W.shape[0]
    z = (W == 0) & ~np.eye(n, dtype=bool)
    fin = dist != INF
    return bool((z & (dist[:, None] == dist[None, :]) & fin[:, None]).any())


def test_closed_form_pred_is_algorithm_1_pred_without_tight_zero_edges():
    """Without a tight zero-weight edge Algorithm 1 settles in (dist, index) order,
    so the closed form equals its pred; with one it can differ (and does here)."""
    rng = np.random.default_rng(602)
    clean = differ = 0
    for trial in range(3000):
        n = int(rng.integers(2, 10))
        W = random_dense(rng, n, float(rng.choice([0.3, 0.6])), 0, int(rng.choice([1, 2, 4])),
                         directed=bool(trial % 2))
        src = int(rng.integers(0, n))
        dist, pred, _ = oracle.dijkstra(W, src)
        cf = oracle.closed_form_pred(W, dist)
        cf[src] = -1
        py = lexmin_tight_pred(W, dist)
        py[src] = -1
        assert np.array_equal(cf, py)
        if tight_zero_edge(W, dist):
            differ += int(not np.array_equal(cf, pred))
        else:
            clean += 1
            assert np.array_equal(cf, pred), (W, src)
    assert clean > 500 and differ > 50


def test_zero_weight_regression_is_flagged():
    # the builder's zero-weight case: dist = [0, 1, 2, 1, 1] and the weight-0 edge
    # 3 - 1 joins two vertices at dist 1, so the closed form is not trusted there
    W = from_edges(5, [(0, 3, 1), (0, 4, 1), (3, 1, 0), (1, 2, 1), (4, 2, 1)])
    dist, pred, _ = oracle.dijkstra(W, 0)
    assert tight_zero_edge(W, dist)
    assert list(pred) == [-1, 3, 1, 0, 0]
