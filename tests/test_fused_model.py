"""CPU model of the schedule the GPU kernels use, checked exhaustively against the
oracle.  Not an oracle: a pure-Python statement of the kernels' strategy, so the
strategy's exactness is shown before any kernel runs.

Strategy: each round takes the bucket B of all unvisited vertices at the minimal
dist d.  For every unvisited v the round computes the lexicographic minimum over
u in B of (d + W[u][v], u) and applies it only if strictly below dist[v]; all of
B becomes visited.  If some u in B has a zero-weight edge to an unvisited v with
dist[v] > d, the round is discarded and only the lowest-index member of B is
settled (one literal step of Algorithm 1)."""
import numpy as np

import oracle
from tests.graphs import INF, all_undirected, random_dense


def fused_model(W, src, literal=False):
    n = W.shape[0]
    dist = [INF] * n
    pred = [-1] * n
    vis = [False] * n
    dist[src] = 0
    rounds = fallbacks = 0
    while True:
        cand = [v for v in range(n) if not vis[v]]
        if not cand:
            break
        d = min(dist[v] for v in cand)
        if d == INF:
            break
        B = [v for v in cand if dist[v] == d]
        u0 = B[0]
        rounds += 1
        if not literal:
            best = {}
            zero = False
            for v in cand:
                if dist[v] == d:
                    continue
                k = min(((d + int(W[u, v]), u) for u in B if W[u, v] != INF), default=None)
                if k is not None:
                    best[v] = k
                if any(W[u, v] == 0 for u in B) and dist[v] > d:
                    zero = True
            if not zero:
                for u in B:
                    vis[u] = True
                for v, (c, u) in best.items():
                    if c < dist[v]:
                        dist[v], pred[v] = c, u
                continue
            fallbacks += 1
        vis[u0] = True
        for v in range(n):
            w = int(W[u0, v])
            if not vis[v] and w != INF and d + w < dist[v]:
                dist[v], pred[v] = d + w, u0
    return np.array(dist, np.int32), np.array(pred, np.int32), rounds, fallbacks


def _same(W, s, literal=False):
    d, p, _ = oracle.dijkstra(W, s)
    md, mp, rounds, fb = fused_model(W, s, literal)
    assert (md == d).all() and (mp == p).all(), (W, s)
    return rounds, fb


def test_exhaustive_n4_positive_and_zero_weights():
    for weights in ([1, 2, INF], [0, 1, INF]):
        for W in all_undirected(4, weights):
            for s in range(4):
                _same(W, s)


def test_random_graphs_with_ties_and_zero_weights():
    rng = np.random.default_rng(10)
    fallbacks = 0
    for trial in range(400):
        n = int(rng.integers(2, 14))
        W = random_dense(rng, n, float(rng.uniform(0.1, 0.9)), 1, 3, directed=bool(trial % 2),
                         zero_prob=0.2 if trial % 4 == 0 else 0.0)
        fallbacks += _same(W, int(rng.integers(0, n)))[1]
    assert fallbacks > 0  # the zero-weight path was exercised


def test_rounds_count_distinct_distances():
    """With positive weights the number of rounds is the number of distinct finite
    dist values, the quantity that bounds the kernels' barrier count."""
    rng = np.random.default_rng(11)
    for _ in range(20):
        W = random_dense(rng, 100, 0.1, 1, 5)
        d, _, _ = oracle.dijkstra(W, 0)
        rounds, fb = _same(W, 0)
        assert fb == 0 and rounds == len({int(x) for x in d if x != INF})
