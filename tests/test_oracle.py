"""Pins for the CPU oracle (oracle/): each test checks it against something other
than itself — the paper's worked matrices (outputs stepped by hand), brute-force
path enumeration, textbook/library shortest-path routines, closed forms,
invariants, and planted mistakes that the certificate must catch."""
import numpy as np
import pytest
from scipy.sparse.csgraph import csgraph_from_dense, dijkstra as scipy_dijkstra

import oracle
from tests.graphs import (INF, all_directed, all_undirected, brute_force_dist, from_edges,
                          golden_cases, lexmin_tight_pred, order_and_pred_from_distances,
                          random_dense)


def scipy_dist(W, src):
    """Library Dijkstra (scipy) on the same matrix; zero-weight edges kept as edges."""
    F = W.astype(np.float64)
    F[W == INF] = np.inf
    G = csgraph_from_dense(F, null_value=np.inf)
    d = scipy_dijkstra(G, directed=True, indices=src)
    return np.where(np.isinf(d), INF, d).astype(np.int64)


@pytest.mark.parametrize("name,W,expect", golden_cases(), ids=[c[0] for c in golden_cases()])
def test_worked_examples(name, W, expect):
    for src, e in expect.items():
        dist, pred, order, _ = oracle.dijkstra(W, src, with_order=True)
        assert dist.tolist() == e["dist"], (name, src)
        assert pred.tolist() == e["pred"], (name, src)
        if "order" in e:
            assert order[:len(e["order"])].tolist() == e["order"]


def test_padding_leaves_real_vertices_unchanged():
    """Section III-B pads the matrix with infinite rows/columns; outputs of real
    vertices must not change and padded vertices stay unreachable."""
    rng = np.random.default_rng(1)
    for trial in range(20):
        n = int(rng.integers(2, 40))
        pad = int(rng.integers(1, 8))
        W = random_dense(rng, n, 0.3, 1, 20, directed=bool(trial % 2))
        P = np.full((n + pad, n + pad), INF, np.int32)
        P[:n, :n] = W
        src = int(rng.integers(0, n))
        d0, p0, _ = oracle.dijkstra(W, src)
        d1, p1, _ = oracle.dijkstra(P, src)
        assert (d1[:n] == d0).all() and (p1[:n] == p0).all()
        assert (d1[n:] == INF).all() and (p1[n:] == -1).all()


def _check_against_brute_force(W):
    n = W.shape[0]
    for s in range(n):
        dist, pred, _ = oracle.dijkstra(W, s)
        bf = brute_force_dist(W, s)
        assert (dist.astype(np.int64) == bf).all(), (W, s)
        assert oracle.certificate(W, s, dist, pred)[0] == 0
        if (W[~np.eye(n, dtype=bool)] >= 1).all():
            assert (pred == lexmin_tight_pred(W, dist)).all(), (W, s)


def test_exhaustive_undirected_n4():
    """All 729 undirected 4-vertex graphs with pair weights in {1, 2, inf}, every source."""
    for W in all_undirected(4, [1, 2, INF]):
        _check_against_brute_force(W)


def test_exhaustive_directed_n3():
    """All 729 directed 3-vertex graphs with arc weights in {1, 2, inf}, every source."""
    for W in all_directed(3, [1, 2, INF]):
        _check_against_brute_force(W)


def test_random_directed_n4_to_7():
    rng = np.random.default_rng(2)
    for _ in range(300):
        n = int(rng.integers(4, 8))
        _check_against_brute_force(random_dense(rng, n, float(rng.uniform(0.2, 0.9)), 1, 4,
                                                directed=True))


def test_zero_weights_dist_and_certificate():
    """With zero weights pred is defined only by the algorithm's own order; dist is still
    the textbook distance and (dist, pred) must still be a valid shortest-path tree."""
    for W in all_undirected(4, [0, 1, INF]):
        for s in range(4):
            dist, pred, _ = oracle.dijkstra(W, s)
            assert (dist.astype(np.int64) == brute_force_dist(W, s)).all()
            assert oracle.certificate(W, s, dist, pred)[0] == 0


def _check_zero_weight_order_and_pred(W):
    n = W.shape[0]
    for s in range(n):
        bf = brute_force_dist(W, s)
        dist, pred, order, r = oracle.dijkstra(W, s, with_order=True)
        want_order, want_pred = order_and_pred_from_distances(W, s, bf)
        assert order[:r].tolist() == want_order, (W, s)
        assert (pred == want_pred).all(), (W, s)


def test_zero_weight_order_and_pred_from_distances():
    """With zero weights, the settle order and pred are pinned by Algorithm 1's
    selection rule restated over the brute-force distances (every vertex settled is
    the least (dist, index) vertex with a settled tight in-neighbour; pred is the
    first settled tight in-neighbour): exhaustively over 4-vertex undirected and
    3-vertex directed graphs with weights {0, 1, INF}, and on random directed graphs
    with many zero weights."""
    for W in all_undirected(4, [0, 1, INF]):
        _check_zero_weight_order_and_pred(W)
    for W in all_directed(3, [0, 1, INF]):
        _check_zero_weight_order_and_pred(W)
    rng = np.random.default_rng(11)
    for trial in range(150):
        n = int(rng.integers(4, 8))
        W = random_dense(rng, n, float(rng.uniform(0.3, 0.9)), 0, 3, directed=bool(trial % 2),
                         zero_prob=float(rng.uniform(0.2, 0.6)))
        _check_zero_weight_order_and_pred(W)


def test_random_against_floyd_warshall_bellman_ford_and_scipy():
    rng = np.random.default_rng(3)
    for trial in range(60):
        n = int(rng.integers(1, 65))
        directed = bool(trial % 2)
        W = random_dense(rng, n, float(rng.uniform(0.02, 0.8)), 1, 50, directed,
                         zero_prob=0.05 if trial % 3 == 0 else 0.0)
        D = oracle.floyd_warshall(W)
        for s in sorted({0, n // 2, n - 1}):
            dist, pred, _ = oracle.dijkstra(W, s)
            ref = scipy_dist(W, s)
            d64 = dist.astype(np.int64)
            assert (d64 == ref).all()
            assert (np.where(D[s] >= oracle.INF64, INF, D[s]) == d64).all()
            bf = oracle.bellman_ford(W, s)
            assert (np.where(bf >= oracle.INF64, INF, bf) == d64).all()
            assert oracle.certificate(W, s, dist, pred)[0] == 0


def test_closed_form_pred_equals_oracle_for_positive_weights():
    rng = np.random.default_rng(4)
    for trial in range(40):
        n = int(rng.integers(2, 200))
        W = random_dense(rng, n, float(rng.uniform(0.01, 0.6)), 1, int(rng.integers(1, 10)),
                         directed=bool(trial % 2))
        s = int(rng.integers(0, n))
        dist, pred, _ = oracle.dijkstra(W, s)
        assert (oracle.closed_form_pred(W, dist) == pred).all()
        assert (lexmin_tight_pred(W, dist) == pred).all() if n <= 60 else True


def test_settle_order_is_sorted_by_dist_then_index_for_positive_weights():
    rng = np.random.default_rng(5)
    for _ in range(30):
        n = int(rng.integers(2, 120))
        W = random_dense(rng, n, 0.2, 1, 3)
        dist, pred, order, r = oracle.dijkstra(W, 0, with_order=True)
        settled = order[:r]
        keys = [(int(dist[u]), int(u)) for u in settled]
        assert keys == sorted(keys)


def test_certificate_catches_planted_mistakes():
    rng = np.random.default_rng(6)
    W = random_dense(rng, 60, 0.15, 1, 9)
    dist, pred, _ = oracle.dijkstra(W, 0)
    assert oracle.certificate(W, 0, dist, pred)[0] == 0
    reach = [v for v in range(1, 60) if dist[v] != INF]
    v = reach[len(reach) // 2]
    d = dist.copy(); d[v] += 1
    assert oracle.certificate(W, 0, d, pred)[0] in (2, 3)
    d = dist.copy(); d[v] -= 1
    assert oracle.certificate(W, 0, d, pred)[0] in (2, 3)
    d = dist.copy(); d[0] = 1
    assert oracle.certificate(W, 0, d, pred)[0] == 1
    p = pred.copy(); p[v] = v
    assert oracle.certificate(W, 0, dist, p)[0] == 3
    # a non-tight in-neighbour as pred
    nt = [u for u in range(60) if u != v and W[u, v] != INF and dist[u] != INF
          and dist[u] + W[u, v] != dist[v]]
    if nt:
        p = pred.copy(); p[v] = nt[0]
        assert oracle.certificate(W, 0, dist, p)[0] == 3
    # an unreachable vertex claiming a pred
    W2 = W.copy(); W2[:, 59] = INF; W2[59, :] = INF; W2[59, 59] = 0
    d2, p2, _ = oracle.dijkstra(W2, 0)
    p2[59] = 0
    assert oracle.certificate(W2, 0, d2, p2)[0] == 4
    # a zero-weight pred cycle: two vertices at equal dist pointing at each other
    Z = from_edges(3, [(0, 1, 1), (1, 2, 0)])
    dz, pz, _ = oracle.dijkstra(Z, 0)
    pz[1], pz[2] = 2, 1
    assert oracle.certificate(Z, 0, dz, pz)[0] == 5


def test_special_cases():
    d, p, r = oracle.dijkstra(np.zeros((1, 1), np.int32), 0)
    assert d.tolist() == [0] and p.tolist() == [-1] and r == 1
    # complete graph with all weights c (the paper's complete dense graphs, Section IV-A)
    for n, c in ((10, 7), (100, 1)):
        W = np.full((n, n), c, np.int32); np.fill_diagonal(W, 0)
        for s in (0, n - 1):
            d, p, _ = oracle.dijkstra(W, s)
            assert all(d[v] == (0 if v == s else c) for v in range(n))
            assert all(p[v] == (-1 if v == s else s) for v in range(n))
    # isolated source
    W = random_dense(np.random.default_rng(7), 30, 0.5, 1, 5)
    W[4, :] = INF; W[:, 4] = INF; W[4, 4] = 0
    d, p, r = oracle.dijkstra(W, 4)
    assert r == 1 and (d == np.where(np.arange(30) == 4, 0, INF)).all() and (p == -1).all()
    # path graph: dist = prefix sums of the weights, pred = previous vertex
    ws = [3, 1, 4, 1, 5, 9, 2, 6]
    P = from_edges(9, [(i, i + 1, w) for i, w in enumerate(ws)])
    d, p, _ = oracle.dijkstra(P, 0)
    assert d.tolist() == [0] + list(np.cumsum(ws)) and p.tolist() == [-1] + list(range(8))
    # star: every leaf hangs off the centre
    S = from_edges(6, [(0, k, k) for k in range(1, 6)])
    d, p, _ = oracle.dijkstra(S, 3)
    assert d.tolist() == [3, 4, 5, 0, 7, 8] and p.tolist() == [3, 0, 0, -1, 0, 0]


def test_metamorphic_properties():
    rng = np.random.default_rng(8)
    for trial in range(20):
        n = int(rng.integers(2, 80))
        W = random_dense(rng, n, 0.2, 1, 30)
        s = int(rng.integers(0, n))
        d, p, _ = oracle.dijkstra(W, s)
        # scaling finite weights by k scales dist and keeps pred
        k = int(rng.integers(2, 6))
        Wk = np.where(W == INF, INF, W * k).astype(np.int32)
        dk, pk, _ = oracle.dijkstra(Wk, s)
        assert (dk == np.where(d == INF, INF, d * k)).all() and (pk == p).all()
        # relabelling vertices relabels dist
        perm = rng.permutation(n)
        Wp = W[np.ix_(perm, perm)]
        inv = np.argsort(perm)
        dp, _, _ = oracle.dijkstra(Wp, int(inv[s]))
        assert (dp[inv] == d).all()
        # undirected symmetry: dist_s[t] == dist_t[s]
        t = int(rng.integers(0, n))
        dt, _, _ = oracle.dijkstra(W, t)
        assert d[t] == dt[s]


def test_early_exit_changes_nothing():
    rng = np.random.default_rng(9)
    for _ in range(30):
        n = int(rng.integers(2, 60))
        W = random_dense(rng, n, 0.05, 1, 9, directed=True)
        a = oracle.dijkstra(W, 0, early_exit=True)
        b = oracle.dijkstra(W, 0, early_exit=False)
        assert (a[0] == b[0]).all() and (a[1] == b[1]).all() and a[2] == b[2]


def test_saturating_path_lengths_stay_unreachable():
    """A path whose length reaches INT32_MAX is not representable; it stays infinite."""
    big = INF - 1
    W = from_edges(3, [(0, 1, big), (1, 2, 5)], directed=True)
    d, p, _ = oracle.dijkstra(W, 0)
    assert d.tolist() == [0, big, INF] and p.tolist() == [-1, 0, -1]


def test_exhaustive_directed_n4():
    """All 3^12 directed 4-vertex graphs with arc weights in {1, 2, inf}, every source:
    dist against Floyd-Warshall computed here (vectorised over all graphs), and pred
    against the (dist[u], u)-lexmin tight tail, which is Algorithm 1's pred when every
    weight is at least 1 (settle order = (dist, index))."""
    n = 4
    arcs = [(i, j) for i in range(n) for j in range(n) if i != j]
    vals = np.array([1, 2, INF], np.int64)
    digits = (np.arange(3 ** len(arcs))[:, None] // 3 ** np.arange(len(arcs))[None, :]) % 3
    G = np.full((3 ** len(arcs), n, n), INF, np.int64)
    G[:, np.arange(n), np.arange(n)] = 0
    for k, (i, j) in enumerate(arcs):
        G[:, i, j] = vals[digits[:, k]]
    dist, pred = oracle.dijkstra_every_source(G.astype(np.int32))
    # Floyd-Warshall, all graphs at once (int64, INF as a large sentinel)
    BIG = np.int64(1) << 40
    D = np.where(G == INF, BIG, G)
    for k in range(n):
        D = np.minimum(D, D[:, :, k, None] + D[:, None, k, :])
    want = np.where(D >= BIG, INF, D)
    assert np.array_equal(dist.astype(np.int64), want)
    # pred: over tails u != v with a tight finite arc, the smallest (dist[u], u)
    du = dist.astype(np.int64)[:, :, :, None]            # [g, s, u, 1]
    dv = dist.astype(np.int64)[:, :, None, :]            # [g, s, 1, v]
    w = G[:, None, :, :]                                   # [g, 1, u, v]
    u_idx = np.arange(n)[None, None, :, None]
    tight = (w != INF) & (du != INF) & (dv != INF) & (du + w == dv) & (u_idx != np.arange(n)[None, None, None, :])
    key = np.where(tight, du * n + u_idx, np.iinfo(np.int64).max)
    best = key.min(axis=2)                                 # [g, s, v]
    lex = np.where(best == np.iinfo(np.int64).max, -1, best % n)
    lex[:, np.arange(n), np.arange(n)] = -1                # the source has no pred
    assert np.array_equal(pred.astype(np.int64), lex)
