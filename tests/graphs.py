"""Small hand-built graphs and brute-force references used by the CPU tests.

Nothing here follows the paper's algorithm: distances come from enumerating
simple paths, which is the plain definition of a shortest path.
"""
import itertools
import json
import os

import numpy as np

INF = 0x7FFFFFFF
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def from_edges(n, edges, directed=False):
    W = np.full((n, n), INF, dtype=np.int32)
    np.fill_diagonal(W, 0)
    for u, v, w in edges:
        W[u, v] = w
        if not directed:
            W[v, u] = w
    return W


def decode(x):
    return INF if x == "inf" else int(x)


def golden_cases():
    with open(os.path.join(GOLDEN, "worked_examples.json")) as f:
        data = json.load(f)
    out = []
    for c in data["cases"]:
        if "W" in c:
            W = np.array([[decode(x) for x in row] for row in c["W"]], dtype=np.int32)
        else:
            W = from_edges(c["n"], c["edges_undirected"])
        exp = {int(s): {k: [decode(x) for x in v] for k, v in e.items()}
               for s, e in c["expect"].items()}
        out.append((c["name"], W, exp))
    return out


def brute_force_dist(W, src):
    """Minimum over all simple paths src -> v of the summed weights (tiny n only)."""
    n = W.shape[0]
    best = [INF] * n
    best[src] = 0

    def walk(u, length, seen):
        for v in range(n):
            w = int(W[u, v])
            if v in seen or w == INF:
                continue
            L = length + w
            if L < best[v]:
                best[v] = L
            walk(v, L, seen | {v})

    walk(src, 0, {src})
    return np.array([b if b < INF else INF for b in best], dtype=np.int64)


def lexmin_tight_pred(W, dist):
    """pred[v] = u minimising (dist[u], u) over tight in-edges u -> v, u != v (pure Python)."""
    n = W.shape[0]
    pred = [-1] * n
    for v in range(n):
        if dist[v] == INF:
            continue
        cands = [(int(dist[u]), u) for u in range(n)
                 if u != v and W[u, v] != INF and dist[u] != INF
                 and int(dist[u]) + int(W[u, v]) == int(dist[v])]
        if cands:
            pred[v] = min(cands)[1]
    return np.array(pred, dtype=np.int32)


def order_and_pred_from_distances(W, src, dist):
    """Settle order and pred of Algorithm 1 rebuilt from the final distances alone,
    valid with zero weights too (pure Python, tiny n).

    Algorithm 1 settles the unvisited vertex of least (tentative distance, index).
    An unvisited v has tentative distance equal to dist[v] exactly when some
    settled u is a tight in-neighbour (dist[u] + W[u, v] == dist[v]), and more
    otherwise; and the least tentative distance among unvisited vertices is always
    reached by such an "available" vertex (the first unvisited vertex on a shortest
    path to any other one is available and no farther).  So the next settled vertex
    is the available vertex of least (dist, index).  Relaxation lowers only on
    strict improvement, so pred[v] is the first tight in-neighbour settled before v
    (none for the source)."""
    n = W.shape[0]
    settled, done, avail = [], [False] * n, {src}
    while avail:
        v = min(avail, key=lambda x: (int(dist[x]), x))
        avail.discard(v)
        done[v] = True
        settled.append(v)
        for x in range(n):
            if not done[x] and x != v and W[v, x] != INF and int(dist[v]) + int(W[v, x]) == int(dist[x]):
                avail.add(x)
    pred = [-1] * n
    for k, v in enumerate(settled):
        for u in settled[:k]:
            if W[u, v] != INF and int(dist[u]) + int(W[u, v]) == int(dist[v]):
                pred[v] = u
                break
    return settled, np.array(pred, dtype=np.int32)


def all_undirected(n, weights):
    """Every undirected graph on n vertices with each pair's weight drawn from `weights`."""
    pairs = list(itertools.combinations(range(n), 2))
    for combo in itertools.product(weights, repeat=len(pairs)):
        W = np.full((n, n), INF, dtype=np.int32)
        np.fill_diagonal(W, 0)
        for (i, j), w in zip(pairs, combo):
            W[i, j] = W[j, i] = w
        yield W


def all_directed(n, weights):
    pairs = [(i, j) for i in range(n) for j in range(n) if i != j]
    for combo in itertools.product(weights, repeat=len(pairs)):
        W = np.full((n, n), INF, dtype=np.int32)
        np.fill_diagonal(W, 0)
        for (i, j), w in zip(pairs, combo):
            W[i, j] = w
        yield W


def random_dense(rng, n, p, lo, hi, directed=False, zero_prob=0.0):
    W = np.full((n, n), INF, dtype=np.int32)
    mask = rng.random((n, n)) < p
    w = rng.integers(lo, hi + 1, size=(n, n)).astype(np.int32)
    if zero_prob:
        w[rng.random((n, n)) < zero_prob] = 0
    W[mask] = w[mask]
    if not directed:
        iu = np.triu_indices(n, 1)
        W[(iu[1], iu[0])] = W[iu]
    np.fill_diagonal(W, 0)
    return W
