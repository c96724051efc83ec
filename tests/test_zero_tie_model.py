"""CPU model of how the adjacency-list solve sets pred when tight zero-weight
edges exist, checked against the oracle (Algorithm 1 run literally) before any
kernel runs.  Not an oracle: a pure-Python statement of the kernel's strategy.

Strategy, from the exact distances D alone.  Algorithm 1 settles vertices level
by level (a level: all vertices of one distance).  Inside a level the seeds (the
source, and heads of tight edges of positive weight, whose tails lie in lower
levels) are available from the start, and settling a vertex makes the heads of
its tight zero-weight edges available; the lowest-index available vertex is
settled next.  Vertices touched by no tight zero-weight edge inside their level
("plain") are seeds that make nothing available, so only the others need the
sequential pass: their settle sequence y_1, y_2, ... is the same whether or not
the plain vertices are interleaved, and a plain vertex p settles before y_i
exactly when p < max(y_1 .. y_i).  So within a level the order is the order of
the 64-bit keys (p << 32) for plain p and (max(y_1 .. y_i) << 32) | i for y_i,
and pred[v] is the tail of the first-settled tight edge into v: the smallest
(D[u], key[u]) over tight edges u -> v, u != v."""
import numpy as np

import oracle
from tests.graphs import INF, random_dense

def lists_of(W):
    n = W.shape[0]
    rp, col, w = [0], [], []
    for u in range(n):
        for v in range(n):
            if v != u and W[u, v] != INF:
                col.append(v)
                w.append(int(W[u, v]))
        rp.append(len(col))
    return np.array(rp, np.int64), np.array(col, np.int32), np.array(w, np.int32)


def zero_tie_pred(rp, col, w, src, D, index_order=False):
    """index_order: a planted mistake, every level settled in index order."""
    n = rp.size - 1
    tight = []  # (u, v, w) with u != v, D[u] + w == D[v] < INF
    for u in range(n):
        if D[u] == INF:
            continue
        for e in range(rp[u], rp[u + 1]):
            v, wt = int(col[e]), int(w[e])
            if v != u and 0 <= wt < INF and D[u] + wt == D[v]:
                tight.append((u, v, wt))
    nonplain = set()
    seed = {src}
    zero_out = {}
    for u, v, wt in tight:
        if wt == 0:
            nonplain |= {u, v}
            zero_out.setdefault(u, []).append(v)
        else:
            seed.add(v)
    key = {v: v << 32 for v in range(n)}
    levels = {}
    for v in nonplain:
        levels.setdefault(int(D[v]), []).append(v)
    for members in ([] if index_order else levels.values()):
        avail = {v for v in members if v in seed}
        done = set()
        pm, step = 0, 0
        while avail - done:
            x = min(avail - done)  # the lowest-index available vertex settles next
            done.add(x)
            pm = max(pm, x)
            step += 1
            key[x] = (pm << 32) | step
            avail |= {y for y in zero_out.get(x, []) if y in nonplain}
        assert done == set(members)  # every member is reached from the seeds
    pred = np.full(n, -1, np.int32)
    best = {}
    for u, v, wt in tight:
        k = (int(D[u]), key[u])
        if v not in best or k < best[v][0]:
            best[v] = (k, u)
    for v, (_, u) in best.items():
        if v != src:
            pred[v] = u
    return pred


def check_lists(rp, col, w, src):
    dr, pr, _ = oracle.dijkstra_csr(rp, col, w, src)
    p = zero_tie_pred(rp, col, w, src, dr)
    assert np.array_equal(p, pr), (src, p.tolist(), pr.tolist())


def test_all_four_vertex_undirected_graphs_with_zero_weights():
    vals = (0, 1, INF)
    pairs = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    count = 0
    for code in range(3 ** 6):
        W = np.full((4, 4), INF, np.int32)
        np.fill_diagonal(W, 0)
        c = code
        for u, v in pairs:
            W[u, v] = W[v, u] = vals[c % 3]
            c //= 3
        rp, col, w = lists_of(W)
        for src in range(4):
            check_lists(rp, col, w, src)
            count += 1
    assert count == 4 * 729


def test_random_graphs_with_many_zero_weights():
    rng = np.random.default_rng(2504)
    for t in range(1500):
        n = int(rng.integers(2, 24))
        W = random_dense(rng, n, float(rng.choice([0.1, 0.25, 0.5])), 0, int(rng.choice([1, 2, 5])),
                         directed=bool(t % 2), zero_prob=float(rng.choice([0.2, 0.5, 0.8])))
        rp, col, w = lists_of(W)
        check_lists(rp, col, w, int(rng.integers(0, n)))


def test_edge_lists_with_repeats_and_self_loops():
    """Lists with repeated pairs (the smallest weight counts), self-loops and zero
    weights, as the adjacency-list solve takes them."""
    rng = np.random.default_rng(2505)
    for t in range(800):
        n = int(rng.integers(2, 40))
        m = int(rng.integers(1, 4 * n))
        eu = rng.integers(0, n, size=m).astype(np.int32)
        ev = rng.integers(0, n, size=m).astype(np.int32)
        ew = rng.integers(0, 4, size=m).astype(np.int32)
        ew[rng.random(m) < 0.4] = 0
        rp, col, w = oracle.edges_to_csr(eu, ev, ew, n, bool(t % 2))
        check_lists(rp, col, w, int(rng.integers(0, n)))


def test_plain_order_rule_is_needed():
    """Planted mistakes in the model disagree with the oracle: settling each level
    in index order, and a hand-made case whose pred depends on a plain vertex
    settling between two members of the sequential pass."""
    rng = np.random.default_rng(2506)
    wrong = 0
    for t in range(400):
        n = int(rng.integers(3, 16))
        W = random_dense(rng, n, 0.4, 0, 3, directed=bool(t % 2), zero_prob=0.5)
        rp, col, w = lists_of(W)
        dr, pr, _ = oracle.dijkstra_csr(rp, col, w, 0)
        wrong += not np.array_equal(zero_tie_pred(rp, col, w, 0, dr, index_order=True), pr)
    assert wrong > 0
    # Level 1 is {1, 2, 3, 5}: 2, 3 and 5 are seeds (positive tight edges from 0) and 1
    # is reached by the zero edge 3 -> 1.  The sequential pass covers 3 and 1 (keys
    # (3, 1) and (3, 2)); the plain seeds 2 and 5 keep (2, 0) and (5, 0), so 2 settles
    # before 3 and 5 after 1: Algorithm 1's order 0, 2, 3, 1, 5.  Vertex 4 has tight
    # edges from 1, 2 and 5, so pred[4] = 2, where index order would give 1.
    edges = [(0, 2, 1), (0, 3, 1), (0, 5, 1), (3, 1, 0), (1, 4, 4), (2, 4, 4), (5, 4, 4)]
    W = np.full((6, 6), INF, np.int32)
    np.fill_diagonal(W, 0)
    for u, v, wt in edges:
        W[u, v] = wt
    rp, col, w = lists_of(W)
    dr, pr, order, _ = oracle.dijkstra(W, 0, with_order=True)
    assert order[:5].tolist() == [0, 2, 3, 1, 5] and pr[4] == 2
    assert zero_tie_pred(rp, col, w, 0, dr)[4] == 2
    assert zero_tie_pred(rp, col, w, 0, dr, index_order=True)[4] == 1
