"""Pins for the oracle's input step (edge list -> matrix) and output step (hops along
pred): the paper's printed matrices, a round trip through generated matrices with
shuffled duplicate edges, and BFS depths in the pred tree."""
import numpy as np

import gen
import oracle
from tests.graphs import INF, golden_cases, random_dense

# the edges of the paper's 4-vertex example (Section III-A), tail < head
PAPER_EDGES = [(0, 1, 2), (0, 2, 4), (1, 2, 1), (1, 3, 3), (2, 3, 5)]


def test_paper_edge_list_gives_printed_matrices():
    cases = {name: W for name, W, _ in golden_cases()}
    u, v, w = zip(*PAPER_EDGES)
    Wu, bad = oracle.edges_to_dense(u, v, w, 4, directed=False)
    assert bad == 0 and (Wu == cases["undirected_4"]).all()
    Wd, bad = oracle.edges_to_dense(u, v, w, 4, directed=True)
    assert bad == 0 and (Wd == cases["directed_4"]).all()


def edges_of(W, directed):
    n = W.shape[0]
    iu = np.argwhere((W != INF) & ~np.eye(n, dtype=bool))
    if not directed:
        iu = iu[iu[:, 0] < iu[:, 1]]
    return iu[:, 0].astype(np.int32), iu[:, 1].astype(np.int32), W[iu[:, 0], iu[:, 1]].astype(np.int32)


def test_round_trip_with_duplicates_self_loops_and_bad_edges():
    rng = np.random.default_rng(400)
    for spec in (gen.GraphSpec(300, 0.05, 1, 100, 1), gen.GraphSpec(200, 0.2, 1, 9, 2, directed=True)):
        W = gen.dense_host(spec)
        u, v, w = edges_of(W, spec.directed)
        k = len(u) // 3
        pick = rng.integers(0, len(u), size=k)
        # duplicates with heavier weights, flipped orientation for undirected graphs
        du, dv = (v[pick], u[pick]) if not spec.directed else (u[pick], v[pick])
        loops = rng.integers(0, spec.n, size=7).astype(np.int32)
        U = np.concatenate([u, du, loops, [-1, 5, spec.n]]).astype(np.int32)
        V = np.concatenate([v, dv, loops, [0, spec.n + 3, 1]]).astype(np.int32)
        Wt = np.concatenate([w, w[pick] + rng.integers(0, 50, size=k), np.full(7, 3), [1, 1, 1]]).astype(np.int32)
        perm = rng.permutation(len(U))
        R, bad = oracle.edges_to_dense(U[perm], V[perm], Wt[perm], spec.n, spec.directed)
        assert bad == 3 and (R == W).all()


def test_hops_equal_bfs_depth_in_pred_tree():
    rng = np.random.default_rng(401)
    for _ in range(10):
        n = int(rng.integers(2, 300))
        W = random_dense(rng, n, 0.05, 1, 9, directed=True)
        src = int(rng.integers(0, n))
        d, p, _ = oracle.dijkstra(W, src)
        h = oracle.hops(p, d)
        children = {}
        for x in range(n):
            if p[x] >= 0:
                children.setdefault(int(p[x]), []).append(x)
        depth = {src: 0}
        frontier = [src]
        while frontier:
            nxt = []
            for x in frontier:
                for c in children.get(x, []):
                    depth[c] = depth[x] + 1
                    nxt.append(c)
            frontier = nxt
        for x in range(n):
            assert h[x] == (depth[x] if d[x] != INF else -1)
