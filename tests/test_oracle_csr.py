"""Pins for the oracle's adjacency-list (CSR) functions: Algorithm 1 over edge lists
against Algorithm 1 over the matrix the same edge list builds (duplicates, self-loops,
zero weights, out-of-range edges), the certificate against planted mistakes, and the
closed-form pred against the matrix version; plus the seeded sparse edge generator."""
import numpy as np

import gen
import oracle
from tests.graphs import INF


def random_edges(rng, n, m, lo, hi, bad=0):
    eu = rng.integers(0, n, size=m).astype(np.int32)
    ev = rng.integers(0, n, size=m).astype(np.int32)
    ew = rng.integers(lo, hi + 1, size=m).astype(np.int32)
    if bad:
        k = rng.integers(0, m, size=bad)
        eu[k[: bad // 2]] = n + 3  # endpoint out of range
        ew[k[bad // 2:]] = -5       # negative weight: skipped by both conversions
    return eu, ev, ew


def test_csr_dijkstra_equals_matrix_dijkstra():
    rng = np.random.default_rng(800)
    for trial in range(300):
        n = int(rng.integers(1, 40))
        m = int(rng.integers(0, 4 * n + 1))
        directed = bool(trial % 2)
        eu, ev, ew = random_edges(rng, n, m, 0 if trial % 3 == 0 else 1, int(rng.choice([3, 50, 1000])),
                                  bad=2 if trial % 5 == 0 and m > 4 else 0)
        W, _ = oracle.edges_to_dense(eu, ev, ew, n, directed)
        rp, col, w = oracle.edges_to_csr(eu, ev, ew, n, directed)
        src = int(rng.integers(0, n))
        d1, p1, r1 = oracle.dijkstra(W, src)
        d2, p2, r2 = oracle.dijkstra_csr(rp, col, w, src)
        assert np.array_equal(d1, d2) and np.array_equal(p1, p2) and r1 == r2, (trial, n, m)


def test_csr_certificate_and_closed_form():
    rng = np.random.default_rng(801)
    for trial in range(100):
        n = int(rng.integers(2, 60))
        eu, ev, ew = random_edges(rng, n, 3 * n, 1, 20)
        rp, col, w = oracle.edges_to_csr(eu, ev, ew, n, bool(trial % 2))
        W, _ = oracle.edges_to_dense(eu, ev, ew, n, bool(trial % 2))
        d, p, _ = oracle.dijkstra_csr(rp, col, w, 0)
        assert oracle.certificate_csr(rp, col, w, 0, d, p)[0] == 0
        cf = oracle.closed_form_pred_csr(rp, col, w, d)
        cf[0] = -1
        assert np.array_equal(cf, p)  # weights >= 1: the closed form is Algorithm 1's pred
        cfd = oracle.closed_form_pred(W, d)
        cfd[0] = -1
        assert np.array_equal(cf, cfd)
        reach = np.nonzero((d != INF) & (np.arange(n) != 0))[0]
        if reach.size:
            v = int(reach[0])
            bad = d.copy()
            bad[v] += 1
            assert oracle.certificate_csr(rp, col, w, 0, bad, p)[0] in (2, 3)
            badp = p.copy()
            badp[v] = v
            assert oracle.certificate_csr(rp, col, w, 0, d, badp)[0] == 3
        unreach = np.nonzero(d == INF)[0]
        if unreach.size:
            badp = p.copy()
            badp[int(unreach[0])] = 0
            assert oracle.certificate_csr(rp, col, w, 0, d, badp)[0] == 4


def test_sparse_generator():
    u1, v1, w1 = gen.sparse_edges(1000, 3000, 1, 1000, 42)
    u2, v2, w2 = gen.sparse_edges(1000, 3000, 1, 1000, 42)
    assert np.array_equal(u1, u2) and np.array_equal(v1, v2) and np.array_equal(w1, w2)
    assert u1.min() >= 0 and u1.max() < 1000 and v1.min() >= 0 and v1.max() < 1000
    assert w1.min() >= 1 and w1.max() <= 1000
    u3, _, _ = gen.sparse_edges(1000, 3000, 1, 1000, 43)
    assert not np.array_equal(u1, u3)
    # a prefix of a longer list is the shorter list (edge e depends on (seed, e) only)
    u4, v4, w4 = gen.sparse_edges(1000, 5000, 1, 1000, 42)
    assert np.array_equal(u4[:3000], u1) and np.array_equal(w4[:3000], w1)
    _, specs = gen.workload_sparse()
    assert [s.n for s in specs][:3] == [10000, 20000, 40000] and all(s.m == 3 * s.n for s in specs)
