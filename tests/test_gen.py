"""Input generator checks (CPU): the C generator against a numpy re-computation,
the published SplitMix64 test vector, structural properties and manifest determinism."""
import numpy as np

import gen


def test_splitmix64_published_vector():
    # first outputs of the SplitMix64 reference generator seeded with 1234567
    s = gen.Stream(1234567)
    assert [s.next_u64() for _ in range(5)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_host_generator_matches_numpy_recomputation():
    for spec in (gen.GraphSpec(257, 0.3, 1, 100, 11), gen.GraphSpec(130, 0.7, 5, 9, 12, True),
                 gen.GraphSpec(64, 1.0, 1, 1000, 13), gen.GraphSpec(33, 0.0, 1, 1, 14, True)):
        assert (gen.dense_host(spec) == gen.dense_numpy(spec)).all()


def test_structure():
    u = gen.dense_host(gen.GraphSpec(500, 0.2, 1, 100, 21))
    assert (u == u.T).all() and (np.diag(u) == 0).all()
    off = u[~np.eye(500, dtype=bool)]
    fin = off[off != gen.INF]
    assert fin.min() >= 1 and fin.max() <= 100
    assert abs((off != gen.INF).mean() - 0.2) < 0.01
    d = gen.dense_host(gen.GraphSpec(500, 0.2, 1, 100, 21, directed=True))
    assert not (d == d.T).all()
    assert (gen.dense_host(gen.GraphSpec(50, 0.0, 1, 9, 3))[~np.eye(50, dtype=bool)] == gen.INF).all()
    assert (gen.dense_host(gen.GraphSpec(50, 1.0, 1, 9, 3)) != gen.INF).all()


def test_rows_and_padding_and_checksum():
    spec = gen.GraphSpec(300, 0.1, 1, 50, 99)
    W = gen.dense_host(spec)
    assert (gen.dense_rows_host(spec, 100, 37) == W[100:137]).all()
    Wp = gen.dense_host(spec, ld=304)
    assert (Wp[:, :300] == W).all() and (Wp[:, 300:] == gen.INF).all()
    c = gen.checksum_host(W)
    W2 = W.copy(); W2[5, 6] ^= 1
    assert gen.checksum_host(W2) != c and gen.checksum_host(W.copy()) == c


def test_manifests_are_deterministic():
    a, b = gen.workload_batched(), gen.workload_batched()
    assert [g.__dict__ for g in a.graphs] == [g.__dict__ for g in b.graphs]
    assert a.instances == b.instances and len(a.instances) == 320
    srcs = [s for g, s in a.instances if g == 0]
    assert len(set(srcs)) == 256
    for g in a.graphs[1:]:
        assert 512 <= g.n <= 8192 and 0.005 <= g.p <= 0.5
    s1 = gen.workload_serving(n_queries=500)
    s2 = gen.workload_serving(n_queries=500)
    assert [q.__dict__ for q in s1.queries] == [q.__dict__ for q in s2.queries]
    for g in s1.graphs:
        assert 256 <= g.n <= 32768 and 0.001 <= g.p <= 0.5
    for q in s1.queries:
        assert 0 <= q.src < s1.graphs[q.graph].n
    gaps = np.diff([0.0] + [q.arrival_s for q in s1.queries])
    assert (gaps > 0).all() and 1 / 4000 < gaps.mean() < 1 / 1000
