"""GPU tests of the steps around the solve: edge list -> dense matrix on the device,
and hop counts / paths read out of pred, against the oracle."""
import numpy as np
import pytest

import gen
import oracle
from tests.graphs import INF, random_dense
from tests.test_oracle_io import PAPER_EDGES, edges_of

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_03667_amd as m
    m.lib()
    return m


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, np.int32)).cuda()


def test_edges_to_dense_matches_oracle(sp):
    rng = np.random.default_rng(500)
    u, v, w = (np.array(x, np.int32) for x in zip(*PAPER_EDGES))
    for directed in (False, True):
        W = torch.empty((4, 4), dtype=torch.int32, device="cuda")
        assert sp.sssp_edges_to_dense(dev(u), dev(v), dev(w), 4, W, directed=directed) == 0
        R, _ = oracle.edges_to_dense(u, v, w, 4, directed)
        assert np.array_equal(W.cpu().numpy(), R)
    for trial in range(8):
        n = int(rng.integers(1, 700))
        m = int(rng.integers(0, 5 * n))
        U = rng.integers(-2, n + 2, size=m).astype(np.int32)
        V = rng.integers(0, n, size=m).astype(np.int32)
        Wt = rng.integers(-1, 60, size=m).astype(np.int32)
        directed = bool(trial % 2)
        ld = n + (trial % 3)
        W = torch.full((n, ld), 12345, dtype=torch.int32, device="cuda")
        bad = sp.sssp_edges_to_dense(dev(U), dev(V), dev(Wt), n, W, directed=directed)
        R, bad_r = oracle.edges_to_dense(U, V, Wt, n, directed)
        assert bad == bad_r and np.array_equal(W.cpu().numpy()[:, :n], R), trial


def test_edge_list_of_the_medium_workload(sp):
    """The n=16384 workload's edge list, shuffled, rebuilds its matrix exactly; the solve on
    the rebuilt matrix equals the oracle."""
    spec = gen.workload_single_medium().graphs[0]
    Wh = gen.dense_host(spec)
    u, v, w = edges_of(Wh, spec.directed)
    perm = np.random.default_rng(501).permutation(len(u))
    W = torch.empty((spec.n, spec.n), dtype=torch.int32, device="cuda")
    assert sp.sssp_edges_to_dense(dev(u[perm]), dev(v[perm]), dev(w[perm]), spec.n, W) == 0
    assert gen.checksum_device(W) == gen.checksum_host(Wh)
    d, p = sp.solve(W, 7)
    dr, pr, _ = oracle.dijkstra(Wh, 7)
    assert np.array_equal(d.cpu().numpy(), dr) and np.array_equal(p.cpu().numpy(), pr)


def test_hops_and_paths(sp):
    rng = np.random.default_rng(502)
    for trial in range(6):
        n = int(rng.integers(2, 3000))
        Wh = random_dense(rng, n, float(rng.choice([0.002, 0.02, 0.3])), 1, 20, directed=bool(trial % 2))
        src = int(rng.integers(0, n))
        W = dev(Wh)
        d, p = sp.solve(W, src)
        hops = torch.empty(n, dtype=torch.int32, device="cuda")
        sp.sssp_hops(p, d, hops)
        dd, pp = d.cpu().numpy(), p.cpu().numpy()
        assert np.array_equal(hops.cpu().numpy(), oracle.hops(pp, dd))
        targets = sorted(set(rng.integers(0, n, size=20).tolist()) | {src, n - 1})
        got = sp.paths(p, d, targets)
        for t, path in zip(targets, got):
            path = path.cpu().numpy().tolist()
            if dd[t] == INF:
                assert path == []
                continue
            walk = [t]
            while pp[walk[-1]] >= 0:
                walk.append(int(pp[walk[-1]]))
            assert path == walk[::-1] and path[0] == src
            assert sum(int(Wh[a, b]) for a, b in zip(path, path[1:])) == dd[t]


def test_stream_read_diagnostic(sp):
    """sssp_stream_read reads every 16-byte word of the buffer exactly once (the xor of
    all words it reports equals the buffer's, which a skipped or repeated chunk would
    change), for ragged sizes and several chunk sizes, three calls in a row (the
    claim counter resets itself), and leaves the buffer unchanged."""
    rng = np.random.default_rng(501)
    for words, chunk in ((1, 0), (65, 1024), (4097, 0), (1_000_003, 16384), (4_194_304, 0), (3_000_001, 1 << 20)):
        host = rng.integers(-2**31, 2**31, size=4 * words, dtype=np.int64).astype(np.int32)
        buf = torch.from_numpy(host).cuda()
        want = int(np.bitwise_xor.reduce(host.view(np.uint32)))
        for rep in range(3):
            fold = torch.zeros(1, dtype=torch.int32, device="cuda")
            sp.sssp_stream_read(buf, chunk_bytes=chunk, fold=fold)
            torch.cuda.synchronize()
            assert int(fold.item()) & 0xFFFFFFFF == want, (words, chunk, rep)
        assert np.array_equal(buf.cpu().numpy(), host)
    # a prefix of the buffer
    host = rng.integers(-2**31, 2**31, size=4 * 1000, dtype=np.int64).astype(np.int32)
    buf = torch.from_numpy(host).cuda()
    fold = torch.zeros(1, dtype=torch.int32, device="cuda")
    sp.sssp_stream_read(buf, nbytes=16 * 300, fold=fold)
    torch.cuda.synchronize()
    assert int(fold.item()) & 0xFFFFFFFF == int(np.bitwise_xor.reduce(host[:1200].view(np.uint32)))


def test_edges_to_dense_beyond_32bit_offsets(sp):
    """An edge list written into a 25.6 GB matrix (n = 80000: element offsets past
    2^32), with edges at the last row and column: the device matrix's checksum equals
    that of the oracle's host matrix, and the last row and column match exactly."""
    n = 80000
    eu, ev, ew = gen.sparse_edges(n, 3 * n, 1, 1000, 1503)
    eu = np.concatenate([eu, np.array([n - 1, 1, n - 1], np.int32)])
    ev = np.concatenate([ev, np.array([0, n - 1, n - 2], np.int32)])
    ew = np.concatenate([ew, np.array([5, 7, 0], np.int32)])
    W = torch.empty((n, n), dtype=torch.int32, device="cuda")
    assert sp.sssp_edges_to_dense(dev(eu), dev(ev), dev(ew), n, W) == 0
    R, bad = oracle.edges_to_dense(eu, ev, ew, n)
    assert bad == 0
    assert gen.checksum_device(W) == gen.checksum_host(R)
    assert np.array_equal(W[n - 1].cpu().numpy(), R[n - 1])
    assert np.array_equal(W[:, n - 1].cpu().numpy(), R[:, n - 1])
    del W
    torch.cuda.empty_cache()
