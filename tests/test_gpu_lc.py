"""GPU parity of the label-correcting solve (SSSP_FLAG_LABEL_CORRECTING), through
the C ABI: dist and pred equal Algorithm 1's (the oracle) bit for bit, and the
sweep and row counts equal those of the label-correcting oracle."""
import numpy as np
import pytest

import gen
import oracle
from tests.graphs import INF, golden_cases, random_dense

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LC, SINGLE = 16, 2


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_03667_amd as m
    m.lib()
    return m


def tight_zero_edge(W, dist):
    n = W.shape[0]
    z = (W == 0) & ~np.eye(n, dtype=bool)
    fin = dist != INF
    return bool((z & (dist[:, None] == dist[None, :]) & fin[:, None]).any())


def check_lc(sp, W, src, workgroups=0, single=False, Wt=None, tag=""):
    if Wt is None:
        Wt = torch.from_numpy(np.ascontiguousarray(W)).cuda()
    d, p = sp.solve(Wt, src, flags=LC | (SINGLE if single else 0), workgroups=workgroups)
    status, stats = sp.sssp_last_status()
    d, p = d.cpu().numpy(), p.cpu().numpy()
    dr, pr, _ = oracle.dijkstra(W, src)
    assert status & 3 == 0, (tag, status)
    bad = np.nonzero((d != dr) | (p != pr))[0]
    assert bad.size == 0, (tag, "n", W.shape[0], "src", src, bad[:5].tolist(), d[bad[:5]].tolist(),
                           dr[bad[:5]].tolist(), p[bad[:5]].tolist(), pr[bad[:5]].tolist())
    fell_back = bool(status & 4)
    assert fell_back == tight_zero_edge(W, dr), (tag, status)
    if not fell_back:
        _, sweeps, rows = oracle.label_correcting(W, src)
        reach = int((dr != INF).sum())
        assert (stats[0], stats[1]) == (sweeps, rows + reach), (tag, stats, sweeps, rows, reach)
    return status


def test_worked_examples(sp):
    for name, W, expect in golden_cases():
        for src, e in expect.items():
            for single in (False, True):
                Wt = torch.from_numpy(W).cuda()
                d, p = sp.solve(Wt, src, flags=LC | (SINGLE if single else 0))
                assert d.cpu().tolist() == e["dist"] and p.cpu().tolist() == e["pred"], (name, src, single)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 64, 127, 128, 129, 255, 1000, 1023, 1025, 2047, 3001, 4097])
def test_sizes_and_slices(sp, n):
    rng = np.random.default_rng(700 + n)
    for trial, (p, hi) in enumerate([(0.3, 9), (0.02, 1000), (min(1.0, 8.0 / n), 100)]):
        W = random_dense(rng, n, p, 1, hi, directed=bool(trial % 2))
        Wt = torch.from_numpy(W).cuda()
        srcs = sorted({0, n - 1, int(rng.integers(0, n))})
        for src in srcs:
            check_lc(sp, W, src, Wt=Wt, tag=("default", n, trial))
        check_lc(sp, W, srcs[-1], workgroups=3, Wt=Wt, tag=("wg3", n, trial))
        if n <= 16384:
            check_lc(sp, W, srcs[0], single=True, Wt=Wt, tag=("single", n, trial))


def test_workgroup_counts(sp):
    rng = np.random.default_rng(710)
    W = random_dense(rng, 2500, 0.01, 1, 500)
    Wt = torch.from_numpy(W).cuda()
    for wg in (1, 2, 7, 17, 64, 200, 625):
        check_lc(sp, W, 11, workgroups=wg, Wt=Wt, tag=("wg", wg))


def test_zero_weights_fall_back_exactly(sp):
    rng = np.random.default_rng(711)
    seen_fallback = seen_clean = 0
    for trial in range(12):
        n = int(rng.integers(50, 1500))
        W = random_dense(rng, n, 0.05, 0 if trial % 3 else 1, 20, directed=bool(trial % 2),
                         zero_prob=0.05 if trial % 3 else 0.0)
        src = int(rng.integers(0, n))
        status = check_lc(sp, W, src, tag=("zero", trial))
        check_lc(sp, W, src, single=True, tag=("zero-single", trial))
        if status & 4:
            seen_fallback += 1
        else:
            seen_clean += 1
    assert seen_fallback > 0 and seen_clean > 0


def test_special_graphs(sp):
    # empty graph, complete graph with equal weights (every pred = src), a path
    n = 700
    W = np.full((n, n), INF, np.int32)
    np.fill_diagonal(W, 0)
    check_lc(sp, W, 5, tag="empty")
    C = np.full((n, n), 3, np.int32)
    np.fill_diagonal(C, 0)
    check_lc(sp, C, 9, tag="complete")
    P = np.full((n, n), INF, np.int32)
    np.fill_diagonal(P, 0)
    for i in range(n - 1):
        P[i, i + 1] = P[i + 1, i] = 1 + i % 5
    check_lc(sp, P, 0, tag="path")
    check_lc(sp, P, n // 2, workgroups=9, tag="path-mid")


def test_strides(sp):
    rng = np.random.default_rng(712)
    n = 1500
    W = random_dense(rng, n, 0.02, 1, 100)
    for ld in (n + 4, n + 1):  # padded aligned rows, then rows that need scalar loads
        big = torch.full((n, ld), 0x12345678, dtype=torch.int32)
        big[:, :n] = torch.from_numpy(W)
        Wt = big.cuda()[:, :n]
        check_lc(sp, W, 3, Wt=Wt, tag=("ld", ld))


def test_sparse_many_levels(sp):
    """Sparse graphs with a wide weight range: hundreds of distinct distances, few sweeps."""
    for seed, (n, p) in enumerate([(4096, 0.002), (8192, 0.001)]):
        W = gen.dense_host(gen.GraphSpec(n, p, 1, 1000, 800 + seed))
        for src in (0, n // 3):
            check_lc(sp, W, src, tag=("sparse", n))


def test_medium_workload(sp):
    """n=16384, p=0.01, undirected and directed, sources 0, 7 and 12345."""
    wl = gen.workload_single_medium()
    for gi, g in enumerate(wl.graphs):
        Wh = gen.dense_host(g)
        Wt = gen.dense_device(g)
        for g2, src in wl.instances:
            if g2 == gi:
                check_lc(sp, Wh, src, Wt=Wt, tag=("medium", g.directed, src))
