"""GPU tests of graphs stored as adjacency lists (CSR), through the C ABI.  The device
edge-list conversion means the same graph as the oracle's matrix conversion of the
same edges; the CSR solve equals Algorithm 1 (the oracle over the oracle's own lists)
bit for bit, whether it is given those lists (unsorted rows, repeated pairs,
self-loops) or the device conversion of the same edges."""
import numpy as np
import pytest

import gen
import oracle
from tests.graphs import INF

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
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def random_edges(rng, n, m, lo, hi, zero_prob=0.0, bad=0):
    eu = rng.integers(0, n, size=m).astype(np.int32)
    ev = rng.integers(0, n, size=m).astype(np.int32)
    ew = rng.integers(lo, hi + 1, size=m).astype(np.int32)
    if zero_prob:
        ew[rng.random(m) < zero_prob] = 0
    if bad and m >= bad:
        k = rng.choice(m, size=bad, replace=False)
        eu[k[: bad // 3]] = -1
        ev[k[bad // 3: 2 * bad // 3]] = n
        ew[k[2 * bad // 3:]] = INF
    return eu, ev, ew


def tight_zero_edge(rp, col, w, dist):
    n = rp.size - 1
    u = np.repeat(np.arange(n), np.diff(rp))
    ok = (col != u) & (w == 0) & (dist[u] != INF)
    return bool(np.any(ok & (dist[u] == dist[col])))


class Graph:
    """One edge list: the oracle's lists on the host and on the device, and the
    device conversion of the same edges."""

    def __init__(self, sp, eu, ev, ew, n, directed):
        self.n = n
        self.host = oracle.edges_to_csr(eu, ev, ew, n, directed)
        self.dev_oracle_lists = tuple(dev(a) for a in self.host)
        rp, col, w, self.bad = sp.csr_from_edges(dev(eu), dev(ev), dev(ew), n, directed)
        self.dev_converted = (rp, col, w)
        self._ref = {}

    def ref(self, src):
        if src not in self._ref:
            self._ref[src] = oracle.dijkstra_csr(*self.host, src)
        return self._ref[src]


def check(sp, g, src, lists, workgroups=0, tag=""):
    d, p = sp.csr_solve(*lists, src, workgroups=workgroups)
    status, stats = sp.sssp_last_status()
    dr, pr, _ = g.ref(src)
    assert status & 3 == 0, (tag, status)
    d, p = d.cpu().numpy(), p.cpu().numpy()
    bad = np.nonzero((d != dr) | (p != pr))[0]
    assert bad.size == 0, (tag, g.n, src, workgroups, bad[:5].tolist(), d[bad[:5]].tolist(),
                           dr[bad[:5]].tolist(), p[bad[:5]].tolist(), pr[bad[:5]].tolist())
    return status, stats


def test_edges_to_csr_matches_matrix_conversion(sp):
    rng = np.random.default_rng(900)
    for trial in range(10):
        n = int(rng.integers(1, 400))
        m = int(rng.integers(0, 5 * n + 1)) if trial else 0
        directed = bool(trial % 2)
        eu, ev, ew = random_edges(rng, n, m, 0, 50, bad=6 if m > 12 else 0)
        if m:
            k = min(3, m)
            ev[:k] = eu[:k]  # a few self-loops
        eud = dev(eu) if m else torch.empty(0, dtype=torch.int32, device="cuda")
        evd = dev(ev) if m else torch.empty(0, dtype=torch.int32, device="cuda")
        ewd = dev(ew) if m else torch.empty(0, dtype=torch.int32, device="cuda")
        rp, col, w, bad = sp.csr_from_edges(eud, evd, ewd, n, directed)
        rp, col, w = rp.cpu().numpy(), col.cpu().numpy(), w.cpu().numpy()
        Wr, bad_r = oracle.edges_to_dense(eu, ev, ew, n, directed)
        assert bad == bad_r, trial
        assert rp[0] == 0 and np.all(np.diff(rp) >= 0)
        W = np.full((n, n), INF, np.int32)
        np.fill_diagonal(W, 0)
        for u in range(n):
            seg = list(zip(col[rp[u]:rp[u + 1]].tolist(), w[rp[u]:rp[u + 1]].tolist()))
            assert seg == sorted(seg), (trial, u)
            for v, wt in seg:
                assert v != u and 0 <= v < n
                W[u, v] = min(W[u, v], wt)
        assert np.array_equal(W, Wr), trial


@pytest.mark.parametrize("n", [1, 2, 5, 100, 1000, 3001, 20000])
def test_csr_solve_matches_oracle(sp, n):
    rng = np.random.default_rng(910 + n)
    for directed in (False, True):
        eu, ev, ew = gen.sparse_edges(n, 3 * n, 1, 1000, 77 + n)
        if n > 2:
            ev[:3] = eu[:3]               # self-loops
            eu[3:6], ev[3:6] = eu[6:9], ev[6:9]  # repeated pairs
        g = Graph(sp, eu, ev, ew, n, directed)
        srcs = sorted({0, n - 1, int(rng.integers(0, n))})
        for src in srcs:
            for wg in (0, 1, 3):
                check(sp, g, src, g.dev_oracle_lists, wg, ("oracle lists", directed))
            check(sp, g, src, g.dev_converted, 0, ("converted", directed))


def test_csr_zero_weights_exact(sp):
    rng = np.random.default_rng(920)
    seen = {True: 0, False: 0}
    for trial in range(12):
        n = int(rng.integers(20, 3000))
        eu, ev, ew = random_edges(rng, n, 3 * n, 0 if trial % 2 else 1, 9, zero_prob=0.2 if trial % 2 else 0.0)
        g = Graph(sp, eu, ev, ew, n, bool(trial % 3 == 0))
        src = int(rng.integers(0, n))
        for lists in (g.dev_oracle_lists, g.dev_converted):
            status, _ = check(sp, g, src, lists, tag=("zero", trial))
            tz = tight_zero_edge(*g.host, g.ref(src)[0])
            assert bool(status & sp.SSSP_STATUS_ZERO_FALLBACK) == tz, (trial, status)
        seen[tz] += 1
    assert seen[True] > 0 and seen[False] > 0


def test_csr_sweep_counts(sp):
    """Stats: SETTLED counts the edge lists relaxed, at least one per reachable vertex."""
    rng = np.random.default_rng(922)
    n = 5000
    eu, ev, ew = random_edges(rng, n, 3 * n, 1, 1000)
    g = Graph(sp, eu, ev, ew, n, False)
    _, stats = check(sp, g, 0, g.dev_oracle_lists)
    reach = int((g.ref(0)[0] != INF).sum())
    assert stats[0] >= 1 and stats[1] >= reach


def test_csr_isolated_source(sp):
    n = 1000
    eu = np.array([1, 2, 3], np.int32)
    ev = np.array([2, 3, 4], np.int32)
    ew = np.array([5, 5, 5], np.int32)
    g = Graph(sp, eu, ev, ew, n, False)
    for src in (0, 2):
        check(sp, g, src, g.dev_oracle_lists, tag="isolated")


def test_csr_large_with_zero_ties(sp):
    """Above 65536 vertices with many tight zero-weight edges (weights in [0, 20], a
    tenth of them forced to 0), undirected and directed: dist and pred equal the
    oracle's Algorithm 1 over the same lists, and the zero-weight pass is reported."""
    for directed, seed in ((False, 921), (True, 924)):
        rng = np.random.default_rng(seed)
        n = 70000
        eu, ev, ew = random_edges(rng, n, 3 * n, 0, 20, zero_prob=0.1)
        rp, col, w = oracle.edges_to_csr(eu, ev, ew, n, directed)
        print("[csr] n=%d zero weights, directed=%s" % (n, directed), flush=True)
        d, p = sp.csr_solve(dev(rp), dev(col), dev(w), 0)
        status, _ = sp.sssp_last_status()
        d, p = d.cpu().numpy(), p.cpu().numpy()
        assert status & 3 == 0
        assert status & sp.SSSP_STATUS_ZERO_FALLBACK
        assert tight_zero_edge(rp, col, w, d)
        dr, pr, _ = oracle.dijkstra_csr(rp, col, w, 0)
        bad = np.nonzero((d != dr) | (p != pr))[0]
        assert bad.size == 0, (directed, bad[:5].tolist(), p[bad[:5]].tolist(), pr[bad[:5]].tolist())


def test_csr_zero_weight_levels(sp):
    """Large levels of equal distance held together by zero-weight edges (weights 0
    or 1, half of them 0), where the settle order inside a level decides pred."""
    for n, seed in ((3000, 925), (20000, 926)):
        rng = np.random.default_rng(seed)
        eu, ev, ew = random_edges(rng, n, 3 * n, 0, 1, zero_prob=0.5)
        g = Graph(sp, eu, ev, ew, n, bool(seed % 2))
        for src in (0, n // 2):
            check(sp, g, src, g.dev_oracle_lists, tag="levels %d" % n)


def test_csr_sparse_workload(sp):
    """The paper's sparse family (m = 3n): n = 10000 / 20000 / 40000 against the oracle;
    n = 10^6 against the certificate and the closed-form pred (weights >= 1, so the
    closed form is Algorithm 1's pred).  Repeated solves agree."""
    _, specs = gen.workload_sparse()
    g, per_cu, cus = sp.sssp_csr_grid(10 ** 6)
    assert g == min(1024, per_cu * cus) and sp.sssp_csr_grid(10 ** 6, workgroups=5000)[0] == g
    for s in specs:
        eu, ev, ew = gen.sparse_edges(s.n, s.m, s.lo, s.hi, s.seed)
        rp, col, w = oracle.edges_to_csr(eu, ev, ew, s.n, s.directed)
        rpd, cold, wd, bad = sp.csr_from_edges(dev(eu), dev(ev), dev(ew), s.n, s.directed)
        assert bad == 0
        ref = None
        for which, lists in (("oracle lists", (dev(rp), dev(col), dev(w))), ("converted", (rpd, cold, wd))):
            print("[csr] n=%d %s grid=%s" % (s.n, which, sp.sssp_csr_grid(s.n)), flush=True)
            d, p = sp.csr_solve(*lists, 0)
            status, _ = sp.sssp_last_status()
            assert status & 3 == 0
            d, p = d.cpu().numpy(), p.cpu().numpy()
            if ref is None:
                if s.n <= 40000:
                    dr, pr, _ = oracle.dijkstra_csr(rp, col, w, 0)
                else:
                    assert oracle.certificate_csr(rp, col, w, 0, d, p)[0] == 0
                    dr = d
                    pr = oracle.closed_form_pred_csr(rp, col, w, d)
                    pr[0] = -1
                ref = (dr, pr)
            assert np.array_equal(d, ref[0]) and np.array_equal(p, ref[1]), s.n
        for _ in range(2):
            d2, p2 = sp.csr_solve(rpd, cold, wd, 0)
            assert np.array_equal(d2.cpu().numpy(), ref[0]) and np.array_equal(p2.cpu().numpy(), ref[1])


def test_csr_plain_launch(sp, monkeypatch):
    """The ordinary (non-cooperative) launch that profilers need gives the same results."""
    rng = np.random.default_rng(923)
    n = 30000
    eu, ev, ew = random_edges(rng, n, 3 * n, 1, 500)
    g = Graph(sp, eu, ev, ew, n, False)
    monkeypatch.setenv("SSSP_GRID_LAUNCH", "plain")
    check(sp, g, 0, g.dev_oracle_lists, tag="plain")
    check(sp, g, 17, g.dev_converted, workgroups=7, tag="plain wg7")
    monkeypatch.delenv("SSSP_GRID_LAUNCH")
