"""GPU tests of lockstep groups in batched plans: sources of one shared matrix
solved together by a gang, each row read once per round for every source whose
bucket holds it.  Every source's dist and pred must equal the oracle's
(Algorithm 1, Section III-A) for every group size and slice width, int32 and
compact matrices, ragged n, duplicate and isolated sources, and groups mixed
with ordinary instances in one launch."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from tests.graphs import random_dense

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CORES = max(1, min(16, len(os.sched_getaffinity(0))))


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_03667_amd as m
    m.lib()
    return m


def shared_items(Wt, sources):
    n = Wt.shape[0]
    return [(Wt, s, torch.full((n,), -7, dtype=torch.int32, device="cuda"),
             torch.full((n,), -7, dtype=torch.int32, device="cuda")) for s in sources]


def oracle_all(W, sources):
    with ThreadPoolExecutor(CORES) as ex:
        return list(ex.map(lambda s: oracle.dijkstra(W, s), sources))


def check(tag, items, refs):
    for k, ((_, s, d, p), (dr, pr, _)) in enumerate(zip(items, refs)):
        dd, pp = d.cpu().numpy(), p.cpu().numpy()
        bad = np.nonzero((dd != dr) | (pp != pr))[0]
        assert bad.size == 0, (tag, k, s, bad[:5].tolist(), dd[bad[:5]].tolist(), dr[bad[:5]].tolist(),
                               pp[bad[:5]].tolist(), pr[bad[:5]].tolist())


def poison(items):
    for _, _, d, p in items:
        d.fill_(-7)
        p.fill_(-7)


CONFIGS = [(2, 1024), (3, 4096), (4, 2048), (5, 1024), (8, 1024), (8, 512), (16, 512), (16, 1024)]


@pytest.mark.parametrize("n,p,hi,directed", [(500, 0.1, 9, False), (1001, 0.05, 100, True),
                                             (3001, 0.02, 100, False), (8192, 0.05, 100, False)])
def test_group_sizes_and_widths(sp, n, p, hi, directed):
    rng = np.random.default_rng(n)
    W = random_dense(rng, n, p, 1, hi, directed=directed)
    W[:, n - 1] = 0x7FFFFFFF  # vertex n-1 has no in-edges: unreachable from every other source
    W[n - 1, n - 1] = 0
    sources = [int(x) for x in rng.integers(0, n, size=45)] + [0, 0, n - 1]
    refs = oracle_all(W, sources)
    Wt = torch.from_numpy(W).cuda()
    items = shared_items(Wt, sources)
    for flags in (0, sp.SSSP_FLAG_COMPACT):
        for K, cols in CONFIGS:
            poison(items)
            with sp.BatchPlan(items, flags, group_sources=K, group_columns=cols) as plan:
                plan.launch()
                status, stats = plan.status()
                info = plan.info()
                assert status & 3 == 0, (K, cols, status)
                assert info["group_items"] > 0 and info["group_sources"] == K, info
                assert stats[1] == sum(r for _, _, r in refs), (K, cols, stats)
                check((flags, K, cols), items, refs)


def test_groups_need_positive_weights(sp):
    """A shared matrix with a zero off-diagonal weight is never grouped; the plan
    stays exact."""
    rng = np.random.default_rng(77)
    n = 1200
    W = random_dense(rng, n, 0.05, 1, 20, zero_prob=0.01)
    sources = [int(x) for x in rng.integers(0, n, size=40)]
    refs = oracle_all(W, sources)
    items = shared_items(torch.from_numpy(W).cuda(), sources)
    with sp.BatchPlan(items, 0, group_sources=8, group_columns=1024) as plan:
        plan.launch()
        status, _ = plan.status()
        assert status & 3 == 0
        assert plan.info()["group_items"] == 0 and plan.info()["group_candidates"] == 0
        check("zero", items, refs)


def test_groups_beside_other_instances(sp):
    """Two shared matrices (one of them too large for a single workgroup's slice)
    and unshared graphs in one autotuned launch, and the same with groups forced;
    replays of the captured graph agree."""
    rng = np.random.default_rng(78)
    mats, items, refs = [], [], []
    for n, cnt in ((2000, 40), (6000, 33)):
        W = random_dense(rng, n, 0.03, 1, 100, directed=n == 6000)
        Wt = torch.from_numpy(W).cuda()
        srcs = [int(x) for x in rng.integers(0, n, size=cnt)]
        mats.append(Wt)
        items += shared_items(Wt, srcs)
        refs += oracle_all(W, srcs)
    for n in (700, 3000, 17000):
        W = random_dense(rng, n, 0.01, 1, 1000)
        Wt = torch.from_numpy(W).cuda()
        mats.append(Wt)
        items += shared_items(Wt, [1])
        refs += oracle_all(W, [1])
    for tuning in (dict(), dict(group_sources=8, group_columns=1024), dict(group_sources=1)):
        poison(items)
        with sp.BatchPlan(items, sp.SSSP_FLAG_COMPACT, **tuning) as plan:
            for rep in range(2):
                poison(items)
                plan.launch()
                status, _ = plan.status()
                assert status & 3 == 0, (tuning, status)
                check((tuning, rep), items, refs)
            info = plan.info()
            assert info["group_candidates"] == 73
            if tuning.get("group_sources") == 8:
                assert info["group_items"] == 5 + 5
            if tuning.get("group_sources") == 1:
                assert info["group_items"] == 0
