"""GPU tests of batched plans (compact copies, autotuned workgroups per instance,
captured hipGraph) and of the one-shot batched call with gangs: every instance
must equal the oracle bit for bit."""
import numpy as np
import pytest

import gen
import oracle
from tests.graphs import INF, random_dense

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_03667_amd as m
    m.lib()
    return m


def make_items(rng, graphs, per_graph=3):
    dev = [torch.from_numpy(W).cuda() for W in graphs]
    items, refs = [], []
    for gi, W in enumerate(graphs):
        n = W.shape[0]
        for src in sorted({0, n - 1, int(rng.integers(0, n))})[:per_graph]:
            d = torch.full((n,), -7, dtype=torch.int32, device="cuda")
            p = torch.full((n,), -7, dtype=torch.int32, device="cuda")
            items.append((dev[gi], src, d, p))
            refs.append((gi, src))
    return dev, items, refs


def check_items(graphs, items, refs, cache):
    total = 0
    for (Wt, src, d, p), (gi, s) in zip(items, refs):
        if (gi, s) not in cache:
            cache[(gi, s)] = oracle.dijkstra(graphs[gi], s)
        dr, pr, rel = cache[(gi, s)]
        total += rel
        dd, pp = d.cpu().numpy(), p.cpu().numpy()
        assert np.array_equal(dd, dr) and np.array_equal(pp, pr), (gi, s, graphs[gi].shape[0])
    return total


def poison(items):
    for _, _, d, p in items:
        d.fill_(-7)
        p.fill_(-7)


def test_plans_all_configurations(sp):
    rng = np.random.default_rng(300)
    graphs = [random_dense(rng, n, pr, 1, hi, directed=bool(i % 2), zero_prob=0.03 if i == 3 else 0.0)
              for i, (n, pr, hi) in enumerate([(3000, 0.02, 100), (1500, 0.3, 100), (777, 0.01, 1000),
                                               (2500, 0.05, 200), (64, 0.5, 9), (4100, 0.01, 60000)])]
    dev, items, refs = make_items(rng, graphs)
    cache = {}
    configs = [dict(), dict(single_max_n=16384), dict(single_max_n=1024, gang_columns=512),
               dict(single_max_n=500, gang_columns=256)]
    for flags in (0, sp.SSSP_FLAG_COMPACT):
        for cfg in configs:
            poison(items)
            with sp.BatchPlan(items, flags, **cfg) as plan:
                plan.launch()
                status, stats = plan.status()
                info = plan.info()
                assert status & 3 == 0, (flags, cfg, status)
                total = check_items(graphs, items, refs, cache)
                print("plan", flags, cfg, "lc_instances", info["lc_instances"], "rows", stats[1], "settled", total,
                      flush=True)
                if info["lc_instances"] == 0:
                    assert stats[1] == total, (flags, cfg, stats, total)
                else:  # label-correcting items count rows streamed, every reachable row at least once
                    assert stats[1] >= total, (flags, cfg, stats, total)
                assert info["graph"] == 1
                if cfg:
                    assert info["single_max_n"] == cfg["single_max_n"]
                    # the host-side layout query describes the launch the plan runs
                    from paper_2504_03667_amd import sssp
                    arr, count = sssp.make_instances(items)
                    entries, _ = sp.sssp_batch_layout(list(arr[:count]), 0, cfg["single_max_n"],
                                                      cfg.get("gang_columns", 0), max(2, info["workgroups"] // 2))
                    assert max(e["parts"] for e in entries) == info["max_parts"]
                else:
                    assert info["candidates"] >= 2
                if cfg.get("single_max_n", 16384) < 4100:
                    assert info["max_parts"] > 1
                if flags:
                    # every matrix here has weights that fit 16 bits (one needs 16, the rest 8)
                    assert info["compact_graphs"] == len(graphs)


def test_plan_graph_replays_match_eager(sp):
    """Replays of the captured graph, with eager work and synchronisation between them,
    each reproduce the eager one-shot result."""
    rng = np.random.default_rng(301)
    graphs = [random_dense(rng, n, 0.03, 1, 100) for n in (2000, 1000, 3000)]
    dev, items, refs = make_items(rng, graphs)
    sp.sssp_dense_solve_batched(items)
    torch.cuda.synchronize()
    eager = [(d.cpu().numpy().copy(), p.cpu().numpy().copy()) for _, _, d, p in items]
    with sp.BatchPlan(items, sp.SSSP_FLAG_COMPACT, single_max_n=1024, gang_columns=512) as plan:
        for rep in range(4):
            poison(items)
            x = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
            sp.solve(dev[rep % 3], 1)
            torch.cuda.synchronize()
            plan.launch()
            status, _ = plan.status()
            assert status & 3 == 0 and float(x) == float(x)
            for (_, _, d, p), (de, pe) in zip(items, eager):
                assert np.array_equal(d.cpu().numpy(), de) and np.array_equal(p.cpu().numpy(), pe), rep


def test_one_shot_batched_with_gangs(sp):
    """An instance above the one-workgroup limit runs as a gang inside the batched launch."""
    rng = np.random.default_rng(302)
    big = random_dense(rng, 17000, 0.002, 1, 50)
    small = random_dense(rng, 900, 0.05, 1, 50)
    dev, items, refs = make_items(rng, [big, small], per_graph=2)
    assert big.shape[0] > sp.sssp_batch_max_n()
    sp.sssp_dense_solve_batched(items)
    status, stats = sp.sssp_last_status()
    assert status & 3 == 0
    assert stats[1] == check_items([big, small], items, refs, {})


def test_validate_and_compact_boundaries(sp):
    rng = np.random.default_rng(303)
    base = random_dense(rng, 300, 0.2, 1, 9)
    cases = [(254, 1), (255, 2), (65534, 2), (65535, 4), (-3, 4)]
    for wmax, elem in cases:
        W = base.copy()
        W[5, 7] = wmax
        if wmax < 0:
            W[9, 2] = 4
        Wt = torch.from_numpy(W).cuda()
        mn, mx = sp.sssp_dense_validate(Wt, 300, 300)
        fin = W[W != INF]
        assert mn == int(W.min()) and mx == int(fin.max())
        if wmax < 0:
            continue  # a negative weight violates the precondition; no parity claim
        d = torch.empty(300, dtype=torch.int32, device="cuda")
        p = torch.empty(300, dtype=torch.int32, device="cuda")
        with sp.BatchPlan([(Wt, 0, d, p)], sp.SSSP_FLAG_COMPACT, single_max_n=16384) as plan:
            plan.launch()
            plan.status()
            assert plan.info()["compact_graphs"] == (1 if elem < 4 else 0)
        dr, pr, _ = oracle.dijkstra(W, 0)
        assert np.array_equal(d.cpu().numpy(), dr) and np.array_equal(p.cpu().numpy(), pr)


def test_plans_label_correcting(sp):
    """Every instance through the label-correcting items (int32 and compact, with a
    zero-weight graph that forces the in-gang fallback), and the one-shot call."""
    rng = np.random.default_rng(305)
    graphs = [random_dense(rng, n, pr, 1, hi, directed=bool(i % 2), zero_prob=0.05 if i == 1 else 0.0)
              for i, (n, pr, hi) in enumerate([(700, 0.01, 1000), (1200, 0.05, 20), (2500, 0.003, 1000),
                                               (64, 0.3, 9), (300, 0.02, 60000)])]
    dev, items, refs = make_items(rng, graphs)
    cache = {}
    for flags in (sp.SSSP_FLAG_LABEL_CORRECTING, sp.SSSP_FLAG_LABEL_CORRECTING | sp.SSSP_FLAG_COMPACT):
        poison(items)
        with sp.BatchPlan(items, flags) as plan:
            plan.launch()
            status, stats = plan.status()
            assert status & 3 == 0, (flags, status)
            assert plan.info()["lc_instances"] == len(items)
            check_items(graphs, items, refs, cache)
    poison(items)
    sp.sssp_dense_solve_batched(items, sp.SSSP_FLAG_LABEL_CORRECTING)
    status, _ = sp.sssp_last_status()
    assert status & 3 == 0
    check_items(graphs, items, refs, cache)


def test_plan_chooses_label_correcting_for_many_levels(sp):
    """Sparse graphs with wide weights need hundreds of rounds: the plan measures them
    as candidates; whatever it keeps, the results are exact."""
    rng = np.random.default_rng(306)
    graphs = [gen.dense_host(gen.GraphSpec(n, p, 1, 1000, 900 + i))
              for i, (n, p) in enumerate([(3000, 0.002), (2000, 0.003), (800, 0.3)])]
    dev, items, refs = make_items(rng, graphs)
    for flags in (0, sp.SSSP_FLAG_COMPACT):
        poison(items)
        with sp.BatchPlan(items, flags) as plan:
            plan.launch()
            status, _ = plan.status()
            info = plan.info()
            assert status & 3 == 0
            sparse = sum(1 for gi, _ in refs if gi < 2)  # instances of the two sparse graphs
            assert info["lc_candidates"] == sparse
            assert info["lc_instances"] in (0, sparse)
            check_items(graphs, items, refs, {})


def test_compact_plan_large_offsets(sp):
    """A uint8 compact copy whose row offsets pass 2^31 bytes (n = 50000), solved by
    gangs of one column group per thread, against the oracle."""
    spec = gen.GraphSpec(50000, 0.002, 1, 200, 77001)
    W = gen.dense_device(spec)
    items = [(W, src, torch.full((spec.n,), -9, dtype=torch.int32, device="cuda"),
              torch.full((spec.n,), -9, dtype=torch.int32, device="cuda")) for src in (0, 49999)]
    with sp.BatchPlan(items, sp.SSSP_FLAG_COMPACT, single_max_n=4096, gang_columns=2048) as plan:
        plan.launch()
        status, _ = plan.status()
        assert status & 3 == 0
        assert plan.info()["compact_graphs"] == 1
    del W
    torch.cuda.empty_cache()
    Wh = gen.dense_host(spec)
    for _, src, d, p in items:
        dr, pr, _ = oracle.dijkstra(Wh, src)
        assert np.array_equal(d.cpu().numpy(), dr) and np.array_equal(p.cpu().numpy(), pr), src
