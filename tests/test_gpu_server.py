"""GPU tests of the serving path (persistent kernel + host admission): every served
query must equal the oracle and its own solve alone, whatever else runs beside it."""
import numpy as np
import pytest

import gen
import oracle
from tests.graphs import random_dense

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_03667_amd as m
    m.lib()
    return m


def make_graphs(rng, sizes):
    out = []
    for i, n in enumerate(sizes):
        W = random_dense(rng, n, float(rng.choice([0.003, 0.02, 0.2])), 1, 1000, directed=bool(i % 3 == 0),
                         zero_prob=0.02 if i == 2 else 0.0)
        out.append(W)
    return out


def outputs(n):
    d = torch.full((n,), -9, dtype=torch.int32, device="cuda")
    p = torch.full((n,), -9, dtype=torch.int32, device="cuda")
    # the fill must land before the server writes results; synchronise the stream,
    # not the device (a device-wide sync would also wait for the serving kernel)
    torch.cuda.current_stream().synchronize()
    return d, p


def test_server_matches_oracle_with_gangs(sp):
    """Small single_max_n / gang_columns force multi-workgroup gangs on modest n."""
    rng = np.random.default_rng(200)
    graphs = make_graphs(rng, [5, 300, 700, 1500, 2100, 3333])
    dev = [torch.from_numpy(W).cuda() for W in graphs]
    plan = []
    for k in range(60):
        g = int(rng.integers(0, len(graphs)))
        plan.append((g, int(rng.integers(0, graphs[g].shape[0])), *outputs(graphs[g].shape[0])))
    with sp.Server(single_max_n=512, gang_columns=256) as srv:
        gids = [srv.add_graph(W) for W in dev]
        jobs = [(g, src, d, p, srv.submit(gids[g], src, d, p)) for g, src, d, p in plan]
        for g, src, d, p, t in jobs:
            srv.wait(t, timeout_s=60)
            info = srv.info(t)
            dr, pr, rel = oracle.dijkstra(graphs[g], src)
            assert info["state"] == sp.SSSP_QUERY_DONE and info["status"] & 3 == 0
            assert info["settled"] == rel
            n = graphs[g].shape[0]
            assert info["parts"] == (1 if n <= 512 else info["parts"]) and (n <= 512 or info["parts"] > 1)
            assert np.array_equal(d.cpu().numpy(), dr) and np.array_equal(p.cpu().numpy(), pr), (g, src)
        st = srv.stats()
        assert st["completed"] == 60 and st["running"] == 0 and st["pending"] == 0
        assert sorted(srv.poll()) == [j[4] for j in jobs]


def test_server_alone_equals_mix(sp):
    """Each query's result alone (submitted and awaited one at a time) equals its result in
    a burst where it overlaps with all the others, and equals sssp_dense_solve."""
    rng = np.random.default_rng(201)
    graphs = make_graphs(rng, [900, 2500, 5000, 6000])
    dev = [torch.from_numpy(W).cuda() for W in graphs]
    qs = [(int(g), int(rng.integers(0, graphs[g].shape[0]))) for g in rng.integers(0, 4, size=40)]
    outs_alone = [outputs(graphs[g].shape[0]) for g, _ in qs]
    outs_mix = [outputs(graphs[g].shape[0]) for g, _ in qs]
    with sp.Server(single_max_n=4096, gang_columns=1024) as srv:
        gids = [srv.add_graph(W) for W in dev]
        alone = []
        for (g, src), (d, p) in zip(qs, outs_alone):
            srv.wait(srv.submit(gids[g], src, d, p), timeout_s=60)
            alone.append((d.cpu().numpy(), p.cpu().numpy()))
        mix = []
        for (g, src), (d, p) in zip(qs, outs_mix):
            mix.append((srv.submit(gids[g], src, d, p), d, p))
        for (t, d, p), (da, pa) in zip(mix, alone):
            srv.wait(t, timeout_s=60)
            assert np.array_equal(d.cpu().numpy(), da) and np.array_equal(p.cpu().numpy(), pa)
    for (g, src), (da, pa) in zip(qs, alone):
        d, p = sp.solve(dev[g], src)
        assert np.array_equal(d.cpu().numpy(), da) and np.array_equal(p.cpu().numpy(), pa)


def test_server_memory_admission(sp):
    """An arena that holds one gang's exchange records at a time: queries wait for memory
    instead of failing, and every one completes correctly."""
    rng = np.random.default_rng(202)
    graphs = make_graphs(rng, [3000, 3100])
    dev = [torch.from_numpy(W).cuda() for W in graphs]
    # footprint of a 3100-vertex gang with 256 columns per member: 13 members
    big = torch.from_numpy(random_dense(rng, 8000, 0.01, 1, 9)).cuda()
    bd, bp = outputs(8000)
    plan = [(k % 2, int(rng.integers(0, graphs[k % 2].shape[0])), *outputs(graphs[k % 2].shape[0]))
            for k in range(12)]
    with sp.Server(single_max_n=256, gang_columns=256, scratch_bytes=60000) as srv:
        gids = [srv.add_graph(W) for W in dev]
        jobs = [(g, src, d, p, srv.submit(gids[g], src, d, p)) for g, src, d, p in plan]
        saw_wait = srv.stats()["pending"] > 0
        for g, src, d, p, t in jobs:
            srv.wait(t, timeout_s=60)
            dr, pr, _ = oracle.dijkstra(graphs[g], src)
            assert np.array_equal(d.cpu().numpy(), dr) and np.array_equal(p.cpu().numpy(), pr)
        assert saw_wait
        gb = srv.add_graph(big)
        with pytest.raises(sp.SsspError) as e:
            srv.submit(gb, 0, bd, bp)  # its gang records alone exceed the arena
        assert e.value.code == -3  # SSSP_ENOMEM


def test_server_errors_and_backpressure(sp):
    rng = np.random.default_rng(203)
    W = torch.from_numpy(random_dense(rng, 2000, 0.5, 1, 9)).cuda()
    d, p = outputs(2000)
    outs = [outputs(2000) for _ in range(30)]
    with sp.Server(max_pending=1, max_inflight=1) as srv:
        gid = srv.add_graph(W)
        with pytest.raises(sp.SsspError) as e:
            srv.submit(gid + 5, 0, d, p)
        assert e.value.code == -5  # SSSP_ENOGRAPH
        with pytest.raises(sp.SsspError) as e:
            srv.submit(gid, 2000, d, p)
        assert e.value.code == -1
        tickets, again = [], 0
        for d, p in outs:
            try:
                tickets.append(srv.submit(gid, 0, d, p))
            except sp.SsspError as ex:
                assert ex.code == -4  # SSSP_EAGAIN
                again += 1
        assert again > 0 and tickets
        for t in tickets:
            srv.wait(t, timeout_s=60)
    dr, pr, _ = oracle.dijkstra(W.cpu().numpy(), 0)
    assert np.array_equal(outs[0][0].cpu().numpy(), dr)


def test_server_compact_graphs(sp):
    """Graphs registered with SSSP_FLAG_COMPACT are streamed from exact 8/16-bit copies and
    give the same results as the int32 matrices."""
    rng = np.random.default_rng(204)
    graphs = [random_dense(rng, 1200, 0.05, 1, 100), random_dense(rng, 5000, 0.01, 1, 1000),
              random_dense(rng, 900, 0.1, 1, 70000)]
    dev = [torch.from_numpy(W).cuda() for W in graphs]
    plan = [(g, int(rng.integers(0, graphs[g].shape[0])), *outputs(graphs[g].shape[0]))
            for g in (0, 1, 2, 1, 0, 2, 1)]
    with sp.Server() as srv:
        gids = [srv.add_graph(W, sp.SSSP_FLAG_COMPACT) for W in dev]
        assert [srv.graph_elem(g) for g in gids] == [1, 2, 4]
        jobs = [(g, src, d, p, srv.submit(gids[g], src, d, p)) for g, src, d, p in plan]
        for g, src, d, p, t in jobs:
            srv.wait(t, timeout_s=60)
            dr, pr, _ = oracle.dijkstra(graphs[g], src)
            assert np.array_equal(d.cpu().numpy(), dr) and np.array_equal(p.cpu().numpy(), pr)


def test_server_label_correcting(sp):
    """Graphs added with SSSP_FLAG_LABEL_CORRECTING, and a server that switches a graph
    to label-correcting after its first query (lc_rounds=1): every query exact."""
    rng = np.random.default_rng(207)
    graphs = make_graphs(rng, [40, 900, 1700, 2600])
    dev = [torch.from_numpy(W).cuda() for W in graphs]
    cases = []
    for k in range(40):
        g = int(rng.integers(0, len(graphs)))
        cases.append((g, int(rng.integers(0, graphs[g].shape[0])), *outputs(graphs[g].shape[0])))
    for forced, cfg in ((True, {}), (False, dict(lc_rounds=1, lc_gang_columns=128, lc_model=-1))):
        with sp.Server(**cfg) as srv:
            flags = sp.SSSP_FLAG_LABEL_CORRECTING if forced else 0
            gids = [srv.add_graph(W, flags | (sp.SSSP_FLAG_COMPACT if i % 2 else 0)) for i, W in enumerate(dev)]
            if not forced:
                # one query per graph first: afterwards every graph has taken >= 1 round
                first = [srv.submit(gids[g], 0, *outputs(graphs[g].shape[0])) for g in range(len(graphs))]
                for t in first:
                    srv.wait(t, timeout_s=60)
                    assert srv.info(t)["method"] == 0
            jobs = [(g, src, d, p, srv.submit(gids[g], src, d, p)) for g, src, d, p in cases]
            for g, src, d, p, t in jobs:
                srv.wait(t, timeout_s=60)
                info = srv.info(t)
                assert info["status"] & 3 == 0 and info["method"] == 1, (forced, info)
                dr, pr, _ = oracle.dijkstra(graphs[g], src)
                assert np.array_equal(d.cpu().numpy(), dr) and np.array_equal(p.cpu().numpy(), pr), (forced, g, src)


def test_server_latency_mode_gangs(sp):
    """A gang query admitted while nothing waits behind it is split into narrower
    slices (idle_gang_columns); a burst keeps the wide default.  Results are the
    oracle's either way."""
    rng = np.random.default_rng(205)
    graphs = make_graphs(rng, [3000, 5000])
    dev = [torch.from_numpy(W).cuda() for W in graphs]
    with sp.Server(single_max_n=1024, gang_columns=2048, idle_gang_columns=256) as srv:
        gids = [srv.add_graph(W) for W in dev]
        # one at a time: narrow slices
        for g in (0, 1):
            n = graphs[g].shape[0]
            d, p = outputs(n)
            t = srv.submit(gids[g], 1, d, p)
            srv.wait(t, timeout_s=60)
            info = srv.info(t)
            dr, pr, _ = oracle.dijkstra(graphs[g], 1)
            assert info["parts"] == -(-n // 256), info
            assert np.array_equal(d.cpu().numpy(), dr) and np.array_equal(p.cpu().numpy(), pr)
        # a burst: queries behind the first keep the wide split
        outs = [outputs(graphs[k % 2].shape[0]) for k in range(40)]
        ts = [srv.submit(gids[k % 2], 7 + k, *outs[k]) for k in range(40)]
        parts = []
        for k, t in enumerate(ts):
            srv.wait(t, timeout_s=60)
            info = srv.info(t)
            parts.append(info["parts"])
            dr, pr, _ = oracle.dijkstra(graphs[k % 2], 7 + k)
            assert np.array_equal(outs[k][0].cpu().numpy(), dr) and np.array_equal(outs[k][1].cpu().numpy(), pr)
        assert parts.count(2) + parts.count(3) >= 10, parts  # wide: ceil(n / 2048) members
    with sp.Server(single_max_n=1024, gang_columns=2048, idle_gang_columns=-1) as srv:
        gid = srv.add_graph(dev[1])
        d, p = outputs(5000)
        t = srv.submit(gid, 3, d, p)
        srv.wait(t, timeout_s=60)
        assert srv.info(t)["parts"] == 3


def test_server_throughput_mode_gangs(sp):
    """A gang query admitted with at least busy_queue queries waiting behind it is
    split into wider slices (busy_gang_columns; by default twice gang_columns for
    int32 graphs and four times for compact copies); the queries near the end of
    the burst keep the ordinary split.  Results are the oracle's either way."""
    rng = np.random.default_rng(206)
    graphs = make_graphs(rng, [5000, 9000])
    dev = [torch.from_numpy(W).cuda() for W in graphs]
    refs = {}
    for flags in (0, sp.SSSP_FLAG_COMPACT):
        # four queries in flight at most, so that the burst waits for admission
        with sp.Server(single_max_n=1024, gang_columns=1024, idle_gang_columns=-1, busy_queue=8, max_inflight=4,
                       lc_rounds=-1) as srv:
            gids = [srv.add_graph(W, flags) for W in dev]
            outs = [outputs(graphs[k % 2].shape[0]) for k in range(48)]
            ts = [srv.submit(gids[k % 2], 3 + k, *outs[k]) for k in range(48)]
            parts = {0: set(), 1: set()}
            for k, t in enumerate(ts):
                srv.wait(t, timeout_s=60)
                parts[k % 2].add(srv.info(t)["parts"])
                if (k, 3 + k) not in refs:
                    refs[(k, 3 + k)] = oracle.dijkstra(graphs[k % 2], 3 + k)
                dr, pr, _ = refs[(k, 3 + k)]
                assert np.array_equal(outs[k][0].cpu().numpy(), dr) and np.array_equal(outs[k][1].cpu().numpy(), pr)
            elem = srv.graph_elem(gids[1])
            wide_cols = 1024 * (4 if elem < 4 else 2)
            # n = 9000: 9 members in the ordinary split, ceil(9000 / wide_cols) under the backlog
            assert -(-9000 // wide_cols) in parts[1] and 9 in parts[1], (flags, elem, parts)
            assert -(-5000 // wide_cols) in parts[0] or 2 in parts[0], (flags, parts)
