"""Barrier stress: the same sources built with pseudo-random pauses (0 to ~25 us) of
some workgroups before every exchange, barrier arrival and launch exit
(libsssp_stress.so), so that members arrive in many orders and late.  Every
persistent grid (whole-GPU rounds, label-correcting sweeps, batched gangs, serving
gangs, the adjacency-list solve) must still give the oracle's dist and pred bit for
bit, with no barrier time-out, and repeated solves must agree."""
import os

import numpy as np
import pytest

import gen
import oracle
from tests.graphs import random_dense

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

LITERAL, SINGLE, GRID, LC = 1, 2, 4, 16


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_03667_amd as m
    from paper_2504_03667_amd import build, sssp
    if not os.path.exists(build.SO_STRESS):
        pytest.fail("libsssp_stress.so is not built (run the package build first)")
    prev = sssp.use_library(build.SO_STRESS)
    yield m
    sssp._lib = prev


def check_dense(sp, W, src, flags=0, workgroups=0, Wt=None, tag="", balance=0):
    if Wt is None:
        Wt = torch.from_numpy(np.ascontiguousarray(W)).cuda()
    d, p = sp.solve(Wt, src, flags=flags, workgroups=workgroups, balance=balance)
    status, stats = sp.sssp_last_status()
    dr, pr, _ = oracle.dijkstra(W, src)
    assert status & 3 == 0, (tag, status)
    assert np.array_equal(d.cpu().numpy(), dr) and np.array_equal(p.cpu().numpy(), pr), tag
    return stats


def test_stress_library_is_loaded_and_pauses(sp):
    """The calls go to the stress build, and its pauses are live: a literal whole-GPU
    solve (one exchange per vertex) takes clearly longer than with libsssp.so."""
    import time
    from paper_2504_03667_amd import build, sssp
    assert sssp.lib()._name == build.SO_STRESS
    rng = np.random.default_rng(1299)
    W = torch.from_numpy(random_dense(rng, 400, 0.05, 1, 50)).cuda()

    def best_ms():
        ts = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sp.solve(W, 0, flags=GRID | LITERAL, workgroups=16)
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return min(ts)

    stressed = best_ms()
    stress_lib = sssp.use_library(build.SO)
    try:
        plain = best_ms()
    finally:
        sssp._lib = stress_lib
    assert stressed > 1.3 * plain, (stressed, plain)


def test_whole_gpu_rounds(sp):
    rng = np.random.default_rng(1300)
    for trial, (n, p, hi) in enumerate([(3001, 0.02, 100), (2048, 0.002, 1000), (4097, 0.2, 10)]):
        W = random_dense(rng, n, p, 1, hi, directed=bool(trial % 2))
        Wt = torch.from_numpy(W).cuda()
        for wg in (0, 3, 17, 64):
            check_dense(sp, W, int(rng.integers(0, n)), GRID, wg, Wt, ("grid", n, wg))


def test_whole_gpu_balanced_rounds(sp):
    """Rounds of ~8700 vertices (9 chunks): pair members claim each other's chunks,
    and the pauses before claiming make partners steal."""
    rng = np.random.default_rng(1303)
    W = random_dense(rng, 9000, 0.97, 1, 1)
    Wt = torch.from_numpy(W).cuda()
    for wg in (0, 64, 17):
        check_dense(sp, W, int(rng.integers(0, 9000)), GRID, wg, Wt, ("balanced", wg), balance=1)
    Z = random_dense(rng, 9000, 0.95, 0, 1, zero_prob=0.2)
    check_dense(sp, Z, 3, GRID, 0, tag="balanced-zero", balance=1)


def test_whole_gpu_literal_and_zero_fallback(sp):
    rng = np.random.default_rng(1301)
    W = random_dense(rng, 400, 0.05, 1, 50)
    check_dense(sp, W, 3, GRID | LITERAL, 9, tag="literal")
    Z = random_dense(rng, 1500, 0.02, 0, 20, zero_prob=0.1)
    stats = check_dense(sp, Z, 0, GRID, 24, tag="zero")
    assert stats[2] > 0  # fallbacks happened under the pauses too


def test_label_correcting(sp):
    rng = np.random.default_rng(1302)
    for n, p in ((2500, 0.01), (5000, 0.002)):
        W = random_dense(rng, n, p, 1, 1000)
        Wt = torch.from_numpy(W).cuda()
        for wg in (0, 7, 40):
            check_dense(sp, W, 1, LC, wg, Wt, ("lc", n, wg))
    Z = random_dense(rng, 1200, 0.03, 0, 9, zero_prob=0.1)
    check_dense(sp, Z, 2, LC, 12, tag="lc zero")


def test_batched_gangs(sp):
    """Instances above single_max_n run as gangs inside the batched launch."""
    rng = np.random.default_rng(1303)
    graphs = [random_dense(rng, n, 0.02, 1, 100, directed=bool(i % 2)) for i, n in enumerate((700, 1900, 3000, 260))]
    dev = [torch.from_numpy(W).cuda() for W in graphs]
    items, want = [], []
    for g, W in enumerate(graphs):
        for src in rng.integers(0, W.shape[0], size=4):
            n = W.shape[0]
            d = torch.full((n,), -9, dtype=torch.int32, device="cuda")
            p = torch.full((n,), -9, dtype=torch.int32, device="cuda")
            items.append((dev[g], int(src), d, p))
            want.append(oracle.dijkstra(W, int(src))[:2])
    with sp.BatchPlan(items, single_max_n=512, gang_columns=256) as plan:
        for rep in range(3):
            plan.launch()
            status, _ = plan.status()
            assert status & 3 == 0
            for (W, src, d, p), (dr, pr) in zip(items, want):
                assert np.array_equal(d.cpu().numpy(), dr) and np.array_equal(p.cpu().numpy(), pr), (rep, src)


def test_served_gangs(sp):
    rng = np.random.default_rng(1304)
    graphs = [random_dense(rng, n, 0.02, 1, 1000, directed=bool(i % 2)) for i, n in enumerate((300, 1500, 2600))]
    dev = [torch.from_numpy(W).cuda() for W in graphs]
    with sp.Server(single_max_n=512, gang_columns=256) as srv:
        gids = [srv.add_graph(W) for W in dev]
        jobs = []
        for k in range(30):
            g = int(rng.integers(0, len(graphs)))
            n = graphs[g].shape[0]
            src = int(rng.integers(0, n))
            d = torch.full((n,), -9, dtype=torch.int32, device="cuda")
            p = torch.full((n,), -9, dtype=torch.int32, device="cuda")
            torch.cuda.current_stream().synchronize()
            jobs.append((g, src, d, p, srv.submit(gids[g], src, d, p)))
        for g, src, d, p, t in jobs:
            srv.wait(t, timeout_s=60)
            info = srv.info(t)
            dr, pr, _ = oracle.dijkstra(graphs[g], src)
            assert info["state"] == sp.SSSP_QUERY_DONE and info["status"] & 3 == 0
            assert np.array_equal(d.cpu().numpy(), dr) and np.array_equal(p.cpu().numpy(), pr), (g, src)


def test_adjacency_lists(sp):
    rng = np.random.default_rng(1305)
    for n, lo in ((20000, 1), (3000, 0)):
        eu = rng.integers(0, n, size=3 * n).astype(np.int32)
        ev = rng.integers(0, n, size=3 * n).astype(np.int32)
        ew = rng.integers(lo, 1000 if lo else 9, size=3 * n).astype(np.int32)
        rp, col, w = oracle.edges_to_csr(eu, ev, ew, n)
        dr, pr, _ = oracle.dijkstra_csr(rp, col, w, 0)
        lists = tuple(torch.from_numpy(a).cuda() for a in (rp, col, w))
        for wg in (0, 5, 33):
            d, p = sp.csr_solve(*lists, 0, workgroups=wg)
            status, _ = sp.sssp_last_status()
            assert status & 3 == 0
            assert np.array_equal(d.cpu().numpy(), dr) and np.array_equal(p.cpu().numpy(), pr), (n, wg)


def test_repeated_solves_agree(sp):
    """50 whole-GPU solves of one graph under different pause patterns (each launch
    numbers its exchanges differently) are bit-identical."""
    spec = gen.GraphSpec(6000, 0.01, 1, 20, 56)
    Wt = gen.dense_device(spec)
    ref = None
    for rep in range(50):
        d, p = sp.solve(Wt, 5, flags=GRID, workgroups=40)
        status, _ = sp.sssp_last_status()
        assert status & 3 == 0
        cur = (d.cpu().numpy(), p.cpu().numpy())
        if ref is None:
            ref = cur
            dr, pr, _ = oracle.dijkstra(gen.dense_host(spec), 5)
            assert np.array_equal(cur[0], dr) and np.array_equal(cur[1], pr)
        assert np.array_equal(cur[0], ref[0]) and np.array_equal(cur[1], ref[1]), rep
