"""GPU tests of the serving path's failure and lifecycle handling, every condition
forced from the host so that each kernel exits normally: the kernel parks when
idle and is relaunched by the next query; destroy with queries still queued
drains them all; a stalled host heartbeat (a server thread that beats less
often than the kernel's watchdog allows) makes the kernel leave, and the server
notices and relaunches it.  Every result is checked against the oracle."""
import time

import numpy as np
import pytest

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


def outputs(n):
    d = torch.full((n,), -9, dtype=torch.int32, device="cuda")
    p = torch.full((n,), -9, dtype=torch.int32, device="cuda")
    torch.cuda.current_stream().synchronize()
    return d, p


def check(W, src, d, p, tag):
    dr, pr, _ = oracle.dijkstra(W, src)
    assert np.array_equal(d.cpu().numpy(), dr) and np.array_equal(p.cpu().numpy(), pr), tag


def test_park_and_relaunch(sp):
    rng = np.random.default_rng(400)
    W = random_dense(rng, 2500, 0.02, 1, 100)
    Wt = torch.from_numpy(W).cuda()
    with sp.Server(idle_park_ms=5, single_max_n=1024, gang_columns=512) as srv:
        gid = srv.add_graph(Wt)
        base = None
        for k in range(4):
            d, p = outputs(2500)
            t = srv.submit(gid, 11 * k, d, p)
            srv.wait(t, timeout_s=60)
            check(W, 11 * k, d, p, ("park", k))
            assert srv.info(t)["parts"] > 1  # a gang, admitted into a relaunched kernel
            st = srv.stats()
            assert st["running"] == 0, st
            if base is not None:
                # the kernel had parked during the pause: exactly one relaunch per query
                assert st["kernel_launches"] == base + k, (k, base, st)
            time.sleep(0.1)  # 20x the idle time after which the kernel parks
            if base is None:
                base = srv.stats()["kernel_launches"]


def test_destroy_drains_queued_queries(sp):
    rng = np.random.default_rng(401)
    graphs = [random_dense(rng, n, 0.03, 1, 1000, directed=bool(i % 2)) for i, n in enumerate((900, 3000))]
    dev = [torch.from_numpy(W).cuda() for W in graphs]
    jobs = []
    srv = sp.Server(max_inflight=2, single_max_n=1024, gang_columns=1024)
    gids = [srv.add_graph(W) for W in dev]
    for k in range(60):
        g = k % 2
        src = int(rng.integers(0, graphs[g].shape[0]))
        d, p = outputs(graphs[g].shape[0])
        jobs.append((g, src, d, p, srv.submit(gids[g], src, d, p)))
    st = srv.stats()
    assert st["pending"] > 0, st  # most are still queued when destroy begins
    srv.close()  # returns once every admitted and queued query has completed
    for g, src, d, p, _ in jobs:
        check(graphs[g], src, d, p, ("drained", g, src))


def test_watchdog_exit_and_relaunch(sp):
    """The server thread beats the heartbeat every 20 ms while idle, the kernel's
    watchdog allows 1 ms: the kernel leaves in every idle gap, and each query
    submitted afterwards must find it relaunched."""
    rng = np.random.default_rng(402)
    graphs = [random_dense(rng, n, 0.05, 1, 50) for n in (700, 3000)]
    dev = [torch.from_numpy(W).cuda() for W in graphs]
    with sp.Server(watchdog_ms=1, idle_wait_us=20000, idle_park_ms=600000, single_max_n=4096) as srv:
        gids = [srv.add_graph(W) for W in dev]
        for k in range(4):
            g = k % 2
            d, p = outputs(graphs[g].shape[0])
            t = srv.submit(gids[g], 3 + k, d, p)
            srv.wait(t, timeout_s=60)
            info = srv.info(t)
            assert info["status"] & 3 == 0 and info["parts"] == 1, info
            check(graphs[g], 3 + k, d, p, ("watchdog", k))
            time.sleep(0.06)
        st = srv.stats()
        assert st["kernel_launches"] >= 4 and st["failed"] == 0, st
