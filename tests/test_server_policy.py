"""Host policy of the server, on the CPU (sssp_server_shape: the split admission
gives a query, without a device): one workgroup up to single_max_n; gangs of
gang_columns (label-correcting: lc_gang_columns) per member, at least two
members, at most half the kernel's workgroups; the latency-mode split (narrower
slices when nothing waits, within three quarters of the workgroups minus those
busy); the throughput-mode split (wider slices under a backlog of busy_queue
queries, by the graph's entry size); arena bytes; argument errors."""
import pytest

DIJ, LC = 0, 1


@pytest.fixture(scope="module")
def sp():
    import paper_2504_03667_amd as m
    from paper_2504_03667_amd import sssp
    return m, sssp


def ceil_div(a, b):
    return -(-a // b)


def check_split(n, parts, cols):
    assert cols % 4 == 0 and parts * cols >= n and (parts - 1) * cols < n


def test_single_and_wide_gangs(sp):
    m, _ = sp
    # one workgroup up to single_max_n, also with a backlog
    assert m.sssp_server_shape(248, 4096, waiting=5)[:2] == (1, 4096)
    assert m.sssp_server_shape(248, 1, waiting=0)[:2] == (1, 1)
    for n in (4097, 10000, 30979, 65536):
        parts, cols, b = m.sssp_server_shape(248, n, waiting=3)  # a backlog: the wide split
        want = max(2, ceil_div(n, 2048))
        assert parts <= want and parts >= 2
        check_split(n, parts, cols)
        assert b > 0
    # at most half the workgroups
    parts, cols, _ = m.sssp_server_shape(20, 65536, waiting=1)
    assert parts == 10
    check_split(65536, parts, cols)


def test_latency_mode(sp):
    m, _ = sp
    n = 30979
    wide = m.sssp_server_shape(248, n, waiting=1)
    narrow = m.sssp_server_shape(248, n, waiting=0)
    assert wide[0] == ceil_div(n, 2048) and narrow[0] == ceil_div(n, 512)
    check_split(n, *narrow[:2])
    # busy workgroups shrink the budget (3/4 of 248 = 186): the split is as narrow as fits
    mid = m.sssp_server_shape(248, n, busy=150, waiting=0)
    assert wide[0] < mid[0] <= 186 - 150 and mid[0] < narrow[0]
    check_split(n, *mid[:2])
    # no room left: the wide split
    assert m.sssp_server_shape(248, n, busy=180, waiting=0)[:2] == wide[:2]
    # switched off
    assert m.sssp_server_shape(248, n, waiting=0, idle_gang_columns=-1)[:2] == wide[:2]
    # explicit width
    p, c, _ = m.sssp_server_shape(248, n, waiting=0, idle_gang_columns=1024)
    assert p == ceil_div(n, 1024)
    # single-workgroup queries are never split
    assert m.sssp_server_shape(248, 3000, waiting=0)[:2] == (1, 3000)


def test_throughput_mode(sp):
    m, sssp = sp
    n = 30979
    wide = m.sssp_server_shape(248, n, waiting=1)
    assert wide[0] == ceil_div(n, 2048)
    # a backlog of busy_queue (128) queries: twice the width for int32 graphs, four
    # times for compact copies; below it, the ordinary wide split
    assert m.sssp_server_shape(248, n, waiting=127)[:2] == wide[:2]
    p4, c4, b4 = m.sssp_server_shape(248, n, waiting=128)
    assert p4 == ceil_div(n, 4096) and b4 < wide[2]
    check_split(n, p4, c4)
    for elem in (1, 2):
        pc, cc, _ = m.sssp_server_shape(248, n, waiting=500, elem=elem)
        assert pc == ceil_div(n, 8192)
        check_split(n, pc, cc)
    # never fewer than two members, never wider than 16384 columns
    assert m.sssp_server_shape(248, 9000, waiting=1000, elem=1)[0] == 2
    assert m.sssp_server_shape(248, 65536, waiting=1000, elem=1)[:2] == (8, 8192)
    assert m.sssp_server_shape(248, 65536, waiting=1000, elem=1, gang_columns=8192)[:2] == (4, 16384)
    # set explicitly, or switched off; the threshold is configurable
    assert m.sssp_server_shape(248, n, waiting=500, busy_gang_columns=3072)[0] == ceil_div(n, 3072)
    assert m.sssp_server_shape(248, n, waiting=500, busy_gang_columns=-1)[:2] == wide[:2]
    assert m.sssp_server_shape(248, n, waiting=10, busy_queue=10)[0] == ceil_div(n, 4096)
    # label-correcting queries and single-workgroup queries keep their split
    assert m.sssp_server_shape(248, 7323, method=LC, waiting=500)[:2] == m.sssp_server_shape(248, 7323, method=LC,
                                                                                              waiting=1)[:2]
    assert m.sssp_server_shape(248, 3000, waiting=500)[:2] == (1, 3000)
    for kw in (dict(busy_gang_columns=6), dict(busy_gang_columns=16388), dict(elem=3)):
        with pytest.raises(sssp.SsspError) as x:
            m.sssp_server_shape(248, n, waiting=500, **kw)
        assert x.value.code == sssp.SSSP_EINVAL


def test_label_correcting_gangs(sp):
    m, _ = sp
    # label-correcting: a gang even below single_max_n (possibly of one), lc_gang_columns wide
    p, c, b = m.sssp_server_shape(248, 3000, method=LC, waiting=2)
    assert p == ceil_div(3000, 1024) and b > 0
    check_split(3000, p, c)
    p1, c1, _ = m.sssp_server_shape(248, 700, method=LC, waiting=2)
    assert (p1, c1) == (1, 700)
    # latency mode narrows it to idle_gang_columns (512 by default)
    pn, cn, _ = m.sssp_server_shape(248, 7323, method=LC, waiting=0)
    assert pn == ceil_div(7323, 512)
    check_split(7323, pn, cn)


def test_arena_and_errors(sp):
    m, sssp = sp
    _, _, b_wide = m.sssp_server_shape(248, 20000, waiting=1)
    _, _, b_narrow = m.sssp_server_shape(248, 20000, waiting=0)
    assert b_narrow > b_wide > 0 and b_wide % 256 == 0
    # a query that can never fit the arena is refused, as submit refuses it
    with pytest.raises(sssp.SsspError) as x:
        m.sssp_server_shape(248, 20000, waiting=1, scratch_bytes=1000)
    assert x.value.code == sssp.SSSP_ENOMEM
    # the latency split is skipped when its records would not fit
    p, _, b = m.sssp_server_shape(248, 20000, waiting=0, scratch_bytes=b_wide)
    assert p == ceil_div(20000, 2048) and b == b_wide
    for kw in (dict(workgroups=0, n=10), dict(workgroups=8, n=0), dict(workgroups=8, n=10, method=2),
               dict(workgroups=8, n=10, busy=-1), dict(workgroups=8, n=10, gang_columns=6)):
        with pytest.raises(sssp.SsspError) as x:
            m.sssp_server_shape(**kw)
        assert x.value.code == sssp.SSSP_EINVAL


def test_random_shapes_obey_the_contract(sp):
    """2000 random (workgroups, n, method, busy, waiting, configuration) cases: one
    workgroup up to single_max_n for the Dijkstra rounds; otherwise column slices of
    multiples of 4 that cover n exactly, at least two Dijkstra members and never more
    than half the workgroups (or two) in the wide split; the latency split at least as
    many members as the wide one, within three quarters of the workgroups minus those
    busy when it is narrower, and never more members than slices of
    idle_gang_columns need;
    arena bytes a multiple of 256 that hold two record slots and two lists."""
    import numpy as np
    m, sssp = sp
    rng = np.random.default_rng(1600)
    for trial in range(2000):
        W = int(rng.integers(1, 600))
        n = int(rng.integers(1, 70000))
        method = int(rng.integers(0, 2))
        busy = int(rng.integers(0, W + 1))
        single = int(rng.choice([256, 1024, 4096]))
        gang = int(rng.choice([256, 512, 2048]))
        lc_gang = int(rng.choice([256, 1024]))
        idle = int(rng.choice([-1, 256, 512]))
        cfg = dict(single_max_n=single, gang_columns=gang, lc_gang_columns=lc_gang, idle_gang_columns=idle)
        wide = m.sssp_server_shape(W, n, method=method, busy=busy, waiting=1, **cfg)
        lat = m.sssp_server_shape(W, n, method=method, busy=busy, waiting=0, **cfg)
        elem = int(rng.choice([1, 2, 4]))
        busy_cols = int(rng.choice([0, -1, 4096]))
        thr = m.sssp_server_shape(W, n, method=method, busy=busy, waiting=200, elem=elem, busy_gang_columns=busy_cols,
                                  **cfg)
        for parts, cols, b in (wide, lat, thr):
            assert parts >= 1 and b % 256 == 0, (trial, parts, cols, b)
            if parts == 1 and method == 0:
                assert cols == n
            else:  # a gang, also a label-correcting gang of one
                assert cols % 4 == 0 and parts * cols >= n > (parts - 1) * cols, (trial, parts, cols, n)
            if parts > 1 or method == 1:
                entry = 8 if method == 1 else 4
                assert b >= 2 * parts * 32 + 2 * parts * cols * entry, (trial, parts, cols, b)
        if method == 0 and n <= single:
            assert wide[:2] == (1, n) and lat[:2] == (1, n) and wide[2] == 0
            continue
        width = lc_gang if method == 1 else gang
        if method == 0:
            assert 2 <= wide[0] <= max(2, W // 2), (trial, W, n, wide)
            assert wide[0] <= max(2, -(-n // width))
        else:
            assert wide[0] <= max(1, -(-n // width)), (trial, W, n, wide)
        assert lat[0] >= wide[0], (trial, wide, lat)
        if lat[0] > wide[0]:
            assert lat[0] <= (3 * W) // 4 - busy, (trial, W, busy, wide, lat)
            assert idle > 0 and lat[0] <= -(-n // idle), (trial, idle, n, lat)
        if idle < 0:
            assert lat[:2] == wide[:2]
        # the throughput split: never more members than the wide one, at least two
        assert thr[0] <= wide[0], (trial, wide, thr)
        if method == 0:
            assert thr[0] >= 2
        if method == 1 or busy_cols < 0:
            assert thr[:2] == wide[:2]
