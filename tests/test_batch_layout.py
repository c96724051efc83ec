"""Host logic of batched launches, on the CPU: sssp_batch_layout (the order and gang
shapes the batched calls use) obeys its contract for random instance sets — every
instance exactly once, largest first with the instances of shared matrices last,
one workgroup or a gang whose column slices cover n exactly, label-correcting gangs
of at most 256 columns, exchange arenas that tile without overlap — and rejects bad
arguments.  The buffers are never read (fake addresses)."""
import ctypes

import numpy as np
import pytest

FAKE = 1 << 24  # never dereferenced
SHARED = 32     # instances of one matrix from which it counts as shared
LC = 16


@pytest.fixture(scope="module")
def sp():
    import paper_2504_03667_amd as m
    from paper_2504_03667_amd import sssp
    return m, sssp


def inst(sssp, W, n, src=0, ld=None):
    return sssp.sssp_instance(W, n if ld is None else ld, n, src, FAKE, FAKE)


def check_layout(entries, arena, instances, single_max_n, gang_columns, max_parts, lc=False):
    count = len(instances)
    assert sorted(e["instance"] for e in entries) == list(range(count))
    uses = {}
    for I in instances:
        uses[(I.W, I.ld)] = uses.get((I.W, I.ld), 0) + 1
    shared = [uses[(I.W, I.ld)] >= SHARED and I.n <= 16384 for I in instances]
    # order: unshared by n descending (stable), then shared by n descending
    keys = [(shared[e["instance"]], -instances[e["instance"]].n) for e in entries]
    assert keys == sorted(keys)
    off = 0
    for e in entries:
        I = instances[e["instance"]]
        n = I.n
        if shared[e["instance"]] or (not lc and n <= single_max_n):
            assert (e["parts"], e["columns"], e["method"]) == (1, n, 0)
            assert (e["scratch_offset"], e["scratch_bytes"]) == (-1, 0)
            continue
        cols, parts = e["columns"], e["parts"]
        assert cols % 4 == 0 and parts * cols >= n and (parts - 1) * cols < n
        if lc:
            assert e["method"] == 1 and parts >= 1
            assert cols <= 256 or parts == max_parts
        else:
            assert e["method"] == 0 and parts >= 2
            want = max(2, min(-(-n // gang_columns), max_parts))
            assert parts <= want
            assert cols <= gang_columns or parts >= min(want, max_parts)
        assert parts <= max(2, max_parts)
        # arena: consecutive, 256-byte aligned, records and lists fit
        assert e["scratch_offset"] == off and off % 256 == 0
        entry = 8 if lc else 4
        assert e["scratch_bytes"] >= 2 * parts * 32 + 2 * parts * cols * entry
        off += e["scratch_bytes"]
    assert arena == off


def test_random_instance_sets(sp):
    m, sssp = sp
    rng = np.random.default_rng(1400)
    for trial in range(200):
        count = int(rng.integers(1, 60))
        mats = [(FAKE * (k + 2), int(n)) for k, n in enumerate(rng.integers(1, 40000, size=int(rng.integers(1, 8))))]
        instances = []
        for _ in range(count):
            W, n = mats[int(rng.integers(0, len(mats)))]
            instances.append(inst(sssp, W, n, int(rng.integers(0, n))))
        if trial % 5 == 0:  # a matrix with many sources
            W, n = FAKE * 99, int(rng.integers(100, 9000))
            instances += [inst(sssp, W, n, s % n) for s in range(SHARED + int(rng.integers(0, 20)))]
        single = int(rng.choice([0, 256, 1024, 4096]))
        cols = int(rng.choice([0, 256, 512, 2048]))
        maxp = int(rng.choice([0, 8, 64, 512]))
        lc = bool(trial % 7 == 3)
        entries, arena = m.sssp_batch_layout(instances, LC if lc else 0, single, cols, maxp)
        check_layout(entries, arena, instances, single or 16384, cols or 4096, maxp or 512, lc)


def test_shared_matrix_rule(sp):
    m, sssp = sp
    big = [inst(sssp, FAKE * 7, 8192, s) for s in range(SHARED)]
    few = [inst(sssp, FAKE * 8, 8192, s) for s in range(SHARED - 1)]
    entries, _ = m.sssp_batch_layout(big + few, 0, 1024, 1024, 64)
    by = {e["instance"]: e for e in entries}
    assert all(by[i]["parts"] == 1 for i in range(SHARED))                      # shared: one workgroup each
    assert all(by[i]["parts"] == 8 for i in range(SHARED, 2 * SHARED - 1))    # not shared: gangs
    assert [e["instance"] for e in entries][-SHARED:] == list(range(SHARED))   # and queued last
    # the label-correcting method is never used for shared matrices
    entries, _ = m.sssp_batch_layout(big, LC, 0, 0, 0)
    assert all(e["method"] == 0 and e["parts"] == 1 for e in entries)


def test_edges_and_errors(sp):
    m, sssp = sp
    e, arena = m.sssp_batch_layout([inst(sssp, FAKE, 1)])
    assert e == [{"instance": 0, "parts": 1, "columns": 1, "method": 0, "scratch_offset": -1, "scratch_bytes": 0}]
    assert arena == 0
    assert m.sssp_batch_layout([]) == ([], 0)
    # n just above single_max_n makes a gang of two
    e, _ = m.sssp_batch_layout([inst(sssp, FAKE, 1025)], 0, 1024, 4096, 64)
    assert e[0]["parts"] == 2 and e[0]["columns"] == 516
    # too few members for the columns: unsupported
    with pytest.raises(sssp.SsspError) as x:
        m.sssp_batch_layout([inst(sssp, FAKE, 200000)], 0, 1024, 1024, 2)
    assert x.value.code == sssp.SSSP_EUNSUPPORTED
    for bad, kw in ((inst(sssp, FAKE, 10, 10), {}), (inst(sssp, FAKE, 10, 0, ld=5), {}), (inst(sssp, 0, 10), {}),
                    (inst(sssp, FAKE, 10), {"gang_columns": 6}), (inst(sssp, FAKE, 10), {"single_max_n": 1 << 20})):
        with pytest.raises(sssp.SsspError) as x:
            m.sssp_batch_layout([bad], **kw)
        assert x.value.code == sssp.SSSP_EINVAL
    lib = sssp.lib()
    assert lib.sssp_batch_layout(None, 1, 0, 0, 0, 0, None, None) == sssp.SSSP_EINVAL
    one = (sssp.sssp_instance * 1)(inst(sssp, FAKE, 10))
    assert lib.sssp_batch_layout(one, 1, 0, 0, 0, 0, None, None) == sssp.SSSP_EINVAL
    arena = ctypes.c_int64(-5)
    assert lib.sssp_batch_layout(one, 0, 0, 0, 0, 0, None, ctypes.byref(arena)) == 0 and arena.value == 0
