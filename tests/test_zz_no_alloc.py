"""GPU tests of sssp_dense_solve_noalloc, the dense solve whose library scratch is
a fixed per-GPU array: through the C ABI, its dist/pred/status must equal those
of sssp_dense_solve_ex (the entry point with allocated scratch) bit for bit, on
consecutive calls that reuse the array with different shapes."""
import ctypes

import numpy as np
import pytest

import gen
import oracle
from tests.graphs import random_dense

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SINGLE, GRID, LITERAL = 2, 4, 1


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_03667_amd as m
    m.lib()
    return m


def outputs(n):
    return (torch.full((n,), -5, dtype=torch.int32, device="cuda"),
            torch.full((n,), -5, dtype=torch.int32, device="cuda"),
            torch.full((1,), -5, dtype=torch.int32, device="cuda"))


def compare(sp, Wt, src, flags, tag):
    """One no-alloc call and one sssp_dense_solve_ex call on the same input."""
    n = Wt.shape[0]
    d, p, st = outputs(n)
    print("noalloc case", tag, "n", n, "src", src, "flags", flags, flush=True)
    sp.sssp_dense_solve_noalloc(Wt, Wt.stride(0), n, src, d, p, flags, st)
    torch.cuda.current_stream().synchronize()
    d_ref, p_ref, _ = outputs(n)
    sp.sssp_dense_solve_ex(Wt, Wt.stride(0), n, src, d_ref, p_ref, flags)
    status_ref, _ = sp.sssp_last_status()
    assert int(st.item()) == status_ref and status_ref & 3 == 0, (tag, int(st.item()), status_ref)
    dd, pp = d.cpu().numpy(), p.cpu().numpy()
    assert np.array_equal(dd, d_ref.cpu().numpy()), tag
    assert np.array_equal(pp, p_ref.cpu().numpy()), tag
    return dd, pp, status_ref


def test_noalloc_matches_allocating_entry_point(sp):
    # first call: the n=16384 workload (p=0.01, weights [1, 100]) on the whole GPU
    spec = gen.GraphSpec(16384, 0.01, 1, 100, gen.SEED_BASE + 2)
    Wt = gen.dense_device(spec)
    compare(sp, Wt, 12345, GRID, "n16384-grid")
    del Wt
    # second call, smaller and with zero weights (fallback rounds), checked against the oracle too
    rng = np.random.default_rng(71)
    W = random_dense(rng, 3001, 0.02, 1, 50, directed=True, zero_prob=0.05)
    Wt = torch.from_numpy(W).cuda()
    dd, pp, status = compare(sp, Wt, 17, GRID, "n3001-grid-zero")
    dr, pr, _ = oracle.dijkstra(W, 17)
    assert np.array_equal(dd, dr) and np.array_equal(pp, pr)
    assert status & sp.SSSP_STATUS_ZERO_FALLBACK
    # literal mode, one-workgroup kernels (default crossover and forced), a padded row stride
    compare(sp, Wt, 0, GRID | LITERAL, "n3001-grid-literal")
    compare(sp, Wt, 5, SINGLE, "n3001-single")
    small = torch.from_numpy(random_dense(rng, 700, 0.1, 1, 9)).cuda()
    compare(sp, small, 3, 0, "n700-default")
    big = torch.full((900, 1000), 7, dtype=torch.int32, device="cuda")
    Wp = torch.from_numpy(random_dense(rng, 900, 0.05, 1, 30)).cuda()
    big[:, :900] = Wp
    d, p, st = outputs(900)
    sp.sssp_dense_solve_noalloc(big, 1000, 900, 4, d, p, GRID, st)
    d_ref, p_ref = sp.solve(Wp, 4, flags=GRID)
    assert np.array_equal(d.cpu().numpy(), d_ref.cpu().numpy())
    assert np.array_equal(p.cpu().numpy(), p_ref.cpu().numpy())
    assert int(st.item()) == 0


def test_noalloc_status_and_limits(sp, monkeypatch):
    """The status output carries a barrier time-out forced from the host (every
    wait gives up at once), the next call is clean again, and sizes beyond the
    fixed scratch are refused before anything is launched."""
    rng = np.random.default_rng(72)
    W = random_dense(rng, 4000, 0.05, 1, 100)
    Wt = torch.from_numpy(W).cuda()
    d, p, st = outputs(4000)
    monkeypatch.setenv("SSSP_BARRIER_TIMEOUT_US", "0")
    sp.sssp_dense_solve_noalloc(Wt, 4000, 4000, 0, d, p, GRID, st)
    torch.cuda.current_stream().synchronize()
    assert int(st.item()) & sp.SSSP_STATUS_TIMEOUT
    monkeypatch.delenv("SSSP_BARRIER_TIMEOUT_US")
    compare(sp, Wt, 0, GRID, "after-timeout")
    L = sp.lib()
    fake = ctypes.c_void_p(Wt.data_ptr())
    n = sp.SSSP_NOALLOC_MAX_N + 1
    assert L.sssp_dense_solve_noalloc(fake, n, n, 0, fake, fake, 0, None, None) == sp.sssp.SSSP_EUNSUPPORTED
    assert b"SSSP_NOALLOC_MAX_N" in L.sssp_last_error()
    assert L.sssp_dense_solve_noalloc(fake, 4000, 4000, 0, fake, fake, sp.SSSP_FLAG_LABEL_CORRECTING,
                                      None, None) == sp.sssp.SSSP_EUNSUPPORTED
