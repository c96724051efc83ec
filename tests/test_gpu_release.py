"""GPU tests of the library's scratch ownership: per-stream scratch is freed by
sssp_stream_release and sssp_release_all, a released stream solves again
correctly, and loading, using, releasing and unloading the library twice leaves
the device's free memory where it was."""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

import oracle
from tests.graphs import random_dense

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sp():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2504_03667_amd as m
    m.lib()
    return m


def test_stream_release_and_release_all(sp):
    rng = np.random.default_rng(81)
    W = random_dense(rng, 6000, 0.02, 1, 100)
    Wt = torch.from_numpy(W).cuda()
    dr, pr, _ = oracle.dijkstra(W, 9)
    sp.sssp_release_all()
    assert sp.sssp_scratch_bytes() == 0
    streams = [torch.cuda.Stream() for _ in range(3)]
    held = []
    for k, s in enumerate(streams):
        with torch.cuda.stream(s):
            flags = sp.SSSP_FLAG_GRID | (sp.SSSP_FLAG_LABEL_CORRECTING if k == 2 else 0)
            d, p = sp.solve(Wt, 9, flags=flags)
            s.synchronize()
            assert np.array_equal(d.cpu().numpy(), dr) and np.array_equal(p.cpu().numpy(), pr), k
        held.append(sp.sssp_scratch_bytes())
    assert 0 < held[0] < held[1] < held[2]
    sp.sssp_stream_release(streams[1])
    assert sp.sssp_scratch_bytes() == held[2] - (held[1] - held[0])
    with pytest.raises(sp.SsspError):
        sp.sssp_last_status(streams[1])  # forgotten with its scratch
    with torch.cuda.stream(streams[1]):
        d, p = sp.solve(Wt, 9, flags=sp.SSSP_FLAG_GRID)
        status, _ = sp.sssp_last_status(streams[1])
    assert status & 3 == 0
    assert np.array_equal(d.cpu().numpy(), dr) and np.array_equal(p.cpu().numpy(), pr)
    sp.sssp_release_all()
    assert sp.sssp_scratch_bytes() == 0
    d, p = sp.solve(Wt, 9, flags=sp.SSSP_FLAG_GRID)
    assert np.array_equal(d.cpu().numpy(), dr) and np.array_equal(p.cpu().numpy(), pr)


CYCLES = r"""
import ctypes, _ctypes, os, shutil, sys, tempfile
import torch
sys.path.insert(0, ROOT)
import paper_2504_03667_amd.sssp as s
n = 65536
W = torch.full((n, n), 0x7FFFFFFF, dtype=torch.int32, device="cuda")
W.diagonal().zero_()
W[0, 1:] = 5
d = torch.empty(n, dtype=torch.int32, device="cuda")
p = torch.empty(n, dtype=torch.int32, device="cuda")
streams = [torch.cuda.Stream() for _ in range(8)]
tmp = tempfile.mkdtemp()
free = []
for rep in range(2):
    path = os.path.join(tmp, "libsssp_cycle%d.so" % rep)
    shutil.copy(s.SO, path)
    L = s._declare(ctypes.CDLL(path))
    for k, st in enumerate(streams):
        flags = s.SSSP_FLAG_GRID | (s.SSSP_FLAG_LABEL_CORRECTING if k % 2 else 0)
        rc = L.sssp_dense_solve_ex(ctypes.c_void_p(W.data_ptr()), n, n, 0, ctypes.c_void_p(d.data_ptr()),
                                   ctypes.c_void_p(p.data_ptr()), flags, None, ctypes.c_void_p(st.cuda_stream))
        assert rc == 0, (rc, L.sssp_last_error())
        st.synchronize()  # whole-GPU grids: one at a time (a concurrent cooperative launch is refused)
    assert int(d[7]) == 5 and int(p[7]) == 0
    b = ctypes.c_int64(0)
    L.sssp_scratch_bytes(ctypes.byref(b))
    assert b.value > 8 * 500000, b.value
    held = b.value
    assert L.sssp_release_all() == 0
    L.sssp_scratch_bytes(ctypes.byref(b))
    assert b.value == 0
    _ctypes.dlclose(L._handle)
    torch.cuda.synchronize()
    free.append(torch.cuda.mem_get_info()[0])
    print("cycle", rep, "held", held, "free after release and unload", free[-1], flush=True)
grown = free[0] - free[1]
print("device memory lost by the second cycle:", grown, flush=True)
assert grown < held // 2, (grown, held)
print("cycles ok", flush=True)
"""


def test_load_use_release_unload_twice(sp):
    """In a child process (so that a failure cannot take this one down): two cycles
    of loading a copy of the library, solving on 8 streams (each holding its own
    scratch, about 1 MB at n=65536), sssp_release_all and dlclose; the second
    cycle must not lose device memory beyond half of what a cycle held."""
    code = "ROOT = %r\n" % ROOT + textwrap.dedent(CYCLES)
    # the ordinary launch of the same whole-GPU grids: this process may hold the
    # device's cooperative-launch resources, and a second process's cooperative
    # launch is then refused
    env = dict(os.environ, SSSP_GRID_LAUNCH="plain")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240, env=env)
    print(r.stdout)
    assert r.returncode == 0 and "cycles ok" in r.stdout, r.stderr[-3000:]
