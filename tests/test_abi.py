"""CPU checks of the C ABI: the library loads, exports every entry point that
include/*.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*[A-Za-z_][\w\s\*]*?\b(sssp_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def L():
    import paper_2504_03667_amd as sp
    return sp.lib()


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert "sssp_dense_solve" in names and "sssp_dense_solve_batched" in names
    for name in sorted(names):
        assert hasattr(L, name), name


def test_argument_validation_without_gpu(L):
    import paper_2504_03667_amd.sssp as s
    P = ctypes.c_void_p
    fake = P(4096)  # never dereferenced: validation fails first
    assert L.sssp_dense_solve(None, 10, 0, fake, fake, None) == s.SSSP_EINVAL
    assert b"null" in L.sssp_last_error()
    assert L.sssp_dense_solve(fake, 0, 0, fake, fake, None) == s.SSSP_EINVAL
    assert L.sssp_dense_solve(fake, 10, 10, fake, fake, None) == s.SSSP_EINVAL
    assert L.sssp_dense_solve(fake, 10, -1, fake, fake, None) == s.SSSP_EINVAL
    assert L.sssp_dense_solve_ex(fake, 9, 10, 0, fake, fake, 0, None, None) == s.SSSP_EINVAL
    assert b"ld" in L.sssp_last_error()
    assert L.sssp_dense_solve_ex(fake, 10, 10, 0, fake, fake,
                                 s.SSSP_FLAG_SINGLE | s.SSSP_FLAG_GRID, None, None) == s.SSSP_EINVAL
    arr = (s.sssp_instance * 1)()
    arr[0].W, arr[0].ld, arr[0].n, arr[0].src = 4096, 5, 5, 7
    arr[0].dist, arr[0].pred = 4096, 4096
    assert L.sssp_dense_solve_batched(arr, 1, 0, None, None) == s.SSSP_EINVAL
    assert b"instance 0" in L.sssp_last_error()
    assert L.sssp_stream_read(None, 64, 0, None, None) == s.SSSP_EINVAL
    assert L.sssp_stream_read(P(4100), 64, 0, None, None) == s.SSSP_EINVAL   # not 16-byte aligned
    assert L.sssp_stream_read(fake, 8, 0, None, None) == s.SSSP_EINVAL       # under one 16-byte word
    assert L.sssp_stream_read(fake, 40, 0, None, None) == s.SSSP_EINVAL      # not a multiple of 16
    assert L.sssp_stream_read(fake, 64, 512, None, None) == s.SSSP_EINVAL    # chunk under 1 KiB
    assert L.sssp_stream_read(fake, 64, 1032, None, None) == s.SSSP_EINVAL   # chunk not a multiple of 16
    assert L.sssp_strerror(s.SSSP_EAGAIN) == b"try again"
    assert L.sssp_version() >= 1


def test_load_release_unload_twice(tmp_path):
    """Two load / release / unload cycles of separate copies of the library: the
    release calls succeed with nothing held, report zero scratch, and dlclose
    returns cleanly (no kernel is launched)."""
    import _ctypes
    import shutil
    import paper_2504_03667_amd.sssp as s
    for rep in range(2):
        path = str(tmp_path / ("libsssp_copy%d.so" % rep))
        shutil.copy(s.SO, path)
        L = ctypes.CDLL(path)
        L.sssp_scratch_bytes.argtypes = [ctypes.POINTER(ctypes.c_int64)]
        b = ctypes.c_int64(-1)
        assert L.sssp_scratch_bytes(ctypes.byref(b)) == s.SSSP_OK and b.value == 0
        assert L.sssp_release_all() == s.SSSP_OK
        assert L.sssp_scratch_bytes(None) == s.SSSP_EINVAL
        _ctypes.dlclose(L._handle)
