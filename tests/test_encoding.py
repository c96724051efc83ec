"""Host-only checks of encodings the kernels rely on, compiled from the library's
own headers (no GPU needed; no kernel is launched)."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_exchange_stamps_never_match_stale_words():
    """Gang records are reused without clearing: a stamp must differ from every list
    entry and record word an earlier use can leave at a stamp's offset."""
    src = os.path.join(ROOT, "tests", "native", "stamp_encoding.cpp")
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "stamp_encoding")
        b = subprocess.run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17",
                            "-I", os.path.join(ROOT, "include"),
                            "-I", os.path.join(ROOT, "paper_2504_03667_amd", "csrc"), src, "-o", exe],
                           capture_output=True, text=True)
        assert b.returncode == 0, b.stderr[-3000:]
        r = subprocess.run([exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        assert "stamp encoding ok" in r.stdout
