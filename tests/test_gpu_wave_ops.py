"""The wave-wide minimum, OR and prefix sum of the kernels (DPP row shifts plus
lane reads) against the same operations on the host, on one GPU."""
import os
import subprocess

import pytest

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "native", "_build", "wave_ops")


@pytest.mark.gpu
def test_wave_primitives_match_host():
    assert os.path.exists(EXE), "build the package first (paper_2504_03667_amd.build.build())"
    print("wave ops program", flush=True)
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "wave ops ok" in r.stdout
