"""bench.py's command line on the CPU: more than one GPU is refused with a message
(exit status 2) before anything touches a device; the sections are listed."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_help_lists_sections():
    r = run("--help")
    assert r.returncode == 0
    for sec in ("medium", "many_levels", "sparse", "small", "batched", "served"):
        assert sec in r.stdout
