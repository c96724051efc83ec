"""Builds the input generators: gen_host.c with gcc, gen_device.hip with hipcc for gfx950."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
HOST_SO = os.path.join(HERE, "libsssp_gen_host.so")
DEV_SO = os.path.join(HERE, "libsssp_gen_dev.so")

HIP_FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-shared", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))


def build(device=True):
    _run(["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-o", HOST_SO,
          os.path.join(HERE, "gen_host.c")])
    if device:
        _run(["/opt/rocm/bin/hipcc"] + HIP_FLAGS +
             ["-o", DEV_SO, os.path.join(HERE, "gen_device.hip")])


if __name__ == "__main__":
    build()
