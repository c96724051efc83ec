"""Builds the CPU oracle (plain C, gcc -O2) into oracle/liboracle.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "liboracle.so")


def build():
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-pthread", "-o", SO, os.path.join(HERE, "oracle.c")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("oracle build failed:\n%s\n%s" % (r.stdout, r.stderr))


if __name__ == "__main__":
    build()
