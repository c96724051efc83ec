"""Builds libsssp.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
SO = os.path.join(HERE, "libsssp.so")
HIPCC = "/opt/rocm/bin/hipcc"

SOURCES = ["kernels.hip", "lc.hip", "csr.hip", "api.cpp", "server.cpp", "batch.cpp", "paths.hip", "diag.hip",
           "noalloc.hip"]
FLAGS = ["-O3", "--offload-arch=gfx950", "-fPIC", "-std=c++17", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return r.stderr


# Test build: the same sources with pseudo-random pauses before every exchange
# and barrier arrival (stress_delay), loaded only by the barrier-stress tests.
SO_STRESS = os.path.join(HERE, "libsssp_stress.so")
VARIANTS = ((SO, BUILD, []), (SO_STRESS, BUILD + "_stress", ["-DSSSP_STRESS_DELAYS=1"]))


# GPU test programs built from the library's headers (run by the gpu-marked tests).
TEST_NATIVE = os.path.join(ROOT, "tests", "native")
TEST_PROGRAMS = [(os.path.join(TEST_NATIVE, "wave_ops.hip"), os.path.join(TEST_NATIVE, "_build", "wave_ops"))]


def build_test_program(src, exe):
    os.makedirs(os.path.dirname(exe), exist_ok=True)
    _run([HIPCC] + FLAGS + ["-x", "hip", src, "-o", exe + ".tmp"])
    os.replace(exe + ".tmp", exe)


def build(verbose=False):
    jobs = []
    for so, folder, extra in VARIANTS:
        os.makedirs(folder, exist_ok=True)
        jobs += [(src, folder, extra) for src in SOURCES]

    def compile_one(job):
        src, folder, extra = job
        obj = os.path.join(folder, src + ".o")
        cmd = [HIPCC] + FLAGS + extra + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        err = _run(cmd)
        if verbose and err.strip():
            sys.stderr.write(err)
        return obj

    with ThreadPoolExecutor(min(len(jobs) + len(TEST_PROGRAMS), os.cpu_count() or 8)) as ex:
        tests = [ex.submit(build_test_program, src, exe) for src, exe in TEST_PROGRAMS]
        objs = list(ex.map(compile_one, jobs))
        for t in tests:
            t.result()
    for i, (so, _, _) in enumerate(VARIANTS):
        tmp = so + ".tmp"
        _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] +
             objs[i * len(SOURCES):(i + 1) * len(SOURCES)])
        os.replace(tmp, so)
    return SO


# The files the whole-GPU solve (its kernel, launch shape and flags) is built from;
# a profile taken of that kernel stays valid while none of them changes.
GRID_KERNEL_FILES = ("kernels.hip", "solve.h", "lc.h", "engine.h", "sssp_internal.h", "api.cpp")


def code_tokens(text):
    """C/C++ source without its comments and with runs of whitespace collapsed: what
    the compiler sees of it (string and character literals are kept as written)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def source_hash(files=GRID_KERNEL_FILES):
    """Short hash of the code (comments and layout excluded) the whole-GPU solve is
    built from, plus the public header and the compiler flags set in this file:
    ties profiles to the code they measured, and survives comment-only edits."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(files):
        with open(os.path.join(CSRC, name)) as f:
            h.update(name.encode() + b"\0" + code_tokens(f.read()).encode())
    with open(os.path.join(ROOT, "include", "sssp.h")) as f:
        h.update(code_tokens(f.read()).encode())
    h.update(" ".join(f for f in FLAGS if os.sep not in f).encode())  # flags, not paths
    return h.hexdigest()[:16]


if __name__ == "__main__":
    build(verbose=True)
