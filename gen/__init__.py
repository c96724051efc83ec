"""Seeded synthetic inputs: dense G(n, p) weight matrices and the workload manifests.

This module is shared by the oracle side and the GPU side and holds none of the
shortest-path arithmetic.  Every matrix entry is a pure function of
(seed, i, j) (see gen_host.c for the formula); parameter draws (graph sizes,
densities, sources, query arrival times) come from a sequential SplitMix64
stream.  The paper's own graph files are not available, so these seeded
G(n, p) graphs stand in for its edge lists (Section IV-A); the matrix format
follows Section III-A (row = tail, infinity = no edge, zero diagonal).
"""
import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import List

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
INF = 0x7FFFFFFF
SEED_BASE = 2504036670
MASK64 = (1 << 64) - 1

_host = None
_dev = None


def mix64(x):
    """SplitMix64 finaliser (Steele, Lea & Flood 2014), on Python ints."""
    x = (x + 0x9E3779B97F4A7C15) & MASK64
    x = ((x ^ (x >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    x = ((x ^ (x >> 27)) * 0x94D049BB133111EB) & MASK64
    return x ^ (x >> 31)


def threshold(p):
    """Edge threshold floor(p * 2^32); an entry is an edge iff hi32(hash) < threshold."""
    if not (0.0 <= p <= 1.0):
        raise ValueError("p must be in [0, 1]")
    return int(math.floor(p * 4294967296.0))


class Stream:
    """Sequential SplitMix64 stream for parameter draws (sizes, sources, arrivals)."""

    def __init__(self, seed):
        self.state = seed & MASK64

    def next_u64(self):
        self.state = (self.state + 0x9E3779B97F4A7C15) & MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        return z ^ (z >> 31)

    def uniform(self):
        """Uniform double in [0, 1) with 53 random bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def below(self, k):
        """Integer in [0, k) by multiply-shift of a 64-bit draw."""
        return (self.next_u64() * k) >> 64

    def loguniform_int(self, lo, hi):
        v = int(math.floor(math.exp(math.log(lo) + self.uniform() * (math.log(hi + 1) - math.log(lo)))))
        return min(max(v, lo), hi)

    def loguniform(self, lo, hi):
        return math.exp(math.log(lo) + self.uniform() * (math.log(hi) - math.log(lo)))

    def sample_distinct(self, k, n):
        """k distinct integers from [0, n), by a partial Fisher-Yates shuffle."""
        perm = {}
        out = []
        for i in range(k):
            j = i + self.below(n - i)
            vi, vj = perm.get(i, i), perm.get(j, j)
            perm[i], perm[j] = vj, vi
            out.append(vj)
        return out


def _host_lib():
    global _host
    if _host is None:
        path = os.path.join(HERE, "libsssp_gen_host.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build(device=False)
        lib = ctypes.CDLL(path)
        lib.gen_dense_fill.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                       ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        lib.gen_dense_fill.restype = ctypes.c_int
        lib.gen_dense_fill_rows.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                            ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32]
        lib.gen_dense_fill_rows.restype = ctypes.c_int
        lib.gen_dense_checksum.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                           ctypes.c_int32]
        lib.gen_dense_checksum.restype = ctypes.c_uint64
        lib.gen_entry_c.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        lib.gen_entry_c.restype = ctypes.c_int32
        lib.gen_mix64_c.argtypes = [ctypes.c_uint64]
        lib.gen_mix64_c.restype = ctypes.c_uint64
        lib.gen_sparse_edges.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.gen_sparse_edges.restype = ctypes.c_int
        _host = lib
    return _host


def _dev_lib():
    global _dev
    if _dev is None:
        path = os.path.join(HERE, "libsssp_gen_dev.so")
        if not os.path.exists(path):
            raise RuntimeError("device generator not built: run __graft_entry__.build()")
        import torch  # noqa: F401  (share torch's HIP runtime)
        lib = ctypes.CDLL(path)
        lib.gen_dense_fill_device.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                              ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                              ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int32, ctypes.c_void_p]
        lib.gen_dense_fill_device.restype = ctypes.c_int
        lib.gen_dense_checksum_device.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                                  ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p]
        lib.gen_dense_checksum_device.restype = ctypes.c_int
        _dev = lib
    return _dev


def default_threads():
    return max(1, min(16, os.cpu_count() or 1))


@dataclass(frozen=True)
class GraphSpec:
    """One synthetic dense graph: G(n, p) with integer weights uniform in [lo, hi]."""
    n: int
    p: float
    lo: int
    hi: int
    seed: int
    directed: bool = False

    @property
    def thresh(self):
        return threshold(self.p)

    def host(self, ld=None, threads=None):
        return dense_host(self, ld=ld, threads=threads)

    def device(self, ld=None, device="cuda"):
        return dense_device(self, ld=ld, device=device)


def dense_host(spec, ld=None, threads=None):
    """int32 [n, ld] numpy matrix of `spec` (columns >= n, if any, hold INF)."""
    n = spec.n
    ld = n if ld is None else ld
    if ld < n:
        raise ValueError("ld < n")
    W = np.full((n, ld), INF, dtype=np.int32) if ld != n else np.empty((n, n), dtype=np.int32)
    if n == 0:
        return W
    rc = _host_lib().gen_dense_fill(W.ctypes.data, ld, n, spec.seed & MASK64, spec.thresh,
                                    spec.lo, spec.hi, int(spec.directed),
                                    threads or default_threads())
    if rc != 0:
        raise ValueError("gen_dense_fill rejected the arguments")
    return W


def dense_rows_host(spec, r0, rows):
    """Rows [r0, r0+rows) of the matrix, int32 [rows, n]."""
    out = np.empty((rows, spec.n), dtype=np.int32)
    rc = _host_lib().gen_dense_fill_rows(out.ctypes.data, spec.n, spec.n, r0, rows,
                                         spec.seed & MASK64, spec.thresh, spec.lo, spec.hi,
                                         int(spec.directed))
    if rc != 0:
        raise ValueError("gen_dense_fill_rows rejected the arguments")
    return out


def dense_numpy(spec):
    """The same matrix computed with numpy uint64 arithmetic (small n; cross-checks the C code)."""
    n = spec.n
    i = np.arange(n, dtype=np.uint64)[:, None]
    j = np.arange(n, dtype=np.uint64)[None, :]
    if spec.directed:
        key = (i << np.uint64(32)) | j
    else:
        a, b = np.minimum(i, j), np.maximum(i, j)
        key = (a << np.uint64(32)) | b
    with np.errstate(over="ignore"):
        x = np.uint64(mix64(spec.seed & MASK64)) ^ key
        x = x + np.uint64(0x9E3779B97F4A7C15)
        x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        h = x ^ (x >> np.uint64(31))
        span = np.uint64(spec.hi - spec.lo + 1)
        w = (np.uint64(spec.lo) + (((h & np.uint64(0xFFFFFFFF)) * span) >> np.uint64(32)))
    edge = (h >> np.uint64(32)) < np.uint64(spec.thresh)
    W = np.where(edge, w.astype(np.int64), INF).astype(np.int32)
    np.fill_diagonal(W, 0)
    return W


def checksum_host(W, threads=None):
    W = np.ascontiguousarray(W, dtype=np.int32)
    n = W.shape[0]
    return int(_host_lib().gen_dense_checksum(W.ctypes.data, W.shape[1], n,
                                              threads or default_threads()))


def dense_device(spec, ld=None, device="cuda", out=None):
    """int32 [n, ld] torch tensor on the GPU, written in place by the device generator."""
    import torch
    n = spec.n
    ld = n if ld is None else ld
    if out is None:
        out = torch.full((n, ld), INF, dtype=torch.int32, device=device) if ld != n else \
            torch.empty((n, n), dtype=torch.int32, device=device)
    if n:
        stream = torch.cuda.current_stream(out.device).cuda_stream
        rc = _dev_lib().gen_dense_fill_device(out.data_ptr(), ld, n, 0, n, spec.seed & MASK64,
                                              spec.thresh, spec.lo, spec.hi,
                                              int(spec.directed), ctypes.c_void_p(stream))
        if rc != 0:
            raise RuntimeError("gen_dense_fill_device failed: hip error %d" % rc)
    return out


def checksum_device(Wt):
    import torch
    n, ld = Wt.shape[0], Wt.stride(0)
    v = ctypes.c_uint64(0)
    stream = torch.cuda.current_stream(Wt.device).cuda_stream
    rc = _dev_lib().gen_dense_checksum_device(Wt.data_ptr(), ld, n, ctypes.byref(v),
                                              ctypes.c_void_p(stream))
    if rc != 0:
        raise RuntimeError("gen_dense_checksum_device failed: hip error %d" % rc)
    return int(v.value)


def sparse_edges(n, m, lo, hi, seed):
    """The seeded edge list (u, v, w) of a sparse graph: m edges among n vertices
    (see gen_sparse_edges in gen_host.c); numpy int32 arrays."""
    eu = np.empty(m, np.int32)
    ev = np.empty(m, np.int32)
    ew = np.empty(m, np.int32)
    if _host_lib().gen_sparse_edges(n, m, lo, hi, seed, eu.ctypes.data, ev.ctypes.data, ew.ctypes.data) != 0:
        raise ValueError("bad sparse graph parameters")
    return eu, ev, ew


@dataclass
class SparseSpec:
    n: int
    m: int          # edges drawn (an undirected graph stores each in both orientations)
    lo: int
    hi: int
    seed: int
    directed: bool = False


# ---------------------------------------------------------------------------
# Workload manifests.  Base seed S; workload k uses S + k.
# ---------------------------------------------------------------------------

@dataclass
class Query:
    graph: int
    src: int
    arrival_s: float


@dataclass
class Workload:
    name: str
    graphs: List[GraphSpec]
    # (graph index, source) pairs solved by the workload
    instances: List[tuple] = field(default_factory=list)
    queries: List[Query] = field(default_factory=list)


def workload_single_small():
    """n=1024 undirected, p=0.1, weights in [1,100], source 0."""
    g = GraphSpec(1024, 0.1, 1, 100, SEED_BASE + 1)
    return Workload("sssp_n1024_p0.1_undirected", [g], [(0, 0)])


def workload_single_medium():
    """n=16384, p=0.01, weights in [1,100]; undirected and directed; sources 0, 7, 12345."""
    gu = GraphSpec(16384, 0.01, 1, 100, SEED_BASE + 2)
    gd = GraphSpec(16384, 0.01, 1, 100, SEED_BASE + 3, directed=True)
    inst = [(0, s) for s in (0, 7, 12345)] + [(1, s) for s in (0, 7, 12345)]
    return Workload("sssp_n16384_p0.01", [gu, gd], inst)


def workload_single_large():
    """n=65536 undirected, p=0.5, weights in [1,1000] (16 GiB matrix), source 0."""
    g = GraphSpec(65536, 0.5, 1, 1000, SEED_BASE + 4)
    return Workload("sssp_n65536_p0.5_undirected", [g], [(0, 0)])


def workload_batched(shared_sources=256, n_graphs=64):
    """(a) `shared_sources` distinct sources on one n=8192, p=0.05 graph, plus (b)
    `n_graphs` graphs with n log-uniform in [512, 8192], p uniform in [0.005, 0.5],
    one uniformly drawn source each; weights in [1,100]."""
    st = Stream(SEED_BASE + 5)
    g0 = GraphSpec(8192, 0.05, 1, 100, SEED_BASE + 5)
    srcs = st.sample_distinct(shared_sources, g0.n)
    graphs = [g0]
    inst = [(0, s) for s in srcs]
    for _ in range(n_graphs):
        n = st.loguniform_int(512, 8192)
        p = 0.005 + st.uniform() * (0.5 - 0.005)
        seed = st.next_u64()
        graphs.append(GraphSpec(n, p, 1, 100, seed))
        inst.append((len(graphs) - 1, st.below(n)))
    return Workload("batched_256src_n8192_plus_64graphs", graphs, inst)


def workload_serving(n_graphs=32, n_queries=20000, rate_qps=2000.0):
    """`n_graphs` resident graphs, n log-uniform in [256, 32768], p log-uniform in
    [0.001, 0.5], weights in [1,1000]; `n_queries` queries (uniform graph, uniform
    source) with Poisson arrivals at `rate_qps`."""
    st = Stream(SEED_BASE + 6)
    graphs = []
    for _ in range(n_graphs):
        n = st.loguniform_int(256, 32768)
        p = st.loguniform(0.001, 0.5)
        graphs.append(GraphSpec(n, p, 1, 1000, st.next_u64()))
    t = 0.0
    qs = []
    for _ in range(n_queries):
        g = st.below(n_graphs)
        s = st.below(graphs[g].n)
        t += -math.log(1.0 - st.uniform()) / rate_qps
        qs.append(Query(g, s, t))
    return Workload("served_32graphs_20000q_2000qps", graphs, queries=qs)


def workload_sparse():
    """The paper's sparse family (m = 3n undirected edges; Section IV-A lists
    n = 10000, 20000, 40000), weights in [1, 1000], source 0, plus n = 10^6 with
    m = 3 * 10^6, far beyond what an n x n matrix could hold."""
    specs = [SparseSpec(n, 3 * n, 1, 1000, SEED_BASE + 7 + k) for k, n in enumerate((10000, 20000, 40000, 1000000))]
    return Workload("sparse_m3n", [], [(k, 0) for k in range(len(specs))]), specs
