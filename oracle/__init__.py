"""CPU oracle for dense-matrix single-source shortest paths (Algorithm 1 of the paper).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product library.  The arithmetic
lives in oracle.c (plain serial C, exact int64 sums); this file only marshals
numpy arrays.  See oracle.c for the readings taken where the paper is silent
(tie rule, pred initial value, infinity encoding, early exit).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
INF = 0x7FFFFFFF
INF64 = 1 << 62
_lib = None

CERT_CODES = {
    0: "ok",
    1: "dist[src] != 0 or pred[src] != -1",
    2: "infeasible edge: dist[u] + W[u][v] < dist[v]",
    3: "pred edge of a reachable vertex is not tight",
    4: "unreachable vertex with pred != -1",
    5: "pred chain does not reach the source",
}


def lib():
    global _lib
    if _lib is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        L.oracle_dijkstra.argtypes = [P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, P, P,
                                      ctypes.c_int32]
        L.oracle_dijkstra.restype = ctypes.c_int64
        L.oracle_dijkstra_iters.argtypes = [P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, P,
                                            P, ctypes.c_int32, ctypes.c_int32]
        L.oracle_dijkstra_iters.restype = ctypes.c_int64
        L.oracle_dijkstra_every_source.argtypes = [P, ctypes.c_int64, ctypes.c_int32, P, P]
        L.oracle_dijkstra_every_source.restype = ctypes.c_int
        L.oracle_floyd_warshall.argtypes = [P, ctypes.c_int64, ctypes.c_int32, P]
        L.oracle_floyd_warshall.restype = ctypes.c_int
        L.oracle_bellman_ford.argtypes = [P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P]
        L.oracle_bellman_ford.restype = ctypes.c_int
        L.oracle_certificate.argtypes = [P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P, P,
                                         ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]
        L.oracle_certificate.restype = ctypes.c_int
        L.oracle_closed_form_pred.argtypes = [P, ctypes.c_int64, ctypes.c_int32, P, P,
                                              ctypes.c_int32]
        L.oracle_closed_form_pred.restype = ctypes.c_int
        L.oracle_edges_to_dense.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P,
                                            ctypes.c_int64]
        L.oracle_edges_to_dense.restype = ctypes.c_int64
        L.oracle_hops.argtypes = [P, P, ctypes.c_int32, P]
        L.oracle_hops.restype = ctypes.c_int
        L.oracle_label_correcting.argtypes = [P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, P,
                                              ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.oracle_label_correcting.restype = ctypes.c_int
        L.oracle_dijkstra_csr.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_int32, P, P]
        L.oracle_dijkstra_csr.restype = ctypes.c_int64
        L.oracle_certificate_csr.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_int32, P, P,
                                             ctypes.POINTER(ctypes.c_int64)]
        L.oracle_certificate_csr.restype = ctypes.c_int
        L.oracle_closed_form_pred_csr.argtypes = [P, P, P, ctypes.c_int32, P, P]
        L.oracle_closed_form_pred_csr.restype = ctypes.c_int
        _lib = L
    return _lib


def _mat(W):
    W = np.asarray(W)
    if W.dtype != np.int32 or W.ndim != 2 or W.strides[1] != 4 or W.strides[0] % 4:
        W = np.ascontiguousarray(W, dtype=np.int32)
    return W, W.strides[0] // 4


def _threads(t):
    return t or max(1, min(16, os.cpu_count() or 1))


def dijkstra_every_source(Ws):
    """Algorithm 1 from every source of each matrix in Ws ([count, n, n] int32):
    returns (dist, pred), each [count, n (source), n]."""
    Ws = np.ascontiguousarray(Ws, np.int32)
    count, n, _ = Ws.shape
    dist = np.empty((count, n, n), np.int32)
    pred = np.empty((count, n, n), np.int32)
    if lib().oracle_dijkstra_every_source(Ws.ctypes.data, count, n, dist.ctypes.data, pred.ctypes.data) != 0:
        raise ValueError("bad arguments")
    return dist, pred


def dijkstra(W, src, early_exit=True, with_order=False):
    """Algorithm 1: returns (dist, pred[, order], relaxed_rows)."""
    W, ld = _mat(W)
    n = W.shape[0]
    dist = np.empty(n, np.int32)
    pred = np.empty(n, np.int32)
    order = np.empty(n, np.int32) if with_order else None
    r = lib().oracle_dijkstra(W.ctypes.data, ld, n, src, dist.ctypes.data, pred.ctypes.data,
                              order.ctypes.data if with_order else None, int(bool(early_exit)))
    if r < 0:
        raise ValueError("oracle_dijkstra rejected the arguments")
    if with_order:
        return dist, pred, order, int(r)
    return dist, pred, int(r)


def dijkstra_prefix(W, src, iters):
    """The first `iters` iterations of Algorithm 1 (a timing sample); returns rows relaxed."""
    W, ld = _mat(W)
    n = W.shape[0]
    dist = np.empty(n, np.int32)
    pred = np.empty(n, np.int32)
    r = lib().oracle_dijkstra_iters(W.ctypes.data, ld, n, src, dist.ctypes.data, pred.ctypes.data,
                                    None, 1, int(iters))
    if r < 0:
        raise ValueError("oracle_dijkstra_iters rejected the arguments")
    return int(r)


def floyd_warshall(W):
    W, ld = _mat(W)
    n = W.shape[0]
    D = np.empty((n, n), np.int64)
    if lib().oracle_floyd_warshall(W.ctypes.data, ld, n, D.ctypes.data) != 0:
        raise ValueError("bad arguments")
    return D


def bellman_ford(W, src):
    W, ld = _mat(W)
    n = W.shape[0]
    d = np.empty(n, np.int64)
    if lib().oracle_bellman_ford(W.ctypes.data, ld, n, src, d.ctypes.data) != 0:
        raise ValueError("bad arguments")
    return d


def certificate(W, src, dist, pred, threads=None):
    """Returns (code, where); code 0 means (dist, pred) is a valid shortest-path tree."""
    W, ld = _mat(W)
    dist = np.ascontiguousarray(dist, np.int32)
    pred = np.ascontiguousarray(pred, np.int32)
    where = ctypes.c_int64(-1)
    code = lib().oracle_certificate(W.ctypes.data, ld, W.shape[0], src, dist.ctypes.data,
                                    pred.ctypes.data, _threads(threads), ctypes.byref(where))
    if code < 0:
        raise ValueError("bad arguments")
    return code, int(where.value)


def closed_form_pred(W, dist, threads=None):
    W, ld = _mat(W)
    dist = np.ascontiguousarray(dist, np.int32)
    pred = np.empty(W.shape[0], np.int32)
    if lib().oracle_closed_form_pred(W.ctypes.data, ld, W.shape[0], dist.ctypes.data,
                                     pred.ctypes.data, _threads(threads)) != 0:
        raise ValueError("bad arguments")
    return pred


def edges_to_dense(eu, ev, ew, n, directed=False):
    """The edge list written into an n x n matrix; returns (W, skipped edges)."""
    eu = np.ascontiguousarray(eu, np.int32)
    ev = np.ascontiguousarray(ev, np.int32)
    ew = np.ascontiguousarray(ew, np.int32)
    W = np.empty((n, n), np.int32)
    bad = lib().oracle_edges_to_dense(eu.ctypes.data, ev.ctypes.data, ew.ctypes.data, eu.size, n,
                                      int(bool(directed)), W.ctypes.data, n)
    if bad < 0:
        raise ValueError("bad arguments")
    return W, int(bad)


def hops(pred, dist):
    pred = np.ascontiguousarray(pred, np.int32)
    dist = np.ascontiguousarray(dist, np.int32)
    h = np.empty(pred.size, np.int32)
    if lib().oracle_hops(pred.ctypes.data, dist.ctypes.data, pred.size, h.ctypes.data) != 0:
        raise ValueError("bad arguments")
    return h


def label_correcting(W, src):
    """Synchronous label-correcting sweeps (the paper's CUDA method): returns
    (dist, sweeps, rows relaxed)."""
    W, ld = _mat(W)
    n = W.shape[0]
    dist = np.empty(n, np.int32)
    sw, rows = ctypes.c_int64(), ctypes.c_int64()
    if lib().oracle_label_correcting(W.ctypes.data, ld, n, src, dist.ctypes.data, ctypes.byref(sw),
                                     ctypes.byref(rows)) != 0:
        raise ValueError("bad arguments")
    return dist, int(sw.value), int(rows.value)


def _csr(row_ptr, col, w):
    return (np.ascontiguousarray(row_ptr, np.int64), np.ascontiguousarray(col, np.int32),
            np.ascontiguousarray(w, np.int32))


def dijkstra_csr(row_ptr, col, w, src):
    """Algorithm 1 over adjacency lists: returns (dist, pred, relaxed_rows)."""
    row_ptr, col, w = _csr(row_ptr, col, w)
    n = row_ptr.size - 1
    dist = np.empty(n, np.int32)
    pred = np.empty(n, np.int32)
    r = lib().oracle_dijkstra_csr(row_ptr.ctypes.data, col.ctypes.data, w.ctypes.data, n, src,
                                  dist.ctypes.data, pred.ctypes.data)
    if r < 0:
        raise ValueError("bad arguments")
    return dist, pred, int(r)


def certificate_csr(row_ptr, col, w, src, dist, pred):
    row_ptr, col, w = _csr(row_ptr, col, w)
    dist = np.ascontiguousarray(dist, np.int32)
    pred = np.ascontiguousarray(pred, np.int32)
    where = ctypes.c_int64(-1)
    code = lib().oracle_certificate_csr(row_ptr.ctypes.data, col.ctypes.data, w.ctypes.data, row_ptr.size - 1,
                                        src, dist.ctypes.data, pred.ctypes.data, ctypes.byref(where))
    if code < 0:
        raise ValueError("bad arguments")
    return code, int(where.value)


def closed_form_pred_csr(row_ptr, col, w, dist):
    row_ptr, col, w = _csr(row_ptr, col, w)
    dist = np.ascontiguousarray(dist, np.int32)
    pred = np.empty(row_ptr.size - 1, np.int32)
    if lib().oracle_closed_form_pred_csr(row_ptr.ctypes.data, col.ctypes.data, w.ctypes.data,
                                         row_ptr.size - 1, dist.ctypes.data, pred.ctypes.data) != 0:
        raise ValueError("bad arguments")
    return pred


def edges_to_csr(eu, ev, ew, n, directed=False):
    """Adjacency lists of an edge list, in edge order (an undirected edge gives
    u -> v then v -> u); edges with an endpoint outside [0, n) are dropped.
    Plain numpy bookkeeping; duplicates and self-loops are kept (the CSR
    functions ignore self-loops and take a pair's smallest weight)."""
    eu = np.asarray(eu, np.int64)
    ev = np.asarray(ev, np.int64)
    ew = np.asarray(ew, np.int32)
    ok = (eu >= 0) & (eu < n) & (ev >= 0) & (ev < n)
    eu, ev, ew = eu[ok], ev[ok], ew[ok]
    if not directed:
        eu, ev, ew = np.concatenate([eu, ev]), np.concatenate([ev, eu]), np.concatenate([ew, ew])
    order = np.argsort(eu, kind="stable")
    row_ptr = np.zeros(n + 1, np.int64)
    np.add.at(row_ptr, eu + 1, 1)
    return np.cumsum(row_ptr), ev[order].astype(np.int32), ew[order]
