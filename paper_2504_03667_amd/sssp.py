"""Python binding of libsssp (include/sssp.h): argument marshalling only.

Every function here forwards torch device tensors (int32, on the current HIP
device) and the current stream to the C ABI of the same name; all work runs in
the HIP kernels.  There is no CPU fallback: if the library cannot be loaded the
functions raise.
"""
import ctypes
import os

import torch  # loaded first so libsssp binds to the HIP runtime torch already uses

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "libsssp.so")

SSSP_OK = 0
SSSP_EINVAL = -1
SSSP_EDEVICE = -2
SSSP_ENOMEM = -3
SSSP_EAGAIN = -4
SSSP_ENOGRAPH = -5
SSSP_ETIMEDOUT = -6
SSSP_EUNSUPPORTED = -7

SSSP_STATUS_TIMEOUT = 1
SSSP_STATUS_NEG_WEIGHT = 2
SSSP_STATUS_ZERO_FALLBACK = 4

SSSP_FLAG_LITERAL = 1
SSSP_FLAG_SINGLE = 2
SSSP_FLAG_GRID = 4
SSSP_FLAG_COMPACT = 8
SSSP_FLAG_LABEL_CORRECTING = 16

SSSP_STAT_ROUNDS, SSSP_STAT_SETTLED, SSSP_STAT_FALLBACKS, SSSP_STAT_BARRIERS = range(4)

INF = 0x7FFFFFFF


class SsspError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (code %d)" % (msg, code))
        self.code = code


class sssp_tuning(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("single_max_n", ctypes.c_int32), ("gang_columns", ctypes.c_int32),
                ("group_sources", ctypes.c_int32), ("group_columns", ctypes.c_int32),
                ("balance", ctypes.c_int32), ("reserved", ctypes.c_int32 * 1)]


class sssp_plan_info(ctypes.Structure):
    _fields_ = [("threads", ctypes.c_int32), ("workgroups", ctypes.c_int32),
                ("single_max_n", ctypes.c_int32), ("gang_columns", ctypes.c_int32),
                ("max_parts", ctypes.c_int32), ("candidates", ctypes.c_int32),
                ("compact_graphs", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("compact_bytes", ctypes.c_int64), ("tuned_ms", ctypes.c_double),
                ("build_ms", ctypes.c_double), ("lc_instances", ctypes.c_int32),
                ("lc_candidates", ctypes.c_int32), ("group_sources", ctypes.c_int32),
                ("group_columns", ctypes.c_int32), ("group_items", ctypes.c_int32),
                ("group_candidates", ctypes.c_int32)]


class sssp_instance(ctypes.Structure):
    _fields_ = [("W", ctypes.c_void_p), ("ld", ctypes.c_int64), ("n", ctypes.c_int32),
                ("src", ctypes.c_int32), ("dist", ctypes.c_void_p), ("pred", ctypes.c_void_p)]


class sssp_layout_entry(ctypes.Structure):
    _fields_ = [("instance", ctypes.c_int32), ("parts", ctypes.c_int32), ("columns", ctypes.c_int32),
                ("method", ctypes.c_int32), ("scratch_offset", ctypes.c_int64), ("scratch_bytes", ctypes.c_int64)]


class sssp_server_config(ctypes.Structure):
    _fields_ = [("workgroups", ctypes.c_int32), ("ring_slots", ctypes.c_int32),
                ("max_inflight", ctypes.c_int32), ("single_max_n", ctypes.c_int32),
                ("gang_columns", ctypes.c_int32), ("watchdog_ms", ctypes.c_int32),
                ("scratch_bytes", ctypes.c_int64), ("max_pending", ctypes.c_int64),
                ("idle_park_ms", ctypes.c_int32), ("lc_rounds", ctypes.c_int32),
                ("lc_gang_columns", ctypes.c_int32), ("lc_model", ctypes.c_int32),
                ("idle_gang_columns", ctypes.c_int32), ("idle_wait_us", ctypes.c_int32),
                ("busy_gang_columns", ctypes.c_int32), ("busy_queue", ctypes.c_int32)]


class sssp_query_info(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32), ("parts", ctypes.c_int32),
                ("rounds", ctypes.c_int32), ("settled", ctypes.c_int64),
                ("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64), ("method", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class sssp_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("running", ctypes.c_int64),
                ("pending", ctypes.c_int64), ("kernel_launches", ctypes.c_int64),
                ("workgroups", ctypes.c_int32), ("failed", ctypes.c_int32)]


SSSP_QUERY_PENDING, SSSP_QUERY_RUNNING, SSSP_QUERY_DONE = 0, 1, 2

_lib = None


def lib():
    """The loaded libsssp.so; builds it in-tree if it is not there yet."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO):
            from . import build as _b
            _b.build()
        _lib = _declare(ctypes.CDLL(SO))
    return _lib


def use_library(path):
    """Makes every call of this module go to the library at `path` (a build of the
    same sources, e.g. the barrier-stress test build); returns the previous one.
    use_library(None) restores libsssp.so."""
    global _lib
    prev = _lib
    _lib = None if path is None else _declare(ctypes.CDLL(path))
    return prev


def _declare(L):
    """Argument and result types of the C ABI on a loaded library."""
    P, I32, I64, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    L.sssp_version.restype = ctypes.c_int
    L.sssp_last_error.restype = ctypes.c_char_p
    L.sssp_strerror.argtypes = [ctypes.c_int]
    L.sssp_strerror.restype = ctypes.c_char_p
    L.sssp_dense_solve.argtypes = [P, I32, I32, P, P, P]
    L.sssp_dense_solve_ex.argtypes = [P, I64, I32, I32, P, P, U32, ctypes.POINTER(sssp_tuning), P]
    L.sssp_last_status.argtypes = [P, ctypes.POINTER(I32), ctypes.POINTER(I64)]
    L.sssp_dense_solve_noalloc.argtypes = [P, I64, I32, I32, P, P, U32, P, P]
    L.sssp_dense_solve_noalloc.restype = ctypes.c_int
    L.sssp_stream_release.argtypes = [P]
    L.sssp_stream_release.restype = ctypes.c_int
    L.sssp_release_all.argtypes = []
    L.sssp_release_all.restype = ctypes.c_int
    L.sssp_scratch_bytes.argtypes = [ctypes.POINTER(I64)]
    L.sssp_scratch_bytes.restype = ctypes.c_int
    L.sssp_dense_solve_batched.argtypes = [ctypes.POINTER(sssp_instance), I32, U32,
                                           ctypes.POINTER(sssp_tuning), P]
    L.sssp_last_trace.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I32), I32,
                                  ctypes.POINTER(I32)]
    L.sssp_last_trace.restype = ctypes.c_int
    L.sssp_batch_max_n.restype = I32
    L.sssp_batch_layout.argtypes = [ctypes.POINTER(sssp_instance), I32, U32, I32, I32, I32,
                                    ctypes.POINTER(sssp_layout_entry), ctypes.POINTER(I64)]
    L.sssp_batch_plan_create.argtypes = [ctypes.POINTER(sssp_instance), I32, U32,
                                         ctypes.POINTER(sssp_tuning), P, ctypes.POINTER(P)]
    L.sssp_batch_plan_launch.argtypes = [P, P]
    L.sssp_batch_plan_info.argtypes = [P, ctypes.POINTER(sssp_plan_info)]
    L.sssp_batch_plan_status.argtypes = [P, P, ctypes.POINTER(I32), ctypes.POINTER(I64)]
    L.sssp_batch_plan_destroy.argtypes = [P]
    L.sssp_dense_validate.argtypes = [P, I64, I32, ctypes.POINTER(I32), ctypes.POINTER(I32), P]
    L.sssp_server_add_graph_ex.argtypes = [P, P, I64, I32, U32, ctypes.POINTER(I32)]
    L.sssp_server_graph_elem.argtypes = [P, I32, ctypes.POINTER(I32)]
    L.sssp_edges_to_dense.argtypes = [P, P, P, I64, I32, I32, P, I64, ctypes.POINTER(I64), P]
    L.sssp_hops.argtypes = [P, P, I32, P, P]
    L.sssp_paths.argtypes = [P, P, I32, P, I32, P, P, P]
    L.sssp_single_max_n.restype = I32
    L.sssp_stream_read.argtypes = [P, I64, I64, P, P]
    L.sssp_edges_to_csr.argtypes = [P, P, P, I64, I32, I32, P, P, P, ctypes.POINTER(I64),
                                    ctypes.POINTER(I64), P]
    L.sssp_csr_solve.argtypes = [P, P, P, I32, I32, P, P, ctypes.POINTER(sssp_tuning), P]
    L.sssp_csr_grid.argtypes = [I32, ctypes.POINTER(sssp_tuning), P, ctypes.POINTER(I32), ctypes.POINTER(I32),
                                ctypes.POINTER(I32)]
    L.sssp_server_now_ns.restype = I64
    L.sssp_server_shape.argtypes = [ctypes.POINTER(sssp_server_config), I32, I32, I32, I32, I32, I32,
                                    ctypes.POINTER(I32), ctypes.POINTER(I32), ctypes.POINTER(I64)]
    L.sssp_server_create.argtypes = [ctypes.POINTER(sssp_server_config), ctypes.POINTER(P)]
    L.sssp_server_add_graph.argtypes = [P, P, I64, I32, ctypes.POINTER(I32)]
    L.sssp_server_submit.argtypes = [P, I32, I32, P, P, ctypes.POINTER(ctypes.c_uint64)]
    L.sssp_server_poll.argtypes = [P, ctypes.POINTER(ctypes.c_uint64), I32, ctypes.POINTER(I32)]
    L.sssp_server_wait.argtypes = [P, ctypes.c_uint64, I64]
    L.sssp_server_query_info.argtypes = [P, ctypes.c_uint64, ctypes.POINTER(sssp_query_info)]
    L.sssp_server_get_stats.argtypes = [P, ctypes.POINTER(sssp_server_stats)]
    L.sssp_server_destroy.argtypes = [P]
    for name in ("sssp_dense_solve", "sssp_dense_solve_ex", "sssp_last_status",
                 "sssp_dense_solve_batched", "sssp_server_create", "sssp_server_add_graph",
                 "sssp_server_submit", "sssp_server_poll", "sssp_server_wait",
                 "sssp_server_query_info", "sssp_server_get_stats", "sssp_server_destroy"):
        getattr(L, name).restype = ctypes.c_int
    return L


def _check(rc):
    if rc != SSSP_OK:
        msg = lib().sssp_last_error().decode(errors="replace")
        raise SsspError(rc, msg or lib().sssp_strerror(rc).decode())
    return rc


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t, what):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int32:
        raise TypeError("%s must be an int32 tensor on the GPU" % what)
    return ctypes.c_void_p(t.data_ptr())


def _tuning(threads=0, workgroups=0, single_max_n=0, gang_columns=0, group_sources=0, group_columns=0,
            balance=0):
    if not (threads or workgroups or single_max_n or gang_columns or group_sources or group_columns or balance):
        return None
    t = sssp_tuning()
    t.threads, t.workgroups = threads, workgroups
    t.single_max_n, t.gang_columns = single_max_n, gang_columns
    t.group_sources, t.group_columns = group_sources, group_columns
    t.balance = balance
    return ctypes.byref(t)


def sssp_dense_solve(W, n, src, dist, pred, stream=None):
    """sssp_dense_solve: W is an int32 [n, n] contiguous device tensor."""
    if W.dim() != 2 or W.shape[0] != n or W.shape[1] != n or not W.is_contiguous():
        raise ValueError("W must be a contiguous [n, n] tensor")
    return _check(lib().sssp_dense_solve(_ptr(W, "W"), n, src, _ptr(dist, "dist"),
                                         _ptr(pred, "pred"), _stream(stream)))


def sssp_dense_solve_ex(W, ld, n, src, dist, pred, flags=0, threads=0, workgroups=0, stream=None, balance=0):
    """sssp_dense_solve_ex: W is an int32 device tensor holding n rows of stride ld."""
    # W may be a row-strided view (e.g. big[:, :n]): check the storage behind it
    avail = W.untyped_storage().nbytes() // 4 - W.storage_offset()
    if n < 1 or avail < (n - 1) * ld + n or (W.dim() == 2 and W.stride(1) != 1):
        raise ValueError("W is too small for n rows of stride ld, or its rows are not contiguous")
    return _check(lib().sssp_dense_solve_ex(_ptr(W, "W"), ld, n, src, _ptr(dist, "dist"),
                                            _ptr(pred, "pred"), flags,
                                            _tuning(threads, workgroups, balance=balance), _stream(stream)))


SSSP_NOALLOC_SCRATCH_BYTES = 8 << 20
SSSP_NOALLOC_MAX_N = 262144


def sssp_dense_solve_noalloc(W, ld, n, src, dist, pred, flags=0, status=None, stream=None):
    """sssp_dense_solve_noalloc: as sssp_dense_solve_ex with the library's scratch in a
    fixed per-GPU array (nothing allocated); `status`, an int32 device tensor of one
    element or None, receives the solve's status bits in stream order."""
    avail = W.untyped_storage().nbytes() // 4 - W.storage_offset()
    if n < 1 or avail < (n - 1) * ld + n or (W.dim() == 2 and W.stride(1) != 1):
        raise ValueError("W is too small for n rows of stride ld, or its rows are not contiguous")
    st = None if status is None else _ptr(status, "status")
    return _check(lib().sssp_dense_solve_noalloc(_ptr(W, "W"), ld, n, src, _ptr(dist, "dist"),
                                                 _ptr(pred, "pred"), flags, st, _stream(stream)))


def sssp_stream_release(stream=None):
    """Frees the library scratch held for `stream` (default: the current stream) after
    waiting for it; a stream about to be destroyed leaves nothing behind."""
    return _check(lib().sssp_stream_release(_stream(stream)))


def sssp_release_all():
    """Frees every scratch block the library holds (all streams, all devices)."""
    return _check(lib().sssp_release_all())


def sssp_scratch_bytes():
    """Device bytes of library scratch currently held."""
    b = ctypes.c_int64(0)
    _check(lib().sssp_scratch_bytes(ctypes.byref(b)))
    return b.value


def sssp_last_status(stream=None):
    """Synchronises the stream; returns (status bits, [rounds, settled, fallbacks, barriers])."""
    st = ctypes.c_int32(0)
    stats = (ctypes.c_int64 * 4)()
    _check(lib().sssp_last_status(_stream(stream), ctypes.byref(st), stats))
    return st.value, list(stats)


def sssp_last_trace(stream=None, cap=257):
    """Synchronises the stream; returns [(t_ns, rows)] per round of the last solve, then (t_end, -1)."""
    t = (ctypes.c_int64 * cap)()
    r = (ctypes.c_int32 * cap)()
    cnt = ctypes.c_int32(0)
    _check(lib().sssp_last_trace(_stream(stream), t, r, cap, ctypes.byref(cnt)))
    k = min(cnt.value + 1, cap)
    return [(t[i], r[i]) for i in range(k)]


def make_instances(items):
    """items: iterable of (W, src, dist, pred) with W an int32 [n, ld] device tensor."""
    items = list(items)
    arr = (sssp_instance * max(1, len(items)))()
    for i, (W, src, dist, pred) in enumerate(items):
        n = W.shape[0]
        if dist.numel() < n or pred.numel() < n:
            raise ValueError("dist/pred too small for instance %d" % i)
        arr[i].W = _ptr(W, "W").value
        arr[i].ld = W.stride(0)
        arr[i].n = n
        arr[i].src = src
        arr[i].dist = _ptr(dist, "dist").value
        arr[i].pred = _ptr(pred, "pred").value
    return arr, len(items)


def sssp_dense_solve_batched(items, flags=0, threads=0, workgroups=0, stream=None):
    """sssp_dense_solve_batched over (W, src, dist, pred) tuples, one launch."""
    arr, count = make_instances(items)
    return _check(lib().sssp_dense_solve_batched(arr, count, flags, _tuning(threads, workgroups),
                                                 _stream(stream)))


def sssp_batch_layout(instances, flags=0, single_max_n=0, gang_columns=0, max_parts=0):
    """sssp_batch_layout on an array of sssp_instance (host only: the buffers are
    not read).  Returns ([entry dicts in launch order], arena bytes)."""
    count = len(instances)
    arr = (sssp_instance * max(1, count))(*instances)
    out = (sssp_layout_entry * max(1, count))()
    arena = ctypes.c_int64(0)
    _check(lib().sssp_batch_layout(arr, count, flags, single_max_n, gang_columns, max_parts, out,
                                   ctypes.byref(arena)))
    return [{k: getattr(out[i], k) for k, _ in sssp_layout_entry._fields_} for i in range(count)], arena.value


def sssp_batch_max_n():
    return lib().sssp_batch_max_n()


def sssp_stream_read(buf, nbytes=None, chunk_bytes=0, fold=None, stream=None):
    """sssp_stream_read: one plain read of a device tensor's bytes (a bandwidth probe);
    `fold`, an int32 tensor of one element on the GPU, receives the xor of the words read."""
    if not isinstance(buf, torch.Tensor) or not buf.is_cuda:
        raise TypeError("buf must be a tensor on the GPU")
    nbytes = buf.numel() * buf.element_size() if nbytes is None else nbytes
    f = None if fold is None else _ptr(fold, "fold")
    _check(lib().sssp_stream_read(ctypes.c_void_p(buf.data_ptr()), nbytes, chunk_bytes, f, _stream(stream)))


def sssp_single_max_n():
    return lib().sssp_single_max_n()


def sssp_dense_validate(W, ld, n, stream=None):
    """(min weight, max finite weight) of an int32 device matrix; synchronous."""
    mn, mx = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().sssp_dense_validate(_ptr(W, "W"), ld, n, ctypes.byref(mn), ctypes.byref(mx), _stream(stream)))
    return mn.value, mx.value


def sssp_batch_plan_create(items, flags=0, threads=0, workgroups=0, single_max_n=0, gang_columns=0,
                           group_sources=0, group_columns=0, stream=None):
    arr, count = make_instances(items)
    h = ctypes.c_void_p()
    _check(lib().sssp_batch_plan_create(arr, count, flags, _tuning(threads, workgroups, single_max_n,
                                                                    gang_columns, group_sources, group_columns),
                                        _stream(stream), ctypes.byref(h)))
    return h


def sssp_batch_plan_launch(h, stream=None):
    return _check(lib().sssp_batch_plan_launch(h, _stream(stream)))


def sssp_batch_plan_info(h):
    i = sssp_plan_info()
    _check(lib().sssp_batch_plan_info(h, ctypes.byref(i)))
    return {k: getattr(i, k) for k, _ in sssp_plan_info._fields_}


def sssp_batch_plan_status(h, stream=None):
    st = ctypes.c_int32(0)
    stats = (ctypes.c_int64 * 4)()
    _check(lib().sssp_batch_plan_status(h, _stream(stream), ctypes.byref(st), stats))
    return st.value, list(stats)


def sssp_batch_plan_destroy(h):
    return _check(lib().sssp_batch_plan_destroy(h))


class BatchPlan:
    """Owns an sssp_batch_plan and keeps the tensors of its instances alive."""

    def __init__(self, items, flags=0, **tuning):
        self.items = list(items)
        self.h = sssp_batch_plan_create(self.items, flags, **tuning)

    def launch(self, stream=None):
        sssp_batch_plan_launch(self.h, stream)

    def info(self):
        return sssp_batch_plan_info(self.h)

    def status(self, stream=None):
        return sssp_batch_plan_status(self.h, stream)

    def close(self):
        if self.h is not None:
            sssp_batch_plan_destroy(self.h)
            self.h = None
            self.items = []

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _ptr64(t, what):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int64:
        raise TypeError("%s must be an int64 tensor on the GPU" % what)
    return ctypes.c_void_p(t.data_ptr())


def sssp_edges_to_dense(eu, ev, ew, n, W, ld=None, directed=False, stream=None):
    """Writes the edge list (int32 device tensors) into W; returns the number of skipped edges."""
    m = eu.numel()
    if ev.numel() != m or ew.numel() != m:
        raise ValueError("edge arrays differ in length")
    bad = ctypes.c_int64(0)
    nul = ctypes.c_void_p(None)
    _check(lib().sssp_edges_to_dense(_ptr(eu, "eu") if m else nul, _ptr(ev, "ev") if m else nul,
                                     _ptr(ew, "ew") if m else nul, m, n, int(bool(directed)), _ptr(W, "W"),
                                     W.stride(0) if ld is None else ld, ctypes.byref(bad), _stream(stream)))
    return bad.value


def sssp_hops(pred, dist, hops, stream=None):
    return _check(lib().sssp_hops(_ptr(pred, "pred"), _ptr(dist, "dist"), pred.numel(), _ptr(hops, "hops"),
                                  _stream(stream)))


def sssp_paths(pred, hops, targets, offsets, out, stream=None):
    return _check(lib().sssp_paths(_ptr(pred, "pred"), _ptr(hops, "hops"), pred.numel(), _ptr(targets, "targets"),
                                   targets.numel(), _ptr64(offsets, "offsets"), _ptr(out, "out"),
                                   _stream(stream)))


def paths(pred, dist, targets):
    """Shortest paths source ... t for each target, as a list of int32 device tensors."""
    n = pred.numel()
    hops = torch.empty(n, dtype=torch.int32, device=pred.device)
    sssp_hops(pred, dist, hops)
    t = torch.as_tensor(targets, dtype=torch.int32, device=pred.device)
    lens = torch.where(hops[t.long()] >= 0, hops[t.long()] + 1, torch.zeros_like(t)).to(torch.int64)
    offsets = torch.cumsum(lens, 0) - lens
    out = torch.full((int(lens.sum().item()) + 1,), -1, dtype=torch.int32, device=pred.device)
    sssp_paths(pred, hops, t, offsets, out)
    o, l_ = offsets.tolist(), lens.tolist()
    return [out[o[i]:o[i] + l_[i]] for i in range(len(o))]


# ---- convenience wrappers (allocate outputs, return tensors) ----

def solve(W, src, flags=0, threads=0, workgroups=0, stream=None, balance=0):
    """Solve from `src` on the int32 [n, ld] device tensor W; returns (dist, pred) tensors."""
    n = W.shape[0]
    dist = torch.empty(n, dtype=torch.int32, device=W.device)
    pred = torch.empty(n, dtype=torch.int32, device=W.device)
    sssp_dense_solve_ex(W, W.stride(0), n, src, dist, pred, flags, threads, workgroups, stream, balance)
    return dist, pred


# ---- graphs stored as adjacency lists (CSR) ----

def _ptr_t(t, dtype, what):
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise TypeError("%s must be a contiguous %s tensor on the GPU" % (what, dtype))
    return ctypes.c_void_p(t.data_ptr())


def sssp_edges_to_csr(eu, ev, ew, n, directed, row_ptr, col, w, stream=None):
    """sssp_edges_to_csr: returns (edges stored, edges skipped)."""
    m = eu.numel()
    if ev.numel() != m or ew.numel() != m:
        raise ValueError("eu, ev, ew must have the same length")
    cap = m if directed else 2 * m
    if row_ptr.numel() < n + 1 or col.numel() < cap or w.numel() < cap:
        raise ValueError("row_ptr needs n + 1 entries, col and w %d" % cap)
    m_out, bad = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().sssp_edges_to_csr(_ptr_t(eu, torch.int32, "eu"), _ptr_t(ev, torch.int32, "ev"),
                                   _ptr_t(ew, torch.int32, "ew"), m, n, int(bool(directed)),
                                   _ptr_t(row_ptr, torch.int64, "row_ptr"), _ptr_t(col, torch.int32, "col"),
                                   _ptr_t(w, torch.int32, "w"), ctypes.byref(m_out), ctypes.byref(bad),
                                   _stream(stream)))
    return m_out.value, bad.value


def sssp_csr_solve(row_ptr, col, w, n, src, dist, pred, workgroups=0, stream=None):
    if row_ptr.numel() < n + 1 or dist.numel() < n or pred.numel() < n:
        raise ValueError("row_ptr needs n + 1 entries, dist and pred n")
    return _check(lib().sssp_csr_solve(_ptr_t(row_ptr, torch.int64, "row_ptr"), _ptr_t(col, torch.int32, "col"),
                                       _ptr_t(w, torch.int32, "w"), n, src, _ptr(dist, "dist"),
                                       _ptr(pred, "pred"), _tuning(0, workgroups), _stream(stream)))


def sssp_csr_grid(n, workgroups=0, stream=None):
    """(workgroups, co-resident workgroups per CU, CUs) of a CSR solve of n vertices."""
    g, pc, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().sssp_csr_grid(n, _tuning(0, workgroups), _stream(stream), ctypes.byref(g), ctypes.byref(pc),
                               ctypes.byref(c)))
    return g.value, pc.value, c.value


def csr_from_edges(eu, ev, ew, n, directed=False, stream=None):
    """Edge list (device int32 tensors) -> (row_ptr, col, w) device tensors, skipped edges."""
    cap = eu.numel() if directed else 2 * eu.numel()
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=eu.device)
    col = torch.empty(max(1, cap), dtype=torch.int32, device=eu.device)
    w = torch.empty(max(1, cap), dtype=torch.int32, device=eu.device)
    m_out, bad = sssp_edges_to_csr(eu, ev, ew, n, directed, row_ptr, col, w, stream)
    return row_ptr, col[:max(1, m_out)], w[:max(1, m_out)], bad


def csr_solve(row_ptr, col, w, src, workgroups=0, stream=None):
    """Solve from src on a CSR graph; returns (dist, pred) tensors."""
    n = row_ptr.numel() - 1
    dist = torch.empty(n, dtype=torch.int32, device=row_ptr.device)
    pred = torch.empty(n, dtype=torch.int32, device=row_ptr.device)
    sssp_csr_solve(row_ptr, col, w, n, src, dist, pred, workgroups, stream)
    return dist, pred


# ---- serving (sssp_server_*) ----

def sssp_server_now_ns():
    return lib().sssp_server_now_ns()


def sssp_server_shape(workgroups, n, method=0, busy=0, waiting=0, elem=4, **cfg):
    """sssp_server_shape (host only): (parts, columns, scratch_bytes) of an n-vertex query
    on a graph stored with `elem` bytes per entry."""
    c = sssp_server_config()
    names = {f for f, _ in sssp_server_config._fields_} - {"reserved"}
    for k, v in cfg.items():
        if k not in names:
            raise TypeError("unknown server setting %r" % k)
        setattr(c, k, v)
    parts, cols, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check(lib().sssp_server_shape(ctypes.byref(c), workgroups, n, method, elem, busy, waiting, ctypes.byref(parts),
                                   ctypes.byref(cols), ctypes.byref(b)))
    return parts.value, cols.value, b.value


def sssp_server_create(**cfg):
    c = sssp_server_config()
    names = {f for f, _ in sssp_server_config._fields_} - {"reserved"}
    for k, v in cfg.items():
        if k not in names:
            raise TypeError("unknown server setting %r" % k)
        setattr(c, k, v)
    h = ctypes.c_void_p()
    _check(lib().sssp_server_create(ctypes.byref(c), ctypes.byref(h)))
    return h


def sssp_server_add_graph(h, W, ld, n):
    gid = ctypes.c_int32(-1)
    _check(lib().sssp_server_add_graph(h, _ptr(W, "W"), ld, n, ctypes.byref(gid)))
    return gid.value


def sssp_server_add_graph_ex(h, W, ld, n, flags=0):
    gid = ctypes.c_int32(-1)
    _check(lib().sssp_server_add_graph_ex(h, _ptr(W, "W"), ld, n, flags, ctypes.byref(gid)))
    return gid.value


def sssp_server_graph_elem(h, graph_id):
    e = ctypes.c_int32(0)
    _check(lib().sssp_server_graph_elem(h, graph_id, ctypes.byref(e)))
    return e.value


def sssp_server_submit(h, graph_id, src, dist, pred):
    t = ctypes.c_uint64(0)
    _check(lib().sssp_server_submit(h, graph_id, src, _ptr(dist, "dist"), _ptr(pred, "pred"),
                                    ctypes.byref(t)))
    return t.value


def sssp_server_poll(h, cap=4096):
    buf = (ctypes.c_uint64 * cap)()
    cnt = ctypes.c_int32(0)
    _check(lib().sssp_server_poll(h, buf, cap, ctypes.byref(cnt)))
    return list(buf[:cnt.value])


def sssp_server_wait(h, ticket, timeout_s=None):
    ns = -1 if timeout_s is None else int(timeout_s * 1e9)
    return _check(lib().sssp_server_wait(h, ticket, ns))


def sssp_server_query_info(h, ticket):
    i = sssp_query_info()
    _check(lib().sssp_server_query_info(h, ticket, ctypes.byref(i)))
    return {k: getattr(i, k) for k, _ in sssp_query_info._fields_}


def sssp_server_get_stats(h):
    s = sssp_server_stats()
    _check(lib().sssp_server_get_stats(h, ctypes.byref(s)))
    return {k: getattr(s, k) for k, _ in sssp_server_stats._fields_}


def sssp_server_destroy(h):
    return _check(lib().sssp_server_destroy(h))


class Server:
    """Owns an sssp_server and keeps the tensors it borrows alive while it needs them."""

    def __init__(self, **cfg):
        self.h = sssp_server_create(**cfg)
        self._graphs = []
        self._outs = {}

    def add_graph(self, W, flags=0):
        gid = sssp_server_add_graph_ex(self.h, W, W.stride(0), W.shape[0], flags)
        self._graphs.append(W)
        return gid

    def graph_elem(self, graph_id):
        return sssp_server_graph_elem(self.h, graph_id)

    def submit(self, graph_id, src, dist, pred):
        t = sssp_server_submit(self.h, graph_id, src, dist, pred)
        self._outs[t] = (dist, pred)
        return t

    def poll(self, cap=4096):
        done = sssp_server_poll(self.h, cap)
        for t in done:
            self._outs.pop(t, None)
        return done

    def wait(self, ticket, timeout_s=None):
        sssp_server_wait(self.h, ticket, timeout_s)

    def info(self, ticket):
        return sssp_server_query_info(self.h, ticket)

    def stats(self):
        return sssp_server_get_stats(self.h)

    def close(self):
        if self.h is not None:
            sssp_server_destroy(self.h)
            self.h = None
            self._outs.clear()
            self._graphs.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
