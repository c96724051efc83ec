"""Dense-matrix Dijkstra (Algorithm 1 of arXiv 2504.03667) on MI355X (gfx950).

The compute path is libsssp.so (HIP kernels behind the C ABI in include/sssp.h);
this package only binds it.  See sssp.py.
"""
from .sssp import (sssp_stream_release, sssp_release_all, sssp_scratch_bytes, sssp_dense_solve_noalloc, SSSP_NOALLOC_MAX_N, SSSP_NOALLOC_SCRATCH_BYTES, sssp_stream_read, sssp_server_shape, sssp_batch_layout, sssp_csr_grid, csr_from_edges, csr_solve, sssp_csr_solve, sssp_edges_to_csr, SSSP_FLAG_LABEL_CORRECTING, sssp_single_max_n, paths, sssp_edges_to_dense, sssp_hops, sssp_paths, BatchPlan, SSSP_FLAG_COMPACT, sssp_batch_max_n, sssp_batch_plan_create,
                   sssp_batch_plan_destroy, sssp_batch_plan_info, sssp_batch_plan_launch,
                   sssp_batch_plan_status, sssp_dense_validate, sssp_server_add_graph_ex,
                   sssp_server_graph_elem, Server, SSSP_QUERY_DONE, sssp_server_add_graph, sssp_server_create,
                   sssp_server_destroy, sssp_server_get_stats, sssp_server_now_ns, sssp_server_poll,
                   sssp_server_query_info, sssp_server_submit, sssp_server_wait,
                   INF, SSSP_FLAG_GRID, SSSP_FLAG_LITERAL, SSSP_FLAG_SINGLE, SSSP_STAT_BARRIERS,
                   SSSP_STAT_FALLBACKS, SSSP_STAT_ROUNDS, SSSP_STAT_SETTLED,
                   SSSP_STATUS_NEG_WEIGHT, SSSP_STATUS_TIMEOUT, SSSP_STATUS_ZERO_FALLBACK,
                   SsspError, lib, solve, sssp_dense_solve, sssp_dense_solve_batched,
                   sssp_dense_solve_ex, sssp_last_status, sssp_last_trace)

__all__ = ["sssp_stream_release", "sssp_release_all", "sssp_scratch_bytes", "sssp_dense_solve_noalloc", "SSSP_NOALLOC_MAX_N", "SSSP_NOALLOC_SCRATCH_BYTES", "sssp_stream_read", "sssp_server_shape", "sssp_batch_layout", "sssp_csr_grid", "csr_from_edges", "csr_solve", "sssp_csr_solve", "sssp_edges_to_csr", "SSSP_FLAG_LABEL_CORRECTING", "sssp_single_max_n", "paths", "sssp_edges_to_dense", "sssp_hops", "sssp_paths", "BatchPlan", "SSSP_FLAG_COMPACT", "sssp_batch_max_n", "sssp_batch_plan_create",
           "sssp_batch_plan_destroy", "sssp_batch_plan_info", "sssp_batch_plan_launch",
           "sssp_batch_plan_status", "sssp_dense_validate", "sssp_server_add_graph_ex",
           "sssp_server_graph_elem", "Server", "SSSP_QUERY_DONE", "sssp_server_add_graph", "sssp_server_create",
           "sssp_server_destroy", "sssp_server_get_stats", "sssp_server_now_ns", "sssp_server_poll",
           "sssp_server_query_info", "sssp_server_submit", "sssp_server_wait", "INF", "SSSP_FLAG_GRID", "SSSP_FLAG_LITERAL", "SSSP_FLAG_SINGLE", "SSSP_STAT_BARRIERS",
           "SSSP_STAT_FALLBACKS", "SSSP_STAT_ROUNDS", "SSSP_STAT_SETTLED",
           "SSSP_STATUS_NEG_WEIGHT", "SSSP_STATUS_TIMEOUT", "SSSP_STATUS_ZERO_FALLBACK",
           "SsspError", "lib", "solve", "sssp_dense_solve", "sssp_dense_solve_batched",
           "sssp_dense_solve_ex", "sssp_last_status", "sssp_last_trace"]
