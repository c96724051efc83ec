"""Dense-matrix Dijkstra (Algorithm 1 of arXiv 2504.03667) on MI355X (gfx950).

The compute path is libsssp.so (HIP kernels behind the C ABI in include/sssp.h);
this package only binds it.  See sssp.py.
"""
from .sssp import (INF, SSSP_FLAG_GRID, SSSP_FLAG_LITERAL, SSSP_FLAG_SINGLE, SSSP_STAT_BARRIERS,
                   SSSP_STAT_FALLBACKS, SSSP_STAT_ROUNDS, SSSP_STAT_SETTLED,
                   SSSP_STATUS_NEG_WEIGHT, SSSP_STATUS_TIMEOUT, SSSP_STATUS_ZERO_FALLBACK,
                   SsspError, lib, solve, sssp_dense_solve, sssp_dense_solve_batched,
                   sssp_dense_solve_ex, sssp_last_status, sssp_last_trace)

__all__ = ["INF", "SSSP_FLAG_GRID", "SSSP_FLAG_LITERAL", "SSSP_FLAG_SINGLE", "SSSP_STAT_BARRIERS",
           "SSSP_STAT_FALLBACKS", "SSSP_STAT_ROUNDS", "SSSP_STAT_SETTLED",
           "SSSP_STATUS_NEG_WEIGHT", "SSSP_STATUS_TIMEOUT", "SSSP_STATUS_ZERO_FALLBACK",
           "SsspError", "lib", "solve", "sssp_dense_solve", "sssp_dense_solve_batched",
           "sssp_dense_solve_ex", "sssp_last_status", "sssp_last_trace"]
