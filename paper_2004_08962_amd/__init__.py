"""MI355X-native HICU hot path: HIP kernels for gfx950 behind a C ABI
(include/hicu.h, libhicu.so), with a thin torch binding.

HICU (Zhao, Potter, Ahmad) reconstructs unobserved multi-coil k-space by
alternating a nullspace estimate of the multi-level Hankel matrix with
gradient steps and exact line search on ||H(x) Q||_F^2 (Algorithm 1).
"""
from ._lib import HicuError, load, LIB_PATH
from .api import (geom, num_taps, gram, set_gram_route, nullspace, nullspace_rsvd, sketch, jl_compress, workspace_bytes, set_filter_group_budget, filter_group,
                  objective_grad,
                  line_search, update, solve, solve_workspace_bytes, time_average_init, profile_begin,
                  profile_end)

__all__ = ["HicuError", "load", "LIB_PATH", "geom", "num_taps", "gram", "set_gram_route", "nullspace",
           "nullspace_rsvd", "sketch", "jl_compress",
           "set_filter_group_budget", "filter_group",
           "workspace_bytes", "objective_grad", "line_search", "update", "solve", "solve_workspace_bytes",
           "time_average_init",
           "profile_begin",
           "profile_end"]
