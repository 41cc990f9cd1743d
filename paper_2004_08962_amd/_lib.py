"""ctypes view of libhicu.so (declarations mirror include/hicu.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation of any step.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhicu.so")

c_int32, c_int64, c_uint32, c_uint64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
c_size_t, c_void_p, c_double_p = ctypes.c_size_t, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)

HICU_OK, HICU_CONVERGED = 0, 1
STATUS = {
    0: "HICU_OK", 1: "HICU_CONVERGED", -1: "HICU_ERR_ARG", -2: "HICU_ERR_SHAPE", -3: "HICU_ERR_RANK",
    -4: "HICU_ERR_NONFINITE", -5: "HICU_ERR_HIP", -6: "HICU_ERR_WORKSPACE", -7: "HICU_ERR_UNSUPPORTED",
    -8: "HICU_ERR_NOCONV",
}
PREC = {"fp32": 0, "bf16": 1, "bf16x3": 2, "fp16": 3}


class Geom(ctypes.Structure):
    _fields_ = [("ndim", c_int32), ("nchan", c_int32), ("dims", c_int64 * 3), ("kdims", c_int32 * 3),
                ("lo", c_int64 * 3), ("hi", c_int64 * 3), ("wrap", c_int32), ("kmask", c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("rank", c_int32), ("p", c_int32), ("n_outer", c_int32), ("start_outer", c_int32),
                ("steps", ctypes.POINTER(c_int32)), ("regions", ctypes.POINTER(c_int64)),
                ("seed", c_uint64), ("prec", c_int32), ("refine_steps", c_int32), ("warm_start", c_int32),
                ("route", c_int32), ("sketch", c_int32), ("refine_prec", c_int32)]


class Trace(ctypes.Structure):
    _fields_ = [("outer", c_int32), ("inner", c_int32), ("prec", c_int32), ("sweeps", c_int32),
                ("J", ctypes.c_double), ("gnorm2", ctypes.c_double), ("eta", ctypes.c_double)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", c_int64), ("total_ms", ctypes.c_double),
                ("min_ms", ctypes.c_double), ("max_ms", ctypes.c_double), ("flops", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class BatchItem(ctypes.Structure):
    _fields_ = [("geom", Geom), ("x", c_void_p), ("mask", c_void_p), ("Q", c_void_p), ("nq", c_int32),
                ("p", c_int32), ("seed", c_uint64), ("scalars", c_void_p)]


class HicuError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s failed: %s (%d)" % (where, STATUS.get(status, "?"), status))


# name -> (restype, argtypes); the exported C-ABI surface.
SIGNATURES = {
    "hicu_version": (c_int32, []),
    "hicu_status_string": (ctypes.c_char_p, [c_int32]),
    "hicu_num_taps": (c_int64, [ctypes.POINTER(Geom)]),
    "hicu_num_outputs": (c_int64, [ctypes.POINTER(Geom)]),
    "hicu_gram_workspace_bytes": (c_size_t, [ctypes.POINTER(Geom)]),
    "hicu_gram": (c_int32, [ctypes.POINTER(Geom), c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "hicu_set_gram_route": (c_int32, [c_int32]),
    "hicu_nullspace_workspace_bytes": (c_size_t, [c_int32]),
    "hicu_nullspace": (c_int32, [c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                 ctypes.POINTER(c_int32), c_void_p, c_size_t, c_void_p]),
    "hicu_nullspace_rsvd_workspace_bytes": (c_size_t, [ctypes.POINTER(Geom), c_int32, c_int32]),
    "hicu_nullspace_rsvd": (c_int32, [ctypes.POINTER(Geom), c_void_p, c_int32, c_int32, c_uint64, c_uint32,
                                      c_uint32, c_void_p, c_void_p, ctypes.POINTER(c_int32), c_void_p, c_size_t,
                                      c_void_p]),
    "hicu_sketch": (c_int32, [c_int32, c_int32, c_uint64, c_uint32, c_uint32, c_void_p, c_void_p]),
    "hicu_jl_compress": (c_int32, [c_int32, c_int32, c_int32, c_void_p, c_uint64, c_uint32, c_uint32,
                                   c_uint32, c_void_p, c_void_p, c_void_p]),
    "hicu_workspace_bytes": (c_size_t, [ctypes.POINTER(Geom), c_int32, c_int32]),
    "hicu_set_filter_group_budget": (c_int32, [c_size_t]),
    "hicu_filter_group": (c_int32, [ctypes.POINTER(Geom), c_int32, c_int32, ctypes.POINTER(c_int32),
                              ctypes.POINTER(c_int32)]),
    "hicu_objective_grad": (c_int32, [ctypes.POINTER(Geom), c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "hicu_line_search": (c_int32, [ctypes.POINTER(Geom), c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                   c_void_p, c_void_p, c_size_t, c_void_p]),
    "hicu_update": (c_int32, [ctypes.POINTER(Geom), c_void_p, c_void_p, c_void_p, c_void_p]),
    "hicu_time_average_init": (c_int32, [ctypes.POINTER(Geom), c_int32, c_void_p, c_void_p, c_void_p, c_void_p]),
    "hicu_line_search_noalloc_max_bytes": (c_size_t, []),
    "hicu_line_search_noalloc": (c_int32, [ctypes.POINTER(Geom), c_void_p, c_void_p, c_void_p, c_int32, c_int32,
                                           c_void_p, c_void_p]),
    "hicu_profile_begin": (c_int32, []),
    "hicu_profile_begin_major": (c_int32, []),
    "hicu_profile_end": (c_int32, [ctypes.POINTER(KernelStat), c_int32, ctypes.POINTER(c_int32)]),
    "hicu_batch_create": (c_int32, [ctypes.POINTER(BatchItem), c_int32, c_int32, ctypes.POINTER(c_void_p),
                                    ctypes.POINTER(c_size_t)]),
    "hicu_batch_bind": (c_int32, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "hicu_batch_set_counter": (c_int32, [c_void_p, c_uint32, c_uint32, c_void_p]),
    "hicu_batch_step": (c_int32, [c_void_p, c_void_p]),
    "hicu_batch_graph_create": (c_int32, [c_void_p, c_int32, c_void_p]),
    "hicu_batch_graph_launch": (c_int32, [c_void_p, c_void_p]),
    "hicu_batch_info": (c_int32, [c_void_p, ctypes.POINTER(c_int64)]),
    "hicu_batch_destroy": (None, [c_void_p]),
    "hicu_autotune_workspace_bytes": (c_size_t, [ctypes.POINTER(Geom), c_int32, c_int32]),
    "hicu_autotune": (c_int32, [ctypes.POINTER(Geom), c_void_p, c_void_p, c_int32, c_int32, c_void_p, c_size_t,
                                ctypes.POINTER(c_int32), c_void_p]),
    "hicu_autotune_batched": (c_int32, [ctypes.POINTER(Geom), c_void_p, c_void_p, c_int32, c_int32, c_void_p,
                                        c_size_t, ctypes.POINTER(c_int32), c_void_p]),
    "hicu_tune_save": (c_int32, [ctypes.c_char_p]),
    "hicu_tune_load": (c_int32, [ctypes.c_char_p]),
    "hicu_tune_clear": (c_int32, []),
    "hicu_tune_put": (c_int32, [ctypes.POINTER(Geom), c_int32, c_int32, c_int32, c_int32, c_int32]),
    "hicu_tile_count": (c_int32, []),
    "hicu_tile_info": (c_int32, [c_int32, c_void_p]),
    "hicu_solve_workspace_bytes": (c_size_t, [ctypes.POINTER(Geom), ctypes.POINTER(Params)]),
    "hicu_solve": (c_int32, [ctypes.POINTER(Geom), c_void_p, c_void_p, ctypes.POINTER(Params), c_void_p,
                             ctypes.POINTER(Trace), c_void_p, c_size_t, c_void_p]),
}

_LIB = None


def load():
    """Load libhicu.so once; raise ImportError if it is not built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libhicu.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def check(status, where):
    if status < 0:
        raise HicuError(status, where)
    return status
