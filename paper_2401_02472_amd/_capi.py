"""ctypes declarations of the C ABI in include/bc.h (argument marshalling only).

The shared library is built in-tree (``libbc_mi355x.so`` next to this file).
If it is missing it is built once with hipcc; if that fails, loading raises --
there is no fallback path: every step of the computation runs in the HIP
kernels behind this ABI.
"""
from __future__ import annotations

import ctypes
import os
import threading

from . import build as _build

LIB_PATH = _build.LIB_PATH
# BC_MI355X_CHECK_EXEC=1 loads the check build instead (see build.py)
CHECK_EXEC = os.environ.get("BC_MI355X_CHECK_EXEC", "") == "1"

BC_OK = 0
BC_ERR_INVALID_ARG = 1
BC_ERR_INVALID_GRAPH = 2
BC_ERR_OUT_OF_MEMORY = 3
BC_ERR_RANGE = 4
BC_ERR_DEVICE = 5
BC_ERR_UNSUPPORTED = 6
BC_ERR_TOO_LARGE = 7
BC_NOALLOC_SCRATCH_BYTES = 64 << 20

BC_GRAPH_TRUST_SYMMETRIC = 1 << 0
BC_GRAPH_INPUT_ON_DEVICE = 1 << 1
BC_GRAPH_DIRECTED = 1 << 2

BC_MODE_AUTO = 0
BC_MODE_PLAIN = 1
BC_MODE_BATCHED = 2

EXPORTED = ("bc_create_graph", "bc_destroy_graph", "bc_graph_info", "bc_run", "bc_run_async",
            "bc_run_multi", "bc_single_source", "bc_run_detail", "bc_workspace_bytes", "bc_trim_workspaces",
            "bc_profile_enable", "bc_profile_read", "bc_autotune", "bc_set_weights", "bc_sssp",
            "bc_pagerank", "bc_status_str", "bc_run_async_noalloc",
            "bc_workspace_held", "bc_set_work_items", "bc_run_graphs")

BC_LOOP_AUTO = 0
BC_LOOP_HOST = 1
BC_LOOP_DEVICE = 2
BC_LOOP_GRAPH = 3

BC_PROF_FORWARD = 0
BC_PROF_COMPACT = 1
BC_PROF_REVERSE = 2
BC_PROF_FINISH = 3
BC_PROF_FUSED = 4
BC_PROF_SSSP = 5
BC_PROF_PAGERANK = 6
BC_PROF_CLASSES = 7
PROF_CLASS_NAMES = ("forward", "compact", "reverse", "finish", "fused", "sssp", "pagerank")


class bc_options(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("batch_width", ctypes.c_int32),
                ("level_chunk", ctypes.c_int32), ("sparse_div", ctypes.c_int32),
                ("concurrency", ctypes.c_int32), ("level_loop", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class bc_tuning(ctypes.Structure):
    _fields_ = [("batch_width", ctypes.c_int32), ("sparse_div", ctypes.c_int32),
                ("min_batched", ctypes.c_int32), ("sample", ctypes.c_int32),
                ("plain_ms_per_source", ctypes.c_double), ("batch_ms", ctypes.c_double),
                ("cached", ctypes.c_int32), ("group_cut", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class bc_profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * BC_PROF_CLASSES),
                ("ms", ctypes.c_double * BC_PROF_CLASSES),
                ("owners", ctypes.c_int64 * BC_PROF_CLASSES),
                ("arcs", ctypes.c_int64 * BC_PROF_CLASSES),
                ("hits", ctypes.c_int64 * BC_PROF_CLASSES),
                ("runs", ctypes.c_int64),
                ("vertices", ctypes.c_int64 * BC_PROF_CLASSES),
                ("levels", ctypes.c_int64)]


_lib = None
_lock = threading.Lock()


def load():
    """Load (building first if absent) the HIP library and declare its signatures."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        path = _build.CHECK_LIB_PATH if CHECK_EXEC else LIB_PATH
        if not os.path.exists(path):
            _build.build(check_exec=CHECK_EXEC)
        lib = ctypes.CDLL(path)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        f64p = ctypes.POINTER(ctypes.c_double)
        szp = ctypes.POINTER(ctypes.c_size_t)
        vp = ctypes.c_void_p
        optp = ctypes.POINTER(bc_options)
        sig = {
            "bc_create_graph": [ctypes.c_int32, vp, vp, ctypes.c_uint32, vp, ctypes.POINTER(vp)],
            "bc_destroy_graph": [vp],
            "bc_graph_info": [vp, i32p, i64p, szp],
            "bc_run": [vp, i32p, ctypes.c_int32, f64p],
            "bc_run_async": [vp, i32p, ctypes.c_int32, vp, optp, vp],
            "bc_run_async_noalloc": [vp, i32p, ctypes.c_int32, vp, vp],
            "bc_run_multi": [vp, i32p, i32p, ctypes.c_int32, ctypes.POINTER(vp), vp],
            "bc_run_graphs": [ctypes.POINTER(vp), ctypes.c_int32, ctypes.POINTER(vp), i32p,
                              ctypes.POINTER(vp), ctypes.c_int32, i32p, vp],
            "bc_single_source": [vp, ctypes.c_int32, i32p, f64p, f64p],
            "bc_run_detail": [vp, i32p, ctypes.c_int32, optp, f64p, i32p, f64p],
            "bc_workspace_bytes": [vp, ctypes.c_int32, optp, szp],
            "bc_trim_workspaces": [vp],
            "bc_workspace_held": [vp, szp],
            "bc_profile_enable": [vp, ctypes.c_int32],
            "bc_profile_read": [vp, ctypes.POINTER(bc_profile), ctypes.c_int32],
            "bc_autotune": [vp, i32p, ctypes.c_int32, vp, ctypes.POINTER(bc_tuning)],
            "bc_set_work_items": [vp, ctypes.c_int32, ctypes.c_int32],
            "bc_set_weights": [vp, i32p],
            "bc_sssp": [vp, ctypes.c_int32, vp, vp],
            "bc_pagerank": [vp, ctypes.c_double, ctypes.c_double, ctypes.c_int32, vp, i32p, vp],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        if CHECK_EXEC:
            lib.bc_debug_exec_partial.argtypes = []
            lib.bc_debug_exec_partial.restype = ctypes.c_uint
        lib.bc_status_str.argtypes = [ctypes.c_int]
        lib.bc_status_str.restype = ctypes.c_char_p
        _lib = lib
        return lib
