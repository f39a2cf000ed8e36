"""ctypes view of libgcr.so (the C ABI declared in include/gcr.h).

Only marshalling lives here: structs, argument types and the loader.  The
library must have been built in-tree (``python -m paper_2306_08792_amd.build``);
loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgcr.so")

GCR_OK = 0
STATUS_NAMES = {0: "OK", -1: "INVALID", -2: "NOMEM", -3: "HIP", -4: "UNSUPPORTED", -5: "TIMEOUT"}
GCR_ERR_TIMEOUT = -5

# every exported entry point of include/gcr.h
EXPORTS = [
    "gcr_params_default", "gcr_create", "gcr_destroy", "gcr_last_error", "gcr_get_stats",
    "gcr_reserve", "gcr_workspace_bytes", "gcr_workspace_size", "gcr_profile_workspace_size",
    "gcr_propagate_noalloc", "gcr_propagate_noalloc_max_nodes",
    "gcr_reset_stats", "gcr_normalize_rows", "gcr_knn", "gcr_graph_bytes", "gcr_graph_bind",
    "gcr_build_graph", "gcr_propagate", "gcr_final_distances", "gcr_rerank",
    "gcr_profile_vectors", "gcr_set_timing", "gcr_get_timing",
    "gcr_server_config_default", "gcr_server_create", "gcr_server_submit", "gcr_server_wait",
    "gcr_server_get_stats", "gcr_server_last_error", "gcr_server_destroy",
    "gcr_dsfp", "gcr_rerank_local",
    "gcr_server_insert", "gcr_server_remove", "gcr_server_gallery_ids", "gcr_server_save", "gcr_server_load",
]
NUM_TIMERS = 8
TIMER_NAMES = ["sim_topk", "refine", "graph", "propagate", "final_dense", "prep", "final_topk_sweep",
               "final_topk_refine"]


class GcrParams(C.Structure):
    _fields_ = [
        ("k", C.c_int32), ("cross_k", C.c_int32), ("rounds", C.c_int32),
        ("rebuild_each_round", C.c_int32), ("normalize_input", C.c_int32),
        ("precision", C.c_int32), ("topk_out", C.c_int32), ("symmetric", C.c_int32),
        ("gamma", C.c_float), ("alpha", C.c_float), ("beta_same", C.c_float),
        ("beta_cross", C.c_float), ("lambda_", C.c_float),
    ]


class GcrStats(C.Structure):
    _fields_ = [("knn_rows", C.c_int64), ("knn_candidates", C.c_int64),
                ("knn_fallback_rows", C.c_int64), ("splits", C.c_int64),
                ("knn_exhaustive_rows", C.c_int64), ("tile_rows", C.c_int64)]


_P = C.c_void_p


class GcrTiming(C.Structure):
    _fields_ = [("ms", C.c_double * NUM_TIMERS), ("launches", C.c_int64 * NUM_TIMERS)]


class GcrGraph(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("k", C.c_int32), ("cross_k", C.c_int32), ("has_cross", C.c_int32),
        ("asymmetric", C.c_int32),
        ("idx", _P), ("rev_ptr", _P), ("rev_src", _P),
        ("dist", _P), ("w", _P), ("rev_w", _P), ("deg", _P), ("pf", _P), ("pr", _P),
        ("cr_idx", _P), ("cr_rev_ptr", _P), ("cr_rev_src", _P),
        ("cr_dist", _P), ("cr_w", _P), ("cr_rev_w", _P), ("cr_deg", _P), ("cr_pf", _P), ("cr_pr", _P),
        ("self_", _P),
    ]


class GcrServerConfig(C.Structure):
    _fields_ = [("lanes", C.c_int32), ("max_batch", C.c_int32), ("max_requests", C.c_int32),
                ("max_recomputed", C.c_int32), ("gallery_capacity", C.c_int32), ("reserved", C.c_int32),
                ("mem_budget", C.c_uint64)]


class GcrServerStats(C.Structure):
    _fields_ = [("requests_done", C.c_int64), ("queries_done", C.c_int64), ("batches_done", C.c_int64),
                ("max_batch_requests", C.c_int64), ("max_batch_rows", C.c_int64),
                ("max_recomputed_rows", C.c_int64), ("lanes", C.c_int64), ("max_batch", C.c_int64),
                ("max_requests", C.c_int64), ("request_slots", C.c_int64), ("max_recomputed", C.c_int64),
                ("device_bytes", C.c_int64), ("slot_bytes", C.c_int64), ("gallery_size", C.c_int64),
                ("gallery_capacity", C.c_int64), ("enqueue_us", C.c_int64)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libgcr.so once and declare the signatures."""
    global _lib
    if _lib is not None:
        return _lib
    # torch ships its own HIP runtime (soname libamdhip64.so.7).  Loading torch
    # first makes this library bind to that same runtime, so tensors that
    # torch allocated are valid device pointers here.
    import torch  # noqa: F401

    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with `python -m paper_2306_08792_amd.build` "
            "(there is no CPU fallback)")
    L = C.CDLL(path)
    i32, i64, f32, vp = C.c_int32, C.c_int64, C.c_float, C.c_void_p
    pP = C.POINTER(GcrParams)
    L.gcr_params_default.argtypes = [pP]
    L.gcr_params_default.restype = None
    L.gcr_create.argtypes = [C.POINTER(vp), C.c_int, C.c_size_t]
    L.gcr_reserve.argtypes = [vp, C.c_size_t]
    L.gcr_workspace_bytes.argtypes = [vp]
    L.gcr_workspace_bytes.restype = C.c_size_t
    L.gcr_workspace_size.argtypes = [pP, i64, i64, i32, i32]
    L.gcr_workspace_size.restype = C.c_size_t
    L.gcr_profile_workspace_size.argtypes = [i32, i64, i32, i32]
    L.gcr_profile_workspace_size.restype = C.c_size_t
    L.gcr_destroy.argtypes = [vp]
    L.gcr_last_error.argtypes = [vp]
    L.gcr_last_error.restype = C.c_char_p
    L.gcr_get_stats.argtypes = [vp, C.POINTER(GcrStats)]
    L.gcr_reset_stats.argtypes = [vp]
    L.gcr_normalize_rows.argtypes = [vp, vp, vp, i64, i32, vp]
    L.gcr_knn.argtypes = [vp, vp, i64, i32, vp, pP, vp, vp, vp, vp, vp]
    L.gcr_graph_bytes.argtypes = [i64, i32, i32, i32]
    L.gcr_graph_bytes.restype = C.c_size_t
    L.gcr_graph_bind.argtypes = [C.POINTER(GcrGraph), vp, i64, i32, i32, i32]
    L.gcr_build_graph.argtypes = [vp, vp, i64, i32, vp, pP, C.POINTER(GcrGraph), vp]
    L.gcr_propagate.argtypes = [vp, C.POINTER(GcrGraph), vp, vp, i64, i32, vp]
    L.gcr_propagate_noalloc.argtypes = [vp, C.POINTER(GcrGraph), vp, vp, i64, i32, vp]
    L.gcr_propagate_noalloc_max_nodes.argtypes = []
    L.gcr_propagate_noalloc_max_nodes.restype = C.c_size_t
    L.gcr_final_distances.argtypes = [vp, vp, i64, i64, i32, pP, vp, vp, vp, vp]
    L.gcr_rerank.argtypes = [vp, vp, i64, i64, i32, vp, pP, vp, vp, vp, vp, C.POINTER(GcrGraph), vp]
    L.gcr_set_timing.argtypes = [vp, i32]
    L.gcr_get_timing.argtypes = [vp, C.POINTER(GcrTiming)]
    L.gcr_profile_vectors.argtypes = [vp, vp, vp, vp, vp, vp, i32, i32, i32, f32, vp, vp]
    L.gcr_server_config_default.argtypes = [C.POINTER(GcrServerConfig)]
    L.gcr_server_config_default.restype = None
    L.gcr_server_create.argtypes = [vp, vp, i32, i64, i32, pP, C.POINTER(GcrServerConfig), C.POINTER(vp)]
    L.gcr_server_submit.argtypes = [vp, vp, i32, C.POINTER(C.c_uint64)]
    L.gcr_server_wait.argtypes = [vp, C.c_uint64, vp, vp, i32]
    L.gcr_server_get_stats.argtypes = [vp, C.POINTER(GcrServerStats)]
    L.gcr_server_last_error.argtypes = [vp]
    L.gcr_server_last_error.restype = C.c_char_p
    L.gcr_server_destroy.argtypes = [vp]
    L.gcr_dsfp.argtypes = [vp, vp, vp, i64, i32, i32, f32, i32, vp, vp]
    L.gcr_server_insert.argtypes = [vp, vp, i32, vp]
    L.gcr_server_remove.argtypes = [vp, vp, i32]
    L.gcr_server_gallery_ids.argtypes = [vp, vp, i64, C.POINTER(i64)]
    L.gcr_server_save.argtypes = [vp, C.c_char_p]
    L.gcr_server_load.argtypes = [vp, C.c_char_p, C.POINTER(GcrServerConfig), C.POINTER(vp)]
    L.gcr_rerank_local.argtypes = [vp, vp, i64, i64, i32, pP, vp, vp, vp, vp, vp]
    for name in EXPORTS:
        fn = getattr(L, name)
        if fn.restype is C.c_int:  # default restype: gcr_status
            fn.restype = C.c_int
    _lib = L
    return L
