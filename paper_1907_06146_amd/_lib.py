"""ctypes binding of libssg (include/ssg.h). Argument marshalling only.

Every step runs in the HIP kernels of ``csrc/ssg_search.hip`` (search) and
``csrc/ssg_knn.hip`` (kNN graph), ``csrc/ssg_build.hip`` (graph pruning) and
``csrc/ssg_merge.hip`` (partitioned-search aggregation).
There is no CPU or PyTorch fallback: if the shared library is missing or
cannot be loaded, every call raises.
"""

from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssg.so")

SSG_OK, SSG_EINVAL, SSG_ENOMEM, SSG_EDEVICE, SSG_EUNSUPPORTED = 0, -1, -2, -3, -4
SSG_L2, SSG_IP = 0, 1
SSG_F32, SSG_BF16, SSG_FP8E4M3 = 0, 1, 2
SENTINEL = 0xFFFFFFFF
L_MAX, R_MAX, K_MAX = 512, 64, 4096

EXPORTS = ("ssg_search", "ssg_search_ex", "ssg_quantize", "ssg_search_workspace_bytes",
           "ssg_validate_graph", "ssg_last_error", "ssg_version", "ssg_batch_workspace_bytes",
           "ssg_search_batched", "ssg_batch_graph_create", "ssg_batch_graph_launch",
           "ssg_batch_graph_destroy", "ssg_probe_gather", "ssg_knn_workspace_bytes",
           "ssg_knn_graph", "ssg_nssg_prune", "ssg_nssg_reverse_workspace_bytes", "ssg_nssg_reverse",
           "ssg_merge_shards", "ssg_exact_ssg_workspace_bytes", "ssg_exact_ssg",
           "ssg_query_lds_bytes", "ssg_search_batched_noalloc")


class SSGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libssg error {code}: {msg}")
        self.code = code


class SearchOpts(ctypes.Structure):
    _fields_ = [("exact_visited", ctypes.c_int32), ("hash_log2", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32), ("out_ndc", ctypes.c_void_p),
                ("out_hops", ctypes.c_void_p), ("gather_variant", ctypes.c_int32),
                ("base_f32", ctypes.c_void_p), ("rerank_k", ctypes.c_int32),
                ("entry_group_size", ctypes.c_int64), ("visited_kind", ctypes.c_int32),
                ("out_trace", ctypes.c_void_p), ("trace_cap", ctypes.c_int32),
                ("queries_per_wave", ctypes.c_int32)]


class BatchDesc(ctypes.Structure):
    _fields_ = [("base", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("metric", ctypes.c_int32),
                ("dim_scale", ctypes.c_void_p), ("base_f32", ctypes.c_void_p),
                ("rerank", ctypes.c_int32), ("graph", ctypes.c_void_p), ("R", ctypes.c_int32),
                ("entry_ids", ctypes.c_void_p), ("n_entry", ctypes.c_int32),
                ("queries", ctypes.c_void_p), ("nq", ctypes.c_int64), ("L", ctypes.c_void_p),
                ("K", ctypes.c_void_p), ("kstride", ctypes.c_int32), ("out_ids", ctypes.c_void_p),
                ("out_dists", ctypes.c_void_p), ("out_ndc", ctypes.c_void_p),
                ("out_hops", ctypes.c_void_p), ("out_trace", ctypes.c_void_p),
                ("trace_cap", ctypes.c_int32)]


class Bucket(ctypes.Structure):
    _fields_ = [("qlist", ctypes.c_void_p), ("count", ctypes.c_int64), ("max_L", ctypes.c_int32),
                ("gather_variant", ctypes.c_int32), ("hash_log2", ctypes.c_int32),
                ("waves_per_block", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("visited_kind", ctypes.c_int32), ("queries_per_wave", ctypes.c_int32)]


_lock = threading.Lock()
_lib = None


def lib() -> ctypes.CDLL:
    """Load libssg.so (built in-tree by ``__graft_entry__.build()``)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
            L = ctypes.CDLL(LIB_PATH)
            P, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
            L.ssg_search.argtypes = [P, i64, i32, i32, P, P, i32, P, i32, P, i64, i32, i32, i32, P,
                                     P, P, sz, P]
            L.ssg_search.restype = ctypes.c_int
            L.ssg_search_ex.argtypes = [P, i64, i32, i32, P, P, i32, P, i32, P, i64, i32, i32,
                                        i32, P, P, ctypes.POINTER(SearchOpts), P]
            L.ssg_search_ex.restype = ctypes.c_int
            L.ssg_quantize.argtypes = [P, i64, i32, i32, P, P, P]
            L.ssg_quantize.restype = ctypes.c_int
            L.ssg_search_workspace_bytes.argtypes = [i64, i64, i32, i32, i32]
            L.ssg_search_workspace_bytes.restype = sz
            L.ssg_validate_graph.argtypes = [P, i64, i32]
            L.ssg_validate_graph.restype = ctypes.c_int
            L.ssg_batch_workspace_bytes.argtypes = [i32]
            L.ssg_batch_workspace_bytes.restype = sz
            L.ssg_search_batched.argtypes = [ctypes.POINTER(BatchDesc), ctypes.POINTER(Bucket), i32, P,
                                             sz, P]
            L.ssg_search_batched.restype = ctypes.c_int
            L.ssg_batch_graph_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(BatchDesc),
                                                 ctypes.POINTER(Bucket), i32, P, sz]
            L.ssg_batch_graph_create.restype = ctypes.c_int
            L.ssg_batch_graph_launch.argtypes = [P, P]
            L.ssg_batch_graph_launch.restype = ctypes.c_int
            L.ssg_batch_graph_destroy.argtypes = [P]
            L.ssg_batch_graph_destroy.restype = ctypes.c_int
            L.ssg_probe_gather.argtypes = [P, i64, i32, P, i64, i32, P, P]
            L.ssg_probe_gather.restype = ctypes.c_int
            L.ssg_knn_workspace_bytes.argtypes = [i64, i32, i32]
            L.ssg_knn_workspace_bytes.restype = sz
            L.ssg_knn_graph.argtypes = [P, i64, i32, i32, P, P, P, sz, P, P]
            L.ssg_knn_graph.restype = ctypes.c_int
            dbl = ctypes.c_double
            L.ssg_nssg_prune.argtypes = [P, i64, i32, P, i32, i32, i32, dbl, P, P]
            L.ssg_nssg_prune.restype = ctypes.c_int
            L.ssg_nssg_reverse_workspace_bytes.argtypes = [i64, i32]
            L.ssg_nssg_reverse_workspace_bytes.restype = sz
            L.ssg_nssg_reverse.argtypes = [P, i64, i32, P, i32, dbl, P, P, sz, P]
            L.ssg_nssg_reverse.restype = ctypes.c_int
            L.ssg_merge_shards.argtypes = [P, P, i32, i64, i32, P, P, i64, i32, P, P, P]
            L.ssg_merge_shards.restype = ctypes.c_int
            L.ssg_exact_ssg_workspace_bytes.argtypes = [i64]
            L.ssg_exact_ssg_workspace_bytes.restype = sz
            L.ssg_exact_ssg.argtypes = [P, i64, i32, dbl, i32, P, P, P, sz, P]
            L.ssg_exact_ssg.restype = ctypes.c_int
            L.ssg_query_lds_bytes.argtypes = [i32, i32, i32, i32, i64, i32, i32]
            L.ssg_query_lds_bytes.restype = sz
            L.ssg_search_batched_noalloc.argtypes = [ctypes.POINTER(BatchDesc), ctypes.POINTER(Bucket),
                                                     i32, P]
            L.ssg_search_batched_noalloc.restype = ctypes.c_int
            L.ssg_last_error.restype = ctypes.c_char_p
            L.ssg_version.restype = ctypes.c_char_p
            _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != SSG_OK:
        raise SSGError(rc, lib().ssg_last_error().decode())


def last_error() -> str:
    return lib().ssg_last_error().decode()
