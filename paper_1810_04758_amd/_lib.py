"""ctypes binding of libknnjoin.so (the C ABI declared in include/knnjoin.h).

Argument marshalling only: every step of the join runs in the HIP library.
Loading fails loudly when the library has not been built.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libknnjoin.so")

KNN_OK = 0
KNN_EINVAL = -1
KNN_ENOMEM = -2
KNN_EDEVICE = -3
KNN_EBUSY = -4
KNN_ETIMEOUT = -5
KNN_EINTERNAL = -6
KNN_ECANCELED = -7
KNN_MAX_DIMS = 6
KNN_MAX_K = 1024
KNN_MAX_LEVELS = 64
KNN_NOALLOC_SCRATCH_BYTES = 64 << 20

c_i32, c_i64, c_u64, c_f64, c_p = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                   ctypes.c_double, ctypes.c_void_p)


class BuildOpts(ctypes.Structure):
    _fields_ = [("seed", c_u64), ("n_sample", c_i32), ("n_bins", c_i32),
                ("mean_frac", c_f64), ("min_mean_sample", c_i32), ("device", c_i32)]


class JoinStats(ctypes.Structure):
    _fields_ = [("levels", c_i32), ("eps_min", c_f64),
                ("cell_width", c_f64 * KNN_MAX_LEVELS),
                ("attempted", c_i64 * KNN_MAX_LEVELS),
                ("failed", c_i64 * KNN_MAX_LEVELS),
                ("cells", c_i64 * KNN_MAX_LEVELS),
                ("ms_build", c_f64 * KNN_MAX_LEVELS),
                ("ms_search", c_f64 * KNN_MAX_LEVELS),
                ("ms_total", c_f64), ("total_attempted", c_i64), ("total_failed", c_i64),
                ("lanes_per_query", c_i32), ("lanes", c_i32 * KNN_MAX_LEVELS),
                ("cand_per_query", c_f64 * KNN_MAX_LEVELS),
                ("refine_rounds", c_i64 * KNN_MAX_LEVELS),
                ("tail_queries", c_i64), ("tail_rounds", c_i32), ("ms_tail", c_f64),
                ("ms_heavy", c_f64 * KNN_MAX_LEVELS), ("heavy_queries", c_i64 * KNN_MAX_LEVELS),
                ("heavy_failed", c_i64 * KNN_MAX_LEVELS), ("heavy_cand", c_f64 * KNN_MAX_LEVELS),
                ("spec_queries", c_i64 * KNN_MAX_LEVELS),
                ("deferred", c_i64 * KNN_MAX_LEVELS)]

    def as_dict(self):
        L = self.levels
        return dict(levels=L, eps_min=self.eps_min, lanes_per_query=self.lanes_per_query,
                    cell_width=list(self.cell_width[:L]), attempted=list(self.attempted[:L]),
                    failed=list(self.failed[:L]), cells=list(self.cells[:L]),
                    ms_build=list(self.ms_build[:L]), ms_search=list(self.ms_search[:L]),
                    ms_total=self.ms_total, total_attempted=self.total_attempted,
                    total_failed=self.total_failed, lanes=list(self.lanes[:L]),
                    cand_per_query=list(self.cand_per_query[:L]),
                    refine_rounds=list(self.refine_rounds[:L]),
                    tail_queries=self.tail_queries, tail_rounds=self.tail_rounds,
                    ms_tail=self.ms_tail, ms_heavy=list(self.ms_heavy[:L]),
                    heavy_queries=list(self.heavy_queries[:L]),
                    heavy_failed=list(self.heavy_failed[:L]),
                    heavy_cand=list(self.heavy_cand[:L]),
                    spec_queries=list(self.spec_queries[:L]),
                    deferred=list(self.deferred[:L]))


class JoinOpts(ctypes.Structure):
    _fields_ = [("w_factor", c_f64), ("cell_width", c_f64), ("lanes_per_query", c_i32),
                ("schedule", c_i32), ("batch_queries", c_i32), ("eps_step", c_f64),
                ("linear_levels", c_i32), ("growth", c_f64), ("use_graph", c_i32),
                ("tail_pairs", c_f64), ("heavy_min", ctypes.c_int64),
                ("queue_grain", c_i32), ("item_order", c_i32), ("lanes_shift", c_i32),
                ("share_lists", c_i32),
                ("speculate", c_i32),
                ("predict_fail", c_i32),
                ("zorder", c_i32),
                ("stats", ctypes.POINTER(JoinStats))]


class IndexInfo(ctypes.Structure):
    _fields_ = [("n_points", c_i64), ("dims", c_i32), ("device", c_i32),
                ("lo", c_f64 * KNN_MAX_DIMS), ("hi", c_f64 * KNN_MAX_DIMS),
                ("eps_mean", c_f64), ("n_bins", c_i32), ("n_sample", c_i32),
                ("device_bytes", c_i64)]


class AutotuneResult(ctypes.Structure):
    _fields_ = [("w_factor", c_f64), ("growth", c_f64), ("ms_best", c_f64),
                ("ms_default", c_f64), ("trials", c_i32), ("linear_levels", c_i32),
                ("tail_pairs", c_f64), ("lanes_shift", c_i32), ("zorder", c_i32),
                ("queue_pops", c_i32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", c_u64), ("max_inflight", c_i32), ("max_queue", c_i32),
                ("device", c_i32)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", c_i64), ("completed", c_i64), ("failed", c_i64),
                ("p50_ms", c_f64), ("p99_ms", c_f64), ("mean_ms", c_f64), ("max_ms", c_f64),
                ("queries_per_s", c_f64), ("requests_per_s", c_f64), ("peak_bytes", c_u64),
                ("peak_inflight", c_i32)]


class HybridOpts(ctypes.Structure):
    _fields_ = [("n_large", c_f64), ("n_small", c_f64), ("n_cwin", c_f64), ("n_cpu", c_f64),
                ("eps_factor", c_f64), ("cpu_threads", c_i32), ("zorder", c_i32)]


class HybridStats(ctypes.Structure):
    _fields_ = [("ms_total", c_f64), ("ms_gpu", c_f64), ("ms_cpu", c_f64),
                ("load_imbalance", c_f64), ("ms_queue", c_f64), ("ms_cpu_index", c_f64),
                ("ms_merge", c_f64), ("eps_min", c_f64), ("eps_final", c_f64), ("gpu_queries", c_i64),
                ("cpu_queries", c_i64), ("gpu_attempts", c_i64), ("gpu_batches", c_i32),
                ("monolithic_batches", c_i32), ("reindexes", c_i32), ("cpu_threads", c_i32)]


class EpsJoinStats(ctypes.Structure):
    _fields_ = [("n_pairs", c_u64), ("n_batches", c_i64), ("ms_total", c_f64),
                ("ms_count", c_f64), ("ms_wait", c_f64), ("ms_consume", c_f64)]


# int consume(const int32_t* qids, const int32_t* nids, const double* dists,
#             uint64_t n_pairs, void* user)
EpsConsumer = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.POINTER(c_i32), ctypes.POINTER(c_i32),
                               ctypes.POINTER(c_f64), c_u64, c_p)


# name -> (restype, argtypes)
SIGNATURES = {
    "knn_build_opts_default": (None, [ctypes.POINTER(BuildOpts)]),
    "knn_join_opts_default": (None, [ctypes.POINTER(JoinOpts)]),
    "knn_build_index": (ctypes.c_int, [c_p, c_i64, c_i32, ctypes.POINTER(BuildOpts),
                                       ctypes.POINTER(c_p)]),
    "knn_build_index_device": (ctypes.c_int, [c_p, c_i64, c_i32, ctypes.POINTER(BuildOpts), c_p,
                                              ctypes.POINTER(c_p)]),
    "knn_self_join": (ctypes.c_int, [c_p, c_i32, c_p, c_p, ctypes.POINTER(JoinOpts)]),
    "knn_self_join_device": (ctypes.c_int, [c_p, c_i32, c_p, c_p, ctypes.POINTER(JoinOpts),
                                            c_p]),
    "knn_join_device": (ctypes.c_int, [c_p, c_p, c_i64, c_i32, c_p, c_p,
                                       ctypes.POINTER(JoinOpts), c_p]),
    "knn_join": (ctypes.c_int, [c_p, c_p, c_i64, c_i32, c_p, c_p, ctypes.POINTER(JoinOpts)]),
    "knn_self_join_device_noalloc": (ctypes.c_int, [c_p, c_i32, c_p, c_p,
                                                    ctypes.POINTER(JoinOpts), c_p]),
    "knn_self_join_hybrid": (ctypes.c_int, [c_p, c_i32, c_p, c_p, ctypes.POINTER(HybridOpts),
                                             ctypes.POINTER(HybridStats)]),
    "knn_eps_join_size": (ctypes.c_int, [c_p, c_f64, c_i64, ctypes.POINTER(c_u64), c_p, c_p]),
    "knn_eps_join_device": (ctypes.c_int, [c_p, c_f64, c_i64, c_u64, c_p, c_p, c_p,
                                           ctypes.POINTER(c_u64), ctypes.POINTER(c_i64), c_p]),
    "knn_eps_join": (ctypes.c_int, [c_p, c_f64, c_u64, c_i32, EpsConsumer, c_p,
                                    ctypes.POINTER(EpsJoinStats)]),
    "knn_eps_join_release": (ctypes.c_int, [c_p]),
    "knn_destroy_index": (None, [c_p]),
    "knn_last_error": (ctypes.c_char_p, []),
    "knn_index_info_get": (ctypes.c_int, [c_p, ctypes.POINTER(IndexInfo)]),
    "knn_eps_min": (ctypes.c_int, [c_p, c_i32, ctypes.POINTER(c_f64)]),
    "knn_index_sampling_get": (ctypes.c_int, [c_p, c_p, c_p, ctypes.POINTER(c_i64), c_p,
                                              ctypes.POINTER(c_f64)]),
    "knn_join_footprint": (ctypes.c_int, [c_p, c_i32, ctypes.POINTER(c_u64)]),
    "knn_autotune": (ctypes.c_int, [c_p, c_i32, c_p, ctypes.POINTER(AutotuneResult)]),
    "knn_autotune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "knn_autotune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "knn_grid_export": (ctypes.c_int, [c_p, c_f64, c_p, c_p, c_p, c_p, c_p, c_p,
                                       ctypes.POINTER(c_i64)]),
    "knn_sample_mean_dist": (ctypes.c_int, [c_p, c_i64, c_i32, c_p, c_i64,
                                            ctypes.POINTER(c_f64), c_p]),
    "knn_dist_histogram": (ctypes.c_int, [c_p, c_i64, c_i32, c_p, c_i64, c_f64, c_i32, c_p,
                                          c_p]),
    "knn_server_create": (ctypes.c_int, [ctypes.POINTER(ServerOpts), ctypes.POINTER(c_p)]),
    "knn_server_add_dataset": (ctypes.c_int, [c_p, c_p, ctypes.POINTER(c_i32)]),
    "knn_server_submit": (ctypes.c_int, [c_p, c_i32, c_i32, c_p, c_p, ctypes.POINTER(c_i64)]),
    "knn_server_wait": (ctypes.c_int, [c_p, c_i64, c_i64]),
    "knn_server_stats_get": (ctypes.c_int, [c_p, ctypes.POINTER(ServerStats)]),
    "knn_server_destroy": (None, [c_p]),
}

_lib = None


class KnnError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"knnjoin error {code}: {msg}")
        self.code = code


def load():
    """Load libknnjoin.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1810_04758_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != KNN_OK:
        msg = load().knn_last_error()
        raise KnnError(rc, msg.decode() if msg else "")
    return rc
