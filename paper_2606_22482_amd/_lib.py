"""ctypes mirror of ``include/spmm.h``: loads ``libspmm.so`` and declares every
entry point.  Argument marshalling only; all computation is in the library."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspmm.so")

SPMM_OK, SPMM_ERR_INVALID, SPMM_ERR_OOM, SPMM_ERR_DEVICE = 0, 1, 2, 3
SPMM_ERR_UNSUPPORTED, SPMM_ERR_BUDGET, SPMM_ERR_BUSY = 4, 5, 6
SPMM_TOL_FP32, SPMM_TOL_ROUNDED16 = 0, 1
F32, BF16, F16 = 0, 1, 2
MODE_AUTO, MODE_PLAIN_F32, MODE_MIXED, MODE_MFMA_ONLY = 0, 1, 2, 3
ORDER_AUTO, ORDER_ORIGINAL_RANGES, ORDER_COMPACTED, ORDER_LENGTH_SORTED = 0, 1, 2, 3
ORDER_CLUSTERED = 4
AUTO_INT = -(2 ** 31)
KERNEL_SEGMENT, KERNEL_VECTOR, KERNEL_WINDOW = 0, 1, 2
KERNEL_NAMES = {0: "segment", 1: "vector", 2: "window", 3: "window_partial", 4: "vector_path",
                5: "mfma_path", 6: "one_grid"}
EXEC_SERIAL, EXEC_TWO_GRIDS, EXEC_ONE_GRID = 1, 2, 3
TUNE_RUN, TUNE_SUBMIT = 0, 1
KIND_CODE = {"f32": F32, "bf16": BF16, "f16": F16}


class Csr(C.Structure):
    _fields_ = [("m", C.c_int64), ("k", C.c_int64), ("nnz", C.c_int64),
                ("rowptr", C.c_void_p), ("colidx", C.c_void_p), ("vals", C.c_void_p),
                ("val_type", C.c_int32), ("reserved", C.c_int32)]


class Opts(C.Structure):
    _fields_ = [("mode", C.c_int32), ("window_h", C.c_int32), ("t_row", C.c_int32),
                ("kt", C.c_int32), ("n_panel", C.c_int32), ("row_order", C.c_int32),
                ("seg_len", C.c_int32), ("item_cost", C.c_int32), ("xcd_remap", C.c_int32),
                ("hot_cols", C.c_int32), ("alpha_c", C.c_float), ("alpha", C.c_float),
                ("cold_policy", C.c_int32), ("pipeline", C.c_int32),
                ("win_sched", C.c_int32), ("local_reorder", C.c_int32), ("exec", C.c_int32)]


class PlanStats(C.Structure):
    _fields_ = [("m", C.c_int64), ("k", C.c_int64), ("nnz", C.c_int64), ("n", C.c_int64),
                ("val_type", C.c_int32), ("b_type", C.c_int32), ("c_type", C.c_int32),
                ("tile_type", C.c_int32), ("opts", Opts),
                ("windows", C.c_int64), ("tiles", C.c_int64), ("nnz_tiles", C.c_int64),
                ("nnz_remainder", C.c_int64), ("vector_rows", C.c_int64),
                ("segments", C.c_int64), ("vector_items", C.c_int64), ("k_ref", C.c_int64),
                ("hot_cols", C.c_int64),
                ("mean_tile_density", C.c_double), ("zero_fraction_tiles", C.c_double),
                ("device_bytes", C.c_int64), ("workspace_bytes", C.c_int64),
                ("algorithmic_bytes", C.c_double), ("flops", C.c_double),
                ("plan_ms", C.c_double), ("uploaded", C.c_int32), ("tol_class", C.c_int32),
                ("work_vec", C.c_double), ("work_tile", C.c_double), ("work_winrem", C.c_double)]


class PlanDump(C.Structure):
    _fields_ = [("m", C.c_int64), ("nnz", C.c_int64), ("window_h", C.c_int32),
                ("kt", C.c_int32), ("n_windows", C.c_int64), ("windows", C.c_void_p),
                ("n_tiles", C.c_int64), ("tile_window", C.c_void_p), ("tile_cols", C.c_void_p),
                ("tile_bitmap", C.c_void_p), ("tile_val_ptr", C.c_void_p),
                ("tile_vals", C.c_void_p), ("tile_src", C.c_void_p), ("rem_ptr", C.c_void_p),
                ("rem_src", C.c_void_p), ("n_vector_rows", C.c_int64),
                ("vector_rows", C.c_void_p), ("nseg", C.c_void_p), ("n_vitems", C.c_int64),
                ("vitem_ptr", C.c_void_p), ("vitem_seg", C.c_void_p),
                ("n_segments", C.c_int64), ("seg_row", C.c_void_p), ("seg_begin", C.c_void_p),
                ("seg_end", C.c_void_p), ("win_seg", C.c_void_p), ("win_order", C.c_void_p),
                ("rem_col_dev", C.c_void_p), ("n_wparts", C.c_int64), ("win_part", C.c_void_p),
                ("wpart_win", C.c_void_p), ("wpart_t0", C.c_void_p), ("wpart_t1", C.c_void_p),
                ("vexec_rows", C.c_void_p), ("n_dep", C.c_int64), ("seg_win", C.c_void_p),
                ("win_dep", C.c_void_p), ("win_nsseg", C.c_void_p)]


class TuneReport(C.Structure):
    _fields_ = [("candidates", C.c_int32), ("reserved", C.c_int32), ("default_ms", C.c_double),
                ("best_ms", C.c_double), ("alpha_cost", C.c_double), ("p_vec", C.c_double),
                ("p_mfma", C.c_double), ("search_ms", C.c_double)]


class AdaptState(C.Structure):
    _fields_ = [("alpha", C.c_double), ("alpha_star", C.c_double), ("lo", C.c_double),
                ("hi", C.c_double), ("rounds", C.c_int32), ("converged", C.c_int32),
                ("replanned", C.c_int32), ("capped", C.c_int32), ("skew", C.c_double),
                ("p_vec", C.c_double), ("p_mfma", C.c_double), ("t_vec_ms", C.c_double),
                ("t_mfma_ms", C.c_double), ("prev_alpha", C.c_double),
                ("prev_alpha_star", C.c_double)]


class Work(C.Structure):
    _fields_ = [("plan", C.c_void_p), ("B", C.c_void_p), ("ldb", C.c_int64),
                ("C", C.c_void_p), ("ldc", C.c_int64)]


_P = C.c_void_p
_S = C.c_int32
SIGNATURES = {
    "spmm_abi_version": (C.c_int32, []),
    "spmm_sizeof": (C.c_int64, [C.c_int32]),
    "spmm_status_string": (C.c_char_p, [_S]),
    "spmm_last_error": (C.c_char_p, []),
    "spmm_opts_default": (None, [C.POINTER(Opts)]),
    "spmm_plan_build": (_S, [C.POINTER(Csr), C.c_int32, C.c_int32, C.c_int32,
                             C.POINTER(Opts), C.POINTER(_P)]),
    "spmm_plan_upload": (_S, [_P]),
    "spmm_plan": (_S, [C.POINTER(Csr), C.c_int32, C.c_int32, C.c_int32, C.POINTER(Opts),
                       C.POINTER(_P)]),
    "spmm_plan_destroy": (_S, [_P]),
    "spmm_plan_device": (_S, [C.POINTER(Csr), C.c_int32, C.c_int32, C.c_int32, C.POINTER(Opts), _P,
                              C.POINTER(_P)]),
    "spmm_plan_serialize": (_S, [_P, _P, C.c_int64, C.POINTER(C.c_int64)]),
    "spmm_plan_deserialize": (_S, [_P, C.c_int64, C.c_int32, C.POINTER(_P)]),
    "spmm_plan_stats": (_S, [_P, C.POINTER(PlanStats)]),
    "spmm_plan_export": (_S, [_P, C.POINTER(PlanDump)]),
    "spmm_run": (_S, [_P, _P, C.c_int64, _P, C.c_int64, _P]),
    "spmm_run_noalloc": (_S, [_P, _P, C.c_int64, _P, C.c_int64, _P]),
    "spmm_run_bytes": (_S, [_P, C.c_int64, C.c_int64, C.c_int32, C.c_int64, C.POINTER(C.c_int64)]),
    "spmm_timer_create": (_S, [C.c_int32, C.POINTER(_P)]),
    "spmm_timer_reset": (_S, [_P]),
    "spmm_timer_read": (_S, [_P, C.POINTER(C.c_int32), C.POINTER(C.c_float), C.c_int32,
                             C.POINTER(C.c_int32)]),
    "spmm_timer_destroy": (_S, [_P]),
    "spmm_run_timed": (_S, [_P, _P, C.c_int64, _P, C.c_int64, _P, _P]),
    "spmm_submit": (_S, [C.POINTER(Work), C.c_int32, _P, C.POINTER(C.c_uint64)]),
    "spmm_poll": (_S, [C.c_uint64, C.POINTER(C.c_int32)]),
    "spmm_wait": (_S, [C.c_uint64]),
    "spmm_dryrun": (_S, [C.c_int32, C.c_int32, _P, C.POINTER(C.c_double),
                         C.POINTER(C.c_double)]),
    "spmm_copy_bandwidth": (_S, [C.c_int64, _P, C.POINTER(C.c_double)]),
    "spmm_gather_bandwidth": (_S, [_P, C.c_int64, _P, C.c_int64, C.c_int64, C.c_int32, C.c_int32, _P,
                                   C.POINTER(C.c_double)]),
    "spmm_adapt_next": (_S, [C.POINTER(AdaptState), C.c_double, C.c_double, C.c_double,
                             C.c_double, C.c_double, C.c_double, C.c_double, C.c_float]),
    "spmm_adapt_epoch": (_S, [C.POINTER(Csr), C.POINTER(_P), _P, C.c_int64, _P, C.c_int64, _P,
                              C.c_float, C.POINTER(AdaptState)]),
    "spmm_autotune": (_S, [C.POINTER(Csr), C.c_int32, C.c_int32, C.c_int32, _P, C.c_int64, _P,
                           C.c_int64, _P, C.c_double, C.c_int32, C.POINTER(Opts),
                           C.POINTER(TuneReport)]),
    "spmm_profile_key": (_S, [C.POINTER(Csr), C.c_int32, C.c_int32, C.c_char_p, C.c_int32]),
    "spmm_tune_cache_put": (_S, [C.c_char_p, C.POINTER(Opts)]),
    "spmm_tune_cache_get": (_S, [C.c_char_p, C.POINTER(Opts), C.POINTER(C.c_int32)]),
    "spmm_tune_cache_save": (_S, [C.c_char_p]),
    "spmm_tune_cache_load": (_S, [C.c_char_p]),
    "spmm_tune_cache_clear": (None, []),
}

STRUCTS = {0: Csr, 1: Opts, 2: PlanStats, 3: PlanDump, 4: Work, 5: AdaptState}

_lib = None


class SpmmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("spmm status %d: %s" % (status, msg))
        self.status = status


def load():
    """Load the built library.  There is no fallback: without ``libspmm.so``
    this raises, naming the build step."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libspmm.so is not built (%s); run __graft_entry__.build() or "
                           "python -m paper_2606_22482_amd.build" % LIB_PATH)
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    for which, st in STRUCTS.items():
        if lib.spmm_sizeof(which) != C.sizeof(st):
            raise RuntimeError("ABI mismatch for %s: C %d vs ctypes %d"
                               % (st.__name__, lib.spmm_sizeof(which), C.sizeof(st)))
    _lib = lib
    return lib


def check(status):
    if status != SPMM_OK:
        lib = load()
        raise SpmmError(status, lib.spmm_last_error().decode(errors="replace"))
    return status
