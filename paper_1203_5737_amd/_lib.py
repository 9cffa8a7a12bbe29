"""ctypes view of libargcsr.so (the C ABI declared in include/argcsr.h).

There is no fallback: if the library is missing or fails to load, every
entry point raises.  Build it with ``python -m paper_1203_5737_amd.build``.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libargcsr.so")

OK, EINVAL, EOVERFLOW, ENOMEM, EHIP, EBUDGET, EBUSY, ENOTFOUND, EUNSUPPORTED, ENOCONV = (
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9)
PENDING = 1
PROBE_SINK = 16384                    # ARGCSR_PROBE_SINK
CSR_BINS = 8                          # ARGCSR_CSR_BINS
REQ_ADMIT, REQ_SPMV, REQ_CG, REQ_EVICT = 0, 1, 2, 3
F64, F32, BF16, F16 = 0, 1, 2, 3
FORMAT_ARG, FORMAT_RG = 0, 1          # argcsr_format

_NAMES = {OK: "OK", EINVAL: "EINVAL", EOVERFLOW: "EOVERFLOW", ENOMEM: "ENOMEM", EHIP: "EHIP",
          EBUDGET: "EBUDGET", EBUSY: "EBUSY", ENOTFOUND: "ENOTFOUND", EUNSUPPORTED: "EUNSUPPORTED",
          ENOCONV: "ENOCONV"}


class ArgCsrError(RuntimeError):
    def __init__(self, code: int, where: str, message: str):
        super().__init__(f"{where}: {_NAMES.get(code, code)} ({code}): {message}")
        self.code = code


class GroupInfo(ctypes.Structure):
    _fields_ = [("first_row", ctypes.c_int32), ("size", ctypes.c_int32),
                ("offset", ctypes.c_int32), ("chunk_size", ctypes.c_int32)]


class MatrixDesc(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int32), ("n_cols", ctypes.c_int32),
                ("block_dim", ctypes.c_int32), ("desired_chunk_size", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("n_groups", ctypes.c_int32),
                ("nnz", ctypes.c_int64), ("n_slots", ctypes.c_int64),
                ("groups", ctypes.c_void_p), ("threads_mapping", ctypes.c_void_p),
                ("columns", ctypes.c_void_p), ("values", ctypes.c_void_p),
                ("n_heavy", ctypes.c_int32), ("heavy_chunk", ctypes.c_int32),
                ("heavy_groups", ctypes.c_void_p),
                ("format", ctypes.c_int32), ("region_rows", ctypes.c_int32),
                ("region_desired", ctypes.c_void_p),
                ("stage_gap", ctypes.c_int32), ("n_stage_tiles", ctypes.c_int32),
                ("stage_max_tiles", ctypes.c_int32), ("stage_lds", ctypes.c_int32),
                ("tile_ptr", ctypes.c_void_p), ("tile_start", ctypes.c_void_p),
                ("tile_len", ctypes.c_void_p), ("local", ctypes.c_void_p)]


class TuneResult(ctypes.Structure):
    _fields_ = [("block_dim", ctypes.c_int32), ("desired_chunk_size", ctypes.c_int32),
                ("model_us", ctypes.c_double), ("measured_us", ctypes.c_double),
                ("from_cache", ctypes.c_int32), ("n_candidates", ctypes.c_int32),
                ("n_timed", ctypes.c_int32), ("format", ctypes.c_int32),
                ("staged", ctypes.c_int32)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("max_active", ctypes.c_int32),
                ("device", ctypes.c_int32), ("block_dim", ctypes.c_int32),
                ("desired_chunk_size", ctypes.c_int32), ("cg_tol", ctypes.c_double),
                ("cg_inner_tol", ctypes.c_double), ("cg_max_inner", ctypes.c_int32),
                ("cg_max_iter", ctypes.c_int32), ("staging_bytes", ctypes.c_int64),
                ("cg_inner_per_step", ctypes.c_int32)]


class Request(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_rows", ctypes.c_int32), ("n_cols", ctypes.c_int32),
                ("matrix_id", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("val", ctypes.c_void_p), ("in_", ctypes.c_void_p),
                ("out", ctypes.c_void_p)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32),
                ("refinements", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("relres", ctypes.c_double), ("t_submit_ns", ctypes.c_int64),
                ("t_start_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "submitted", "completed", "failed", "admissions", "evictions", "steps",
        "resident_matrices", "resident_bytes", "arena_bytes")]


_lib = None
i32, i64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
pi32 = ctypes.POINTER(i32)

SIGNATURES = {
    "argcsr_last_error": (ctypes.c_char_p, []),
    "argcsr_version": (ctypes.c_int, []),
    "argcsr_plan": (ctypes.c_int, [i32, vp, i32, i32, i32, ctypes.POINTER(i32),
                                   ctypes.POINTER(i64), ctypes.POINTER(i32)]),
    "argcsr_plan_regions": (ctypes.c_int, [i32, vp, i32, i32, vp, ctypes.POINTER(i32),
                                           ctypes.POINTER(i64), ctypes.POINTER(i32)]),
    "argcsr_choose_region_desired": (ctypes.c_int, [i32, vp, i32, i32, vp]),
    "argcsr_plan_device": (ctypes.c_int, [i32, vp, i32, i32, i32, ctypes.POINTER(i32),
                                          ctypes.POINTER(i64), ctypes.POINTER(i32), vp]),
    "argcsr_convert": (ctypes.c_int, [i32, i32, vp, vp, vp, vp, ctypes.POINTER(MatrixDesc), vp]),
    "argcsr_plan_device_keep": (ctypes.c_int, [i32, vp, i32, i32, i32, ctypes.POINTER(i32),
                                               ctypes.POINTER(i64), ctypes.POINTER(i32),
                                               ctypes.POINTER(vp), vp]),
    "argcsr_convert_planned": (ctypes.c_int, [vp, i32, vp, vp, vp, ctypes.POINTER(MatrixDesc),
                                              vp]),
    "argcsr_device_plan_destroy": (ctypes.c_int, [vp]),
    "argcsr_convert_noalloc": (ctypes.c_int, [i32, i32, vp, vp, vp, vp,
                                              ctypes.POINTER(MatrixDesc), vp]),
    "argcsr_stage_plan": (ctypes.c_int, [ctypes.POINTER(MatrixDesc), i32, vp, ctypes.POINTER(i32),
                                         ctypes.POINTER(i32), vp]),
    "argcsr_stage": (ctypes.c_int, [ctypes.POINTER(MatrixDesc), vp]),
    "argcsr_spmv": (ctypes.c_int, [ctypes.POINTER(MatrixDesc), vp, vp, vp]),
    "argcsr_csr_spmv": (ctypes.c_int, [i32, i32, i64, vp, vp, vp, i32, i32, vp, vp, vp]),
    "argcsr_csr_bin_rows": (ctypes.c_int, [i32, vp, vp, vp, vp]),
    "argcsr_csr_spmv_binned": (ctypes.c_int, [i32, i32, i64, vp, vp, vp, i32, vp, vp, vp, vp,
                                              vp]),
    "argcsr_batch_create": (ctypes.c_int, [i32, ctypes.POINTER(MatrixDesc), ctypes.POINTER(vp),
                                           ctypes.POINTER(vp), ctypes.POINTER(vp)]),
    "argcsr_batch_graph_launch": (ctypes.c_int, [vp, vp]),
    "argcsr_batch_launch": (ctypes.c_int, [vp, vp]),
    "argcsr_batch_info": (ctypes.c_int, [vp, pi32, pi32, pi32]),
    "argcsr_batch_destroy": (ctypes.c_int, [vp]),
    "argcsr_autotune": (ctypes.c_int, [i32, i32, vp, vp, vp, vp, i32, i32,
                                       ctypes.POINTER(TuneResult), vp]),
    "argcsr_autotune_member": (ctypes.c_int, [i32, vp, i32, ctypes.POINTER(TuneResult)]),
    "argcsr_autotune_clear_cache": (ctypes.c_int, []),
    "argcsr_probe_read": (ctypes.c_int, [vp, i64, vp, vp]),
    "argcsr_probe_gather": (ctypes.c_int, [vp, i64, vp, i32, i32, vp, vp]),
    "argcsr_server_create": (ctypes.c_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(vp)]),
    "argcsr_server_submit": (ctypes.c_int, [vp, ctypes.POINTER(Request),
                                            ctypes.POINTER(ctypes.c_uint64)]),
    "argcsr_server_poll": (ctypes.c_int, [vp, ctypes.c_uint64, ctypes.POINTER(Result)]),
    "argcsr_server_wait": (ctypes.c_int, [vp, ctypes.c_uint64, i64, ctypes.POINTER(Result)]),
    "argcsr_server_release": (ctypes.c_int, [vp, ctypes.c_uint64]),
    "argcsr_server_get_stats": (ctypes.c_int, [vp, ctypes.POINTER(ServerStats)]),
    "argcsr_server_destroy": (ctypes.c_int, [vp]),
}


def lib():
    """The loaded library; raises if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is not built; run `python -m paper_1203_5737_amd.build` "
                "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code: int, where: str) -> None:
    if code != OK:
        msg = lib().argcsr_last_error()
        raise ArgCsrError(code, where, msg.decode() if msg else "")
