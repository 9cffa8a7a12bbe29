"""Python binding of the request server (argcsr_server_* in include/argcsr.h).

Marshalling only: the scheduler, the device memory arena, the conversion
and every SpMV / CG kernel run inside libargcsr.  Host arrays handed to a
request are kept referenced here until its ticket is released.
"""
from __future__ import annotations

import ctypes
import threading

import numpy as np

from . import _lib
from ._lib import (PENDING, REQ_ADMIT, REQ_CG, REQ_EVICT, REQ_SPMV, Request, Result,
                   ServerConfig, ServerStats, check, lib)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else ctypes.c_void_p(0)


class Server:
    def __init__(self, budget_bytes: int = 64 << 30, max_active: int = 64, device: int = 0,
                 block_dim: int = 0, desired_chunk_size: int = 0, cg_tol: float = 1e-10,
                 cg_inner_tol: float = 1e-5, cg_max_inner: int = 200, cg_max_iter: int = 5000,
                 staging_bytes: int = 0, cg_inner_per_step: int = 0):
        cfg = ServerConfig(int(budget_bytes), int(max_active), int(device), int(block_dim),
                           int(desired_chunk_size), float(cg_tol), float(cg_inner_tol),
                           int(cg_max_inner), int(cg_max_iter), int(staging_bytes),
                           int(cg_inner_per_step))
        self._h = ctypes.c_void_p(0)
        check(lib().argcsr_server_create(ctypes.byref(cfg), ctypes.byref(self._h)),
              "argcsr_server_create")
        self._keep = {}
        self._lock = threading.Lock()

    def _submit(self, req: Request, keep) -> int:
        t = ctypes.c_uint64(0)
        with self._lock:
            check(lib().argcsr_server_submit(self._h, ctypes.byref(req), ctypes.byref(t)),
                  "argcsr_server_submit")
            self._keep[t.value] = keep
        return t.value

    def admit(self, matrix_id: int, rp, col, val, n_cols: int) -> int:
        rp = np.ascontiguousarray(rp, dtype=np.int32)
        col = np.ascontiguousarray(col, dtype=np.int32)
        val = np.ascontiguousarray(val, dtype=np.float64)
        req = Request(REQ_ADMIT, rp.shape[0] - 1, int(n_cols), int(matrix_id), _p(rp), _p(col),
                      _p(val), None, None)
        return self._submit(req, (rp, col, val))

    def evict(self, matrix_id: int) -> int:
        return self._submit(Request(REQ_EVICT, 0, 0, int(matrix_id)), None)

    def spmv(self, matrix_id: int, x, n_rows: int):
        """Queues y = A x (FP32 values, x and y FP32); returns (ticket, y).
        The request states len(x) and n_rows; the server rejects it (EINVAL)
        unless they are the resident matrix's columns and rows."""
        x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1)
        y = np.empty(int(n_rows), dtype=np.float32)
        req = Request(REQ_SPMV, y.shape[0], x.shape[0], int(matrix_id), None, None, None,
                      _p(x), _p(y))
        return self._submit(req, (x, y)), y

    def cg(self, matrix_id: int, b):
        """Queues a CG solve A x = b (FP64 b, x); returns (ticket, x).  The
        server rejects it (EINVAL) unless len(b) is the matrix's size."""
        b = np.ascontiguousarray(b, dtype=np.float64).reshape(-1)
        x = np.empty_like(b)
        req = Request(REQ_CG, b.shape[0], b.shape[0], int(matrix_id), None, None, None,
                      _p(b), _p(x))
        return self._submit(req, (b, x)), x

    def poll(self, ticket: int) -> dict:
        r = Result()
        check(lib().argcsr_server_poll(self._h, ticket, ctypes.byref(r)), "argcsr_server_poll")
        return {k: getattr(r, k) for k, _ in Result._fields_}

    def wait(self, ticket: int, timeout_s: float = 60.0) -> dict:
        r = Result()
        rc = lib().argcsr_server_wait(self._h, ticket, int(timeout_s * 1e9), ctypes.byref(r))
        if rc != 0 and rc != _lib.EBUSY:
            check(rc, "argcsr_server_wait")
        return {k: getattr(r, k) for k, _ in Result._fields_}

    def release(self, ticket: int) -> None:
        check(lib().argcsr_server_release(self._h, ticket), "argcsr_server_release")
        with self._lock:
            self._keep.pop(ticket, None)

    def stats(self) -> dict:
        st = ServerStats()
        check(lib().argcsr_server_get_stats(self._h, ctypes.byref(st)), "argcsr_server_get_stats")
        return {k: getattr(st, k) for k, _ in ServerStats._fields_}

    def close(self) -> None:
        if self._h:
            check(lib().argcsr_server_destroy(self._h), "argcsr_server_destroy")
            self._h = ctypes.c_void_p(0)
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
