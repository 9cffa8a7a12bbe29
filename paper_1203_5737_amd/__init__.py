"""ARG-CSR sparse matrix-vector multiplication on AMD MI355X (gfx950).

Python binding of libargcsr (include/argcsr.h).  Every step of the path runs
in the library's HIP kernels; this module only marshals arguments.  PyTorch
provides device memory and streams.  The library must be built
(``python -m paper_1203_5737_amd.build``); there is no CPU fallback.

Method: Heller & Oberhuber, "Adaptive Row-grouped CSR format for storing of
sparse matrices on GPU" (arXiv:1203.5737), Sec. 3 (format and conversion)
and Sec. 4 (SpMV).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib as _lib_mod
from ._lib import (BF16, F16, F32, F64, FORMAT_ARG, FORMAT_RG, ArgCsrError, MatrixDesc,
                   TuneResult, check, lib)

__all__ = ["F64", "F32", "BF16", "F16", "ArgCsrError", "ArgCsrMatrix", "DeviceCsr",
           "plan", "convert", "stage", "spmv", "csr_spmv", "csr_bins", "csr_spmv_binned",
           "to_device_csr", "storage_dtype",
           "vector_dtype", "Batch", "autotune", "autotune_clear_cache"]

_STORAGE = {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16, F16: torch.float16}


def storage_dtype(dtype: int) -> torch.dtype:
    """torch dtype holding the stored values (bf16/f16 share their bit layout)."""
    return _STORAGE[dtype]


def vector_dtype(dtype: int) -> torch.dtype:
    """torch dtype of x and y: FP64 for the FP64 path, FP32 otherwise."""
    return torch.float64 if dtype == F64 else torch.float32


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() > 0 else 0)


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


@dataclass
class DeviceCsr:
    """A CSR matrix (Sec. 2) resident on the device, with a host copy of the
    row offsets (used when conversion step 1 runs on the host; the device
    grouping path needs only the device arrays)."""
    n_rows: int
    n_cols: int
    row_ptr_host: np.ndarray     # int32 [n_rows+1]
    row_ptr: torch.Tensor        # device int32 [n_rows+1]
    col: torch.Tensor            # device int32 [nnz]
    val: torch.Tensor            # device float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.col.numel())


def to_device_csr(row_ptr, col, val, n_cols: int, device="cuda") -> DeviceCsr:
    rp = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int32))
    return DeviceCsr(
        n_rows=int(rp.shape[0] - 1), n_cols=int(n_cols), row_ptr_host=rp,
        row_ptr=torch.from_numpy(rp).to(device),
        col=torch.from_numpy(np.ascontiguousarray(col, dtype=np.int32)).to(device),
        val=torch.from_numpy(np.ascontiguousarray(val, dtype=np.float64)).to(device))


@dataclass
class ArgCsrMatrix:
    """A converted matrix; the four arrays are device tensors it owns."""
    n_rows: int
    n_cols: int
    block_dim: int
    desired_chunk_size: int
    dtype: int
    n_groups: int
    nnz: int
    n_slots: int
    groups: torch.Tensor           # int32 [n_groups, 4]: firstRow, size, offset, chunkSize
    threads_mapping: torch.Tensor  # int32 [n_rows]
    columns: torch.Tensor          # int32 [n_slots]
    values: torch.Tensor           # storage_dtype(dtype) [n_slots]
    heavy_groups: Optional[torch.Tensor] = None   # int32 [n_heavy] launch schedule
    n_heavy: int = 0
    heavy_chunk: int = 0
    format: int = FORMAT_ARG                      # FORMAT_ARG or FORMAT_RG
    # staging of x (stage()): positions in the group's tiles replace columns
    stage_gap: int = -1
    stage_max_tiles: int = 0
    stage_lds: int = 1
    tile_ptr: Optional[torch.Tensor] = None       # int32 [n_groups+1]
    tile_start: Optional[torch.Tensor] = None     # int32 [n_tiles]
    tile_len: Optional[torch.Tensor] = None       # int32 [n_tiles]
    local: Optional[torch.Tensor] = None          # int16 bits of uint16 [n_slots]

    @property
    def n_stage_tiles(self) -> int:
        return 0 if self.tile_start is None else int(self.tile_start.numel())

    def desc(self) -> MatrixDesc:
        return MatrixDesc(self.n_rows, self.n_cols, self.block_dim, self.desired_chunk_size,
                          self.dtype, self.n_groups, self.nnz, self.n_slots,
                          _ptr(self.groups), _ptr(self.threads_mapping), _ptr(self.columns),
                          _ptr(self.values), self.n_heavy, self.heavy_chunk,
                          _ptr(self.heavy_groups), self.format, 0, None,
                          self.stage_gap, self.n_stage_tiles, self.stage_max_tiles,
                          self.stage_lds, _ptr(self.tile_ptr), _ptr(self.tile_start),
                          _ptr(self.tile_len),
                          _ptr(self.local) if self.local is not None else ctypes.c_void_p(0))

    def nbytes(self) -> int:
        ts = [self.groups, self.threads_mapping, self.columns, self.values, self.heavy_groups,
              self.tile_ptr, self.tile_start, self.tile_len, self.local]
        return sum(t.numel() * t.element_size() for t in ts if t is not None)


def plan(row_ptr_host, block_dim: int, desired_chunk_size: int, fmt: int = FORMAT_ARG):
    """(n_groups, n_slots, n_heavy) of the converted matrix (host only)."""
    rp = np.ascontiguousarray(np.asarray(row_ptr_host, dtype=np.int32))
    g, s, h = ctypes.c_int32(0), ctypes.c_int64(0), ctypes.c_int32(0)
    check(lib().argcsr_plan(int(rp.shape[0] - 1), rp.ctypes.data_as(ctypes.c_void_p),
                            int(block_dim), int(desired_chunk_size), int(fmt), ctypes.byref(g),
                            ctypes.byref(s), ctypes.byref(h)), "argcsr_plan")
    return g.value, s.value, h.value


def plan_regions(row_ptr_host, block_dim: int, region_rows: int, region_desired):
    """(n_groups, n_slots, n_heavy) with a desiredChunkSize per region of rows
    (argcsr_plan_regions)."""
    rp = np.ascontiguousarray(np.asarray(row_ptr_host, dtype=np.int32))
    d = np.ascontiguousarray(np.asarray(region_desired, dtype=np.int32))
    g, s, h = ctypes.c_int32(0), ctypes.c_int64(0), ctypes.c_int32(0)
    check(lib().argcsr_plan_regions(int(rp.shape[0] - 1), rp.ctypes.data_as(ctypes.c_void_p),
                                    int(block_dim), int(region_rows),
                                    d.ctypes.data_as(ctypes.c_void_p), ctypes.byref(g),
                                    ctypes.byref(s), ctypes.byref(h)), "argcsr_plan_regions")
    return g.value, s.value, h.value


def choose_region_desired(row_ptr_host, region_rows: int, max_desired: int = 64) -> np.ndarray:
    """desiredChunkSize per region of rows by the local regularity rule
    (argcsr_choose_region_desired)."""
    rp = np.ascontiguousarray(np.asarray(row_ptr_host, dtype=np.int32))
    n = int(rp.shape[0] - 1)
    out = np.zeros(max(1, -(-n // int(region_rows))), dtype=np.int32)
    check(lib().argcsr_choose_region_desired(n, rp.ctypes.data_as(ctypes.c_void_p),
                                             int(region_rows), int(max_desired),
                                             out.ctypes.data_as(ctypes.c_void_p)),
          "argcsr_choose_region_desired")
    return out[: -(-n // int(region_rows))] if n else out[:0]


def plan_device(row_ptr: torch.Tensor, block_dim: int, desired_chunk_size: int, stream=None,
                fmt: int = FORMAT_ARG):
    """(n_groups, n_slots, n_heavy) from a device row_ptr (argcsr_plan_device)."""
    if row_ptr.dtype != torch.int32 or not row_ptr.is_contiguous() or not row_ptr.is_cuda:
        raise ValueError("row_ptr must be a contiguous int32 device tensor")
    g, s, h = ctypes.c_int32(0), ctypes.c_int64(0), ctypes.c_int32(0)
    check(lib().argcsr_plan_device(int(row_ptr.numel() - 1), _ptr(row_ptr), int(block_dim),
                                   int(desired_chunk_size), int(fmt), ctypes.byref(g),
                                   ctypes.byref(s), ctypes.byref(h), _stream(stream)),
          "argcsr_plan_device")
    return g.value, s.value, h.value


def convert(A: DeviceCsr, block_dim: int = 64, desired_chunk_size: int = 1,
            dtype: int = F64, stream=None, schedule: bool = True,
            device_grouping: bool = False, fmt: int = FORMAT_ARG, region_rows: int = 0,
            region_desired=None, noalloc: bool = False, keep_plan: bool = False) -> ArgCsrMatrix:
    """CSR -> ARG-CSR (or, with fmt=FORMAT_RG, row-grouped CSR) on the GPU
    (argcsr_convert); allocates the result.  `schedule` also builds the
    heavy-group launch schedule.  With `device_grouping` step 1 runs on the
    device and the host copy of row_ptr is not used: steps 1-3 run twice
    (argcsr_plan_device, then argcsr_convert with row_ptr_host = NULL), or,
    with `keep_plan`, once, kept on the device between sizing and conversion
    (argcsr_plan_device_keep + argcsr_convert_planned).
    `region_desired` (with `region_rows`) gives ARG-CSR a desiredChunkSize
    per region of rows (argcsr_plan_regions; the sizes are planned on the
    host).  `noalloc` converts with argcsr_convert_noalloc (the library
    allocates no device memory; the result tensors are still allocated here,
    as the caller's outputs)."""
    if noalloc and device_grouping:
        raise ValueError("argcsr_convert_noalloc groups the rows on the host")
    if fmt == FORMAT_RG:
        desired_chunk_size = 0
    regions = None
    plan_h = None
    if region_desired is not None:
        regions = np.ascontiguousarray(np.asarray(region_desired, dtype=np.int32))
        desired_chunk_size = 0
        G, S, H = plan_regions(A.row_ptr_host, block_dim, region_rows, regions)
    elif device_grouping and keep_plan:
        if A.row_ptr.dtype != torch.int32 or not A.row_ptr.is_contiguous():
            raise ValueError("row_ptr must be a contiguous int32 device tensor")
        g, s_, h = ctypes.c_int32(0), ctypes.c_int64(0), ctypes.c_int32(0)
        plan_h = ctypes.c_void_p(0)
        check(lib().argcsr_plan_device_keep(A.n_rows, _ptr(A.row_ptr), int(block_dim),
                                            int(desired_chunk_size), int(fmt), ctypes.byref(g),
                                            ctypes.byref(s_), ctypes.byref(h),
                                            ctypes.byref(plan_h), _stream(stream)),
              "argcsr_plan_device_keep")
        G, S, H = g.value, s_.value, h.value
    elif device_grouping:
        G, S, H = plan_device(A.row_ptr, block_dim, desired_chunk_size, stream, fmt)
    else:
        G, S, H = plan(A.row_ptr_host, block_dim, desired_chunk_size, fmt)
    try:
        dev = A.row_ptr.device
        out = ArgCsrMatrix(
            A.n_rows, A.n_cols, int(block_dim), int(desired_chunk_size), int(dtype), G, A.nnz, S,
            torch.empty((G, 4), dtype=torch.int32, device=dev),
            torch.empty(A.n_rows, dtype=torch.int32, device=dev),
            torch.empty(S, dtype=torch.int32, device=dev),
            torch.empty(S, dtype=_STORAGE[dtype], device=dev),
            torch.empty(H, dtype=torch.int32, device=dev) if schedule else None,
            H if schedule else 0, 0, int(fmt))
        d = out.desc()
        if schedule and H == 0:
            d.heavy_groups = None
        if regions is not None:
            d.region_rows = int(region_rows)
            d.region_desired = regions.ctypes.data_as(ctypes.c_void_p)
        if plan_h is not None:
            check(lib().argcsr_convert_planned(plan_h, A.n_cols, _ptr(A.row_ptr), _ptr(A.col),
                                               _ptr(A.val), ctypes.byref(d), _stream(stream)),
                  "argcsr_convert_planned")
        else:
            rp_host = (None if device_grouping
                       else A.row_ptr_host.ctypes.data_as(ctypes.c_void_p))
            fn, name = ((lib().argcsr_convert_noalloc, "argcsr_convert_noalloc") if noalloc
                        else (lib().argcsr_convert, "argcsr_convert"))
            check(fn(A.n_rows, A.n_cols, rp_host, _ptr(A.row_ptr), _ptr(A.col), _ptr(A.val),
                     ctypes.byref(d), _stream(stream)), name)
    finally:
        if plan_h is not None:
            lib().argcsr_device_plan_destroy(plan_h)
    out.nnz = int(d.nnz)
    out.heavy_chunk = int(d.heavy_chunk)
    if not schedule:
        out.n_heavy = 0
    return out


def stage(A: ArgCsrMatrix, gap: int = 0, lds: bool = True, stream=None,
          keep_columns: bool = True) -> ArgCsrMatrix:
    """Staging of x for banded matrices (argcsr_stage_plan + argcsr_stage):
    returns a matrix sharing A's arrays plus the group tile tables and the
    16-bit positions that argcsr_spmv then reads instead of the columns.
    `lds` selects how the SpMV reads x (the group's tiles loaded into LDS
    first, or gathered from memory through the tile table); without
    `keep_columns` the result drops its reference to the column array."""
    dev = A.groups.device
    tile_ptr = torch.empty(A.n_groups + 1, dtype=torch.int32, device=dev)
    d = A.desc()
    nt, mx = ctypes.c_int32(0), ctypes.c_int32(0)
    check(lib().argcsr_stage_plan(ctypes.byref(d), int(gap), _ptr(tile_ptr), ctypes.byref(nt),
                                  ctypes.byref(mx), _stream(stream)), "argcsr_stage_plan")
    out = ArgCsrMatrix(**{f: getattr(A, f) for f in A.__dataclass_fields__})
    out.stage_gap, out.stage_max_tiles, out.stage_lds = int(gap), int(mx.value), int(bool(lds))
    out.tile_ptr = tile_ptr
    out.tile_start = torch.empty(nt.value, dtype=torch.int32, device=dev)
    out.tile_len = torch.empty(nt.value, dtype=torch.int32, device=dev)
    out.local = torch.empty(A.n_slots, dtype=torch.int16, device=dev)
    d = out.desc()
    check(lib().argcsr_stage(ctypes.byref(d), _stream(stream)), "argcsr_stage")
    if not keep_columns:
        out.columns = torch.empty(0, dtype=torch.int32, device=dev)
    return out


def spmv(A: ArgCsrMatrix, x: torch.Tensor, y: Optional[torch.Tensor] = None,
         stream=None) -> torch.Tensor:
    """y = A x (argcsr_spmv), enqueued on `stream`."""
    want = vector_dtype(A.dtype)
    if x.dtype != want or not x.is_contiguous() or x.numel() != A.n_cols:
        raise ValueError(f"x must be a contiguous {want} vector of length {A.n_cols}")
    if y is None:
        y = torch.empty(A.n_rows, dtype=want, device=x.device)
    elif y.dtype != want or not y.is_contiguous() or y.numel() != A.n_rows:
        raise ValueError(f"y must be a contiguous {want} vector of length {A.n_rows}")
    d = A.desc()
    check(lib().argcsr_spmv(ctypes.byref(d), _ptr(x), _ptr(y), _stream(stream)), "argcsr_spmv")
    return y


def csr_spmv(A: DeviceCsr, x: torch.Tensor, y: Optional[torch.Tensor] = None,
             values: Optional[torch.Tensor] = None, dtype: int = F64, lanes_per_row: int = 0,
             stream=None) -> torch.Tensor:
    """Plain CSR baseline y = A x (argcsr_csr_spmv).  `values` overrides A.val
    with a tensor of storage_dtype(dtype) (e.g. FP32 values)."""
    vals = A.val if values is None else values
    if dtype not in _STORAGE:
        raise ValueError(f"unknown dtype {dtype}")
    if vals.dtype != _STORAGE[dtype] or not vals.is_contiguous() or vals.numel() != A.nnz:
        raise ValueError(f"values must be a contiguous {_STORAGE[dtype]} vector of length {A.nnz}")
    want = vector_dtype(dtype)
    if x.dtype != want or not x.is_contiguous() or x.numel() != A.n_cols:
        raise ValueError(f"x must be a contiguous {want} vector of length {A.n_cols}")
    if y is None:
        y = torch.empty(A.n_rows, dtype=want, device=x.device)
    elif y.dtype != want or not y.is_contiguous() or y.numel() != A.n_rows:
        raise ValueError(f"y must be a contiguous {want} vector of length {A.n_rows}")
    if y.data_ptr() == x.data_ptr() and x.numel() > 0:
        raise ValueError("y must not alias x")
    check(lib().argcsr_csr_spmv(A.n_rows, A.n_cols, A.nnz, _ptr(A.row_ptr), _ptr(A.col),
                                _ptr(vals), int(dtype), int(lanes_per_row), _ptr(x), _ptr(y),
                                _stream(stream)), "argcsr_csr_spmv")
    return y


@dataclass
class CsrBins:
    """Rows of a CSR matrix grouped by length (argcsr_csr_bin_rows)."""
    rows: torch.Tensor           # device int32 [n_rows], bin by bin
    bin_start: np.ndarray        # host int32 [CSR_BINS + 1]


def csr_bins(A: DeviceCsr, stream=None) -> CsrBins:
    """Bins A's rows by length for csr_spmv_binned (argcsr_csr_bin_rows)."""
    rows = torch.empty(A.n_rows, dtype=torch.int32, device=A.row_ptr.device)
    start = np.zeros(_lib_mod.CSR_BINS + 1, dtype=np.int32)
    check(lib().argcsr_csr_bin_rows(A.n_rows, _ptr(A.row_ptr), _ptr(rows),
                                    start.ctypes.data_as(ctypes.c_void_p), _stream(stream)),
          "argcsr_csr_bin_rows")
    return CsrBins(rows, start)


def csr_spmv_binned(A: DeviceCsr, x: torch.Tensor, bins: CsrBins,
                    y: Optional[torch.Tensor] = None, values: Optional[torch.Tensor] = None,
                    dtype: int = F64, stream=None) -> torch.Tensor:
    """Plain CSR y = A x with a lane count per row-length bin
    (argcsr_csr_spmv_binned); arguments as for csr_spmv."""
    vals = A.val if values is None else values
    if dtype not in _STORAGE:
        raise ValueError(f"unknown dtype {dtype}")
    if vals.dtype != _STORAGE[dtype] or not vals.is_contiguous() or vals.numel() != A.nnz:
        raise ValueError(f"values must be a contiguous {_STORAGE[dtype]} vector of length {A.nnz}")
    want = vector_dtype(dtype)
    if x.dtype != want or not x.is_contiguous() or x.numel() != A.n_cols:
        raise ValueError(f"x must be a contiguous {want} vector of length {A.n_cols}")
    if y is None:
        y = torch.empty(A.n_rows, dtype=want, device=x.device)
    elif y.dtype != want or not y.is_contiguous() or y.numel() != A.n_rows:
        raise ValueError(f"y must be a contiguous {want} vector of length {A.n_rows}")
    if y.data_ptr() == x.data_ptr() and x.numel() > 0:
        raise ValueError("y must not alias x")
    if bins.rows.numel() != A.n_rows or bins.rows.dtype != torch.int32:
        raise ValueError("bins were not made for this matrix")
    st = np.ascontiguousarray(bins.bin_start, dtype=np.int32)
    check(lib().argcsr_csr_spmv_binned(A.n_rows, A.n_cols, A.nnz, _ptr(A.row_ptr), _ptr(A.col),
                                       _ptr(vals), int(dtype), _ptr(bins.rows),
                                       st.ctypes.data_as(ctypes.c_void_p), _ptr(x), _ptr(y),
                                       _stream(stream)), "argcsr_csr_spmv_binned")
    return y


class Batch:
    """Several converted matrices computed by one persistent launch
    (argcsr_batch_create); y_m = A_m x_m for every member.  The x and y
    tensors are bound at creation and must stay alive (the batch keeps
    references)."""

    def __init__(self, mats, xs, ys):
        if not (len(mats) == len(xs) == len(ys)) or not mats:
            raise ValueError("mats, xs and ys must be non-empty and of equal length")
        for A, x, y in zip(mats, xs, ys):
            want = vector_dtype(A.dtype)
            if x.dtype != want or y.dtype != want or x.numel() != A.n_cols or y.numel() != A.n_rows:
                raise ValueError("x/y do not match their matrix")
        self._keep = (list(mats), list(xs), list(ys))
        n = len(mats)
        descs = (MatrixDesc * n)(*[A.desc() for A in mats])
        xp = (ctypes.c_void_p * n)(*[_ptr(x).value for x in xs])
        yp = (ctypes.c_void_p * n)(*[_ptr(y).value for y in ys])
        self._h = ctypes.c_void_p(0)
        check(lib().argcsr_batch_create(n, descs, xp, yp, ctypes.byref(self._h)),
              "argcsr_batch_create")

    def launch(self, stream=None, graph: bool = True) -> None:
        fn = lib().argcsr_batch_graph_launch if graph else lib().argcsr_batch_launch
        check(fn(self._h, _stream(stream)), "argcsr_batch_launch")

    def info(self):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().argcsr_batch_info(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)),
              "argcsr_batch_info")
        return {"n_items": a.value, "n_heavy": b.value, "grid": c.value}

    def close(self) -> None:
        if self._h:
            check(lib().argcsr_batch_destroy(self._h), "argcsr_batch_destroy")
            self._h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PROBE_SINK_ELEMS = _lib_mod.PROBE_SINK


def probe_read(t: torch.Tensor, sink: torch.Tensor, stream=None) -> None:
    """Streams the bytes of device tensor `t` once (argcsr_probe_read); a
    ceiling measurement, not part of the SpMV path."""
    _check_sink(sink)
    if not t.is_contiguous() or not t.is_cuda:
        raise ValueError("t must be a contiguous device tensor")
    check(lib().argcsr_probe_read(_ptr(t), t.numel() * t.element_size(), _ptr(sink),
                                  _stream(stream)), "argcsr_probe_read")


def probe_gather(idx: torch.Tensor, x: torch.Tensor, sink: torch.Tensor, stream=None) -> None:
    """Reads the int32 index stream `idx` (e.g. a converted matrix's columns)
    and gathers x[idx] for idx >= 0 (argcsr_probe_gather); a ceiling
    measurement, not part of the SpMV path."""
    _check_sink(sink)
    if idx.dtype != torch.int32 or not idx.is_contiguous() or not idx.is_cuda:
        raise ValueError("idx must be a contiguous int32 device tensor")
    if x.dtype not in (torch.float64, torch.float32) or not x.is_contiguous() or not x.is_cuda:
        raise ValueError("x must be a contiguous FP64 or FP32 device tensor")
    check(lib().argcsr_probe_gather(_ptr(idx), idx.numel(), _ptr(x), x.numel(),
                                    x.element_size(), _ptr(sink), _stream(stream)),
          "argcsr_probe_gather")


def _check_sink(sink: torch.Tensor) -> None:
    if (sink.dtype != torch.float64 or not sink.is_contiguous() or not sink.is_cuda
            or sink.numel() < PROBE_SINK_ELEMS):
        raise ValueError(f"sink must be a contiguous FP64 device tensor of {PROBE_SINK_ELEMS}")


def autotune(A: DeviceCsr, dtype: int = F64, n_finalists: int = 4, stream=None) -> dict:
    """(block_dim, desired_chunk_size) for A (argcsr_autotune)."""
    r = TuneResult()
    check(lib().argcsr_autotune(A.n_rows, A.n_cols, A.row_ptr_host.ctypes.data_as(ctypes.c_void_p),
                                _ptr(A.row_ptr), _ptr(A.col), _ptr(A.val), int(dtype),
                                int(n_finalists), ctypes.byref(r),
                                _stream(stream) if n_finalists > 0 else ctypes.c_void_p(0)),
          "argcsr_autotune")
    return {k: getattr(r, k) for k, _ in TuneResult._fields_}


def autotune_member(row_ptr_host, dtype: int = F32) -> dict:
    """(block_dim, desired_chunk_size, format) for a matrix that runs as one
    member of a Batch (argcsr_autotune_member: the batch-throughput model,
    host only, nothing timed)."""
    rp = np.ascontiguousarray(np.asarray(row_ptr_host, dtype=np.int32))
    r = TuneResult()
    check(lib().argcsr_autotune_member(int(rp.shape[0] - 1), rp.ctypes.data_as(ctypes.c_void_p),
                                       int(dtype), ctypes.byref(r)), "argcsr_autotune_member")
    return {k: getattr(r, k) for k, _ in TuneResult._fields_}


def autotune_clear_cache() -> None:
    check(lib().argcsr_autotune_clear_cache(), "argcsr_autotune_clear_cache")
