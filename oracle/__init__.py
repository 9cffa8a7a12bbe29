"""CPU oracle for ARG-CSR SpMV (FP64, plain sequential C).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are its only users.  The product library never imports it,
and this module shares no code with it.

Paper: Heller & Oberhuber, "Adaptive Row-grouped CSR format for storing of
sparse matrices on GPU" (arXiv:1203.5737) -- Sec. 2 (CSR), Sec. 3 (format,
Listing 1, conversion), Sec. 4 (Listing 2, SpMV semantics).  The readings R1-R8
of points the paper leaves open are listed in oracle.h.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

F64, F32, BF16, F16 = 0, 1, 2, 3
DTYPE_BYTES = {F64: 8, F32: 4, BF16: 2, F16: 2}
_NP_STORAGE = {F64: np.float64, F32: np.float32, BF16: np.uint16, F16: np.uint16}


def build_oracle() -> str:
    """Compile oracle.c with gcc (FP contraction off, OpenMP for the row split)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_oracle()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


def _bind(L):
    i32, i64, u16, f64, vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint16,
                              ctypes.c_double, ctypes.c_void_p)
    sig = {
        "ora_csr_spmv": (None, [i32, vp, vp, vp, vp, vp, i32]),
        "ora_csr_check": (ctypes.c_int, [i32, i32, i64, vp, vp]),
        "ora_group_rows": (ctypes.c_int, [i32, vp, i32, i32, vp, vp, vp]),
        "ora_chunk_size": (i32, [i32, vp, i32, vp]),
        "ora_argcsr_sizes": (ctypes.c_int, [i32, vp, i32, i32, vp, vp]),
        "ora_argcsr_convert": (ctypes.c_int, [i32, vp, vp, vp, i32, i32, i32, vp, vp, vp, vp]),
        "ora_group_rows_regions": (ctypes.c_int, [i32, vp, i32, i32, vp, vp, vp, vp]),
        "ora_argcsr_sizes_regions": (ctypes.c_int, [i32, vp, i32, i32, vp, vp, vp]),
        "ora_argcsr_convert_regions": (ctypes.c_int, [i32, vp, vp, vp, i32, i32, vp, i32, vp, vp,
                                                      vp, vp]),
        "ora_rgcsr_sizes": (ctypes.c_int, [i32, vp, i32, vp, vp]),
        "ora_rgcsr_convert": (ctypes.c_int, [i32, vp, vp, vp, i32, i32, vp, vp, vp, vp]),
        "ora_argcsr_spmv": (None, [i32, vp, vp, vp, vp, i32, vp, vp]),
        "ora_argcsr_to_csr": (i64, [i32, i32, vp, vp, vp, vp, i32, vp, vp, vp]),
        "ora_round_bf16": (u16, [f64]),
        "ora_round_f16": (u16, [f64]),
        "ora_bf16_value": (f64, [u16]),
        "ora_f16_value": (f64, [u16]),
        "ora_cg": (i32, [i32, vp, vp, vp, vp, vp, f64, i32, vp]),
        "ora_round_array": (None, [i64, vp, i32, vp]),
        "ora_stage": (i64, [i32, vp, vp, i32, i32, i32, vp, vp, vp, i64, vp]),
        "ora_unstage": (None, [i32, vp, i32, vp, vp, vp, vp]),
        "ora_decode_array": (None, [i64, vp, i32, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


@dataclass
class ArgCsr:
    """ARG-CSR arrays as the oracle produces them (Listing 1 + Sec. 3)."""
    n_rows: int
    block_dim: int
    desired_chunk_size: int
    dtype: int
    groups: np.ndarray      # int32 [G, 4] = firstRow, size, offset, chunkSize
    tm: np.ndarray          # int32 [n_rows] threadsMapping (inclusive per group)
    columns: np.ndarray     # int32 [S], -1 = artificial zero
    values: np.ndarray      # [S] float64 / float32 / uint16 bits (bf16, f16)

    @property
    def n_groups(self) -> int:
        return int(self.groups.shape[0])

    @property
    def n_slots(self) -> int:
        return int(self.columns.shape[0])


def csr_spmv(rp, col, val, x, n_threads: int = 1) -> np.ndarray:
    rp, col, val, x = _c(rp, np.int32), _c(col, np.int32), _c(val, np.float64), _c(x, np.float64)
    n = rp.shape[0] - 1
    y = np.empty(n, dtype=np.float64)
    lib().ora_csr_spmv(n, _p(rp), _p(col), _p(val), _p(x), _p(y), int(n_threads))
    return y


def csr_check(n_rows, n_cols, rp, col) -> int:
    rp, col = _c(rp, np.int32), _c(col, np.int32)
    return lib().ora_csr_check(n_rows, n_cols, int(col.shape[0]), _p(rp), _p(col))


def group_rows(rp, block_dim: int, desired_chunk_size: int):
    rp = _c(rp, np.int32)
    n = rp.shape[0] - 1
    first = np.empty(max(n, 1), dtype=np.int32)
    size = np.empty(max(n, 1), dtype=np.int32)
    g = ctypes.c_int32(0)
    rc = lib().ora_group_rows(n, _p(rp), block_dim, desired_chunk_size, _p(first), _p(size),
                              ctypes.byref(g))
    if rc != 0:
        raise ValueError(f"ora_group_rows failed: {rc}")
    return first[: g.value].copy(), size[: g.value].copy()


def chunk_size(row_lengths, block_dim: int):
    L = _c(row_lengths, np.int64)
    t = np.empty(max(block_dim, 1), dtype=np.int32)
    c = lib().ora_chunk_size(int(L.shape[0]), _p(L), block_dim, _p(t))
    return int(c), t[: L.shape[0]].copy()


def sizes(rp, block_dim: int, desired_chunk_size: int):
    rp = _c(rp, np.int32)
    g, s = ctypes.c_int32(0), ctypes.c_int64(0)
    rc = lib().ora_argcsr_sizes(rp.shape[0] - 1, _p(rp), block_dim, desired_chunk_size,
                                ctypes.byref(g), ctypes.byref(s))
    return rc, g.value, s.value


def convert(rp, col, val, block_dim: int, desired_chunk_size: int, dtype: int = F64) -> ArgCsr:
    rp, col, val = _c(rp, np.int32), _c(col, np.int32), _c(val, np.float64)
    n = rp.shape[0] - 1
    rc, G, S = sizes(rp, block_dim, desired_chunk_size)
    if rc != 0:
        raise OverflowError(f"ora_argcsr_sizes failed: {rc}")
    groups = np.empty((G, 4), dtype=np.int32)
    tm = np.empty(n, dtype=np.int32)
    columns = np.empty(S, dtype=np.int32)
    values = np.empty(S, dtype=_NP_STORAGE[dtype])
    rc = lib().ora_argcsr_convert(n, _p(rp), _p(col), _p(val), block_dim, desired_chunk_size,
                                  dtype, _p(groups), _p(tm), _p(columns), _p(values))
    if rc != 0:
        raise ValueError(f"ora_argcsr_convert failed: {rc}")
    return ArgCsr(n, block_dim, desired_chunk_size, dtype, groups, tm, columns, values)


def sizes_regions(rp, block_dim: int, region_rows: int, desired):
    """(rc, groups, slots) with desired[w] for rows [w*region_rows, ...) (reading R10)."""
    rp, d = _c(rp, np.int32), _c(desired, np.int32)
    g, s = ctypes.c_int32(0), ctypes.c_int64(0)
    rc = lib().ora_argcsr_sizes_regions(rp.shape[0] - 1, _p(rp), block_dim, region_rows, _p(d),
                                        ctypes.byref(g), ctypes.byref(s))
    return rc, g.value, s.value


def convert_regions(rp, col, val, block_dim: int, region_rows: int, desired,
                    dtype: int = F64) -> ArgCsr:
    """CSR -> ARG-CSR with a desiredChunkSize per region of rows (reading R10);
    desired_chunk_size is reported as 0."""
    rp, col, val, d = _c(rp, np.int32), _c(col, np.int32), _c(val, np.float64), _c(desired, np.int32)
    n = rp.shape[0] - 1
    rc, G, S = sizes_regions(rp, block_dim, region_rows, d)
    if rc != 0:
        raise ValueError(f"ora_argcsr_sizes_regions failed: {rc}")
    groups = np.empty((G, 4), dtype=np.int32)
    tm = np.empty(n, dtype=np.int32)
    columns = np.empty(S, dtype=np.int32)
    values = np.empty(S, dtype=_NP_STORAGE[dtype])
    rc = lib().ora_argcsr_convert_regions(n, _p(rp), _p(col), _p(val), block_dim, region_rows,
                                          _p(d), dtype, _p(groups), _p(tm), _p(columns),
                                          _p(values))
    if rc != 0:
        raise ValueError(f"ora_argcsr_convert_regions failed: {rc}")
    return ArgCsr(n, block_dim, 0, dtype, groups, tm, columns, values)


def rg_sizes(rp, block_dim: int):
    """(rc, groups, slots) of the row-grouped CSR storage (reading R9)."""
    rp = _c(rp, np.int32)
    g, s = ctypes.c_int32(0), ctypes.c_int64(0)
    rc = lib().ora_rgcsr_sizes(rp.shape[0] - 1, _p(rp), block_dim, ctypes.byref(g),
                               ctypes.byref(s))
    return rc, g.value, s.value


def rg_convert(rp, col, val, block_dim: int, dtype: int = F64) -> ArgCsr:
    """CSR -> row-grouped CSR (reading R9) in the ARG-CSR arrays
    (desired_chunk_size is reported as 0: it plays no part)."""
    rp, col, val = _c(rp, np.int32), _c(col, np.int32), _c(val, np.float64)
    n = rp.shape[0] - 1
    rc, G, S = rg_sizes(rp, block_dim)
    if rc != 0:
        raise OverflowError(f"ora_rgcsr_sizes failed: {rc}")
    groups = np.empty((G, 4), dtype=np.int32)
    tm = np.empty(n, dtype=np.int32)
    columns = np.empty(S, dtype=np.int32)
    values = np.empty(S, dtype=_NP_STORAGE[dtype])
    rc = lib().ora_rgcsr_convert(n, _p(rp), _p(col), _p(val), block_dim, dtype, _p(groups),
                                 _p(tm), _p(columns), _p(values))
    if rc != 0:
        raise ValueError(f"ora_rgcsr_convert failed: {rc}")
    return ArgCsr(n, block_dim, 0, dtype, groups, tm, columns, values)


def values_as_f64(a: ArgCsr) -> np.ndarray:
    """Exact FP64 value of every stored slot (bf16/f16 decoded from bits)."""
    return stored_as_f64(a.values, a.dtype)


def argcsr_spmv(a: ArgCsr, x) -> np.ndarray:
    x = _c(x, np.float64)
    vals = _c(values_as_f64(a), np.float64)
    y = np.zeros(a.n_rows, dtype=np.float64)
    lib().ora_argcsr_spmv(a.n_groups, _p(a.groups), _p(a.tm), _p(a.columns), _p(vals),
                          a.block_dim, _p(x), _p(y))
    return y


@dataclass
class Staging:
    """Staging of x for a converted matrix (reading R11, oracle.h)."""
    tile_ptr: np.ndarray     # int32 [G+1]
    tile_start: np.ndarray   # int32 [n_tiles] first column of each tile
    tile_len: np.ndarray     # int32 [n_tiles] columns in each tile (1..64)
    local: np.ndarray        # uint16 [S] 64*q + (c - tile_start), 0xFFFF = artificial zero

    @property
    def n_tiles(self) -> int:
        return int(self.tile_start.shape[0])

    def max_tiles(self) -> int:
        return int(np.diff(self.tile_ptr).max()) if self.tile_ptr.size > 1 else 0


STAGE_TOO_MANY_TILES = -1      # ORA_EINVAL: a group needs more than max_tiles tiles


def stage(a: ArgCsr, gap: int, max_tiles: int):
    """Windows and tiles of x per group and the 16-bit local column of every
    slot (ora_stage); returns a Staging, or STAGE_TOO_MANY_TILES."""
    g, c = _c(a.groups, np.int32), _c(a.columns, np.int32)
    tile_ptr = np.zeros(a.n_groups + 1, dtype=np.int32)
    n = lib().ora_stage(a.n_groups, _p(g), _p(c), a.block_dim, int(gap), int(max_tiles),
                        _p(tile_ptr), None, None, 0, None)
    if n < 0:
        if n == STAGE_TOO_MANY_TILES:
            return STAGE_TOO_MANY_TILES
        raise ValueError(f"ora_stage failed: {n}")
    ts = np.zeros(max(n, 1), dtype=np.int32)
    tl = np.zeros(max(n, 1), dtype=np.int32)
    local = np.zeros(max(a.n_slots, 1), dtype=np.uint16)
    n2 = lib().ora_stage(a.n_groups, _p(g), _p(c), a.block_dim, int(gap), int(max_tiles),
                         _p(tile_ptr), _p(ts), _p(tl), n, _p(local))
    if n2 != n:
        raise ValueError(f"ora_stage failed: {n2}")
    return Staging(tile_ptr, ts[:n].copy(), tl[:n].copy(), local[:a.n_slots].copy())


def unstage(a: ArgCsr, st: Staging) -> np.ndarray:
    """The column index every slot names, from its local index (ora_unstage)."""
    out = np.empty(max(a.n_slots, 1), dtype=np.int32)
    ts = st.tile_start if st.tile_start.size else np.zeros(1, np.int32)
    lib().ora_unstage(a.n_groups, _p(_c(a.groups, np.int32)), a.block_dim,
                      _p(_c(st.tile_ptr, np.int32)), _p(_c(ts, np.int32)),
                      _p(_c(st.local if st.local.size else np.zeros(1, np.uint16), np.uint16)),
                      _p(out))
    return out[:a.n_slots]


def argcsr_to_csr(a: ArgCsr, nnz_capacity: int):
    vals = _c(values_as_f64(a), np.float64)
    rp = np.empty(a.n_rows + 1, dtype=np.int32)
    col = np.empty(max(nnz_capacity, 1), dtype=np.int32)
    val = np.empty(max(nnz_capacity, 1), dtype=np.float64)
    nnz = lib().ora_argcsr_to_csr(a.n_rows, a.n_groups, _p(a.groups), _p(a.tm), _p(a.columns),
                                  _p(vals), a.block_dim, _p(rp), _p(col), _p(val))
    if nnz < 0:
        raise ValueError(f"ora_argcsr_to_csr failed: {nnz}")
    return rp, col[:nnz].copy(), val[:nnz].copy()


def round_bf16(v: float) -> int:
    return int(lib().ora_round_bf16(float(v)))


def round_f16(v: float) -> int:
    return int(lib().ora_round_f16(float(v)))


def round_array(v, dtype: int) -> np.ndarray:
    """Stored representation of FP64 values (float32 / uint16 bits)."""
    v = _c(v, np.float64)
    out = np.empty(v.shape, dtype=_NP_STORAGE[dtype])
    lib().ora_round_array(v.size, _p(v), dtype, _p(out))
    return out


def stored_as_f64(stored: np.ndarray, dtype: int) -> np.ndarray:
    """Exact FP64 value of stored values (float32 / uint16 bits)."""
    st = _c(stored, _NP_STORAGE[dtype])
    out = np.empty(st.shape, dtype=np.float64)
    lib().ora_decode_array(st.size, _p(st), dtype, _p(out))
    return out


def cg(rp, col, val, b, tol: float = 1e-10, max_iter: int = 10000):
    rp, col, val, b = _c(rp, np.int32), _c(col, np.int32), _c(val, np.float64), _c(b, np.float64)
    n = rp.shape[0] - 1
    x = np.zeros(n, dtype=np.float64)
    rel = ctypes.c_double(0.0)
    it = lib().ora_cg(n, _p(rp), _p(col), _p(val), _p(b), _p(x), tol, max_iter, ctypes.byref(rel))
    return x, int(it), rel.value
