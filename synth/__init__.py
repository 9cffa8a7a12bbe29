"""Seeded synthetic sparse matrices and vectors.

These generators serve both the oracle and the GPU path (tests, smoke check,
benchmark).  They contain none of the method's arithmetic: they only build CSR
input (Sec. 2 storage) and right-hand vectors.  The paper measured on ~1600
matrices from public collections (Sec. 5) which are not reproduced here; these
stand-ins mimic the families it discusses:

* 2D 5-point and 3D 27-point stencils -- the regular, finite-difference and
  structural matrices (Sec. 5);
* power-law row lengths with uniformly random columns -- the irregular circuit
  and optimisation matrices where the format gains most (Sec. 5);
* batches of small/medium matrices of mixed regularity, and shifted Laplacians
  for iterative solves.

Seeds: workload k draws from ``numpy.random.SeedSequence([12035737, k])``
spawned into a structure stream, a value stream and a vector stream.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED_BASE = 12035737


@dataclass
class Csr:
    n_rows: int
    n_cols: int
    rp: np.ndarray    # int32 [n_rows+1]
    col: np.ndarray   # int32 [nnz]
    val: np.ndarray   # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.rp.astype(np.int64))


def streams(*key: int):
    """Three independent generators (structure, values, vectors) for a key."""
    ss = np.random.SeedSequence([SEED_BASE, *key])
    a, b, c = ss.spawn(3)
    return np.random.default_rng(a), np.random.default_rng(b), np.random.default_rng(c)


def uniform_vector(n: int, rng: np.random.Generator, lo: float = -1.0, hi: float = 1.0):
    return rng.uniform(lo, hi, n)


# --------------------------------------------------------------------------
# stencils
# --------------------------------------------------------------------------

def _stencil(shape, offsets, value_fn):
    """CSR of a stencil on a grid with Dirichlet boundary (neighbours outside
    the grid are dropped).  ``offsets`` are per-axis displacement tuples;
    entries are emitted in increasing column order.  ``value_fn(k, rows,
    mask)`` returns the values of offset k for the rows where ``mask``."""
    shape = tuple(int(s) for s in shape)
    N = int(np.prod(shape))
    strides = [int(np.prod(shape[d + 1:])) for d in range(len(shape))]
    lin = [sum(o[d] * strides[d] for d in range(len(shape))) for o in offsets]
    order = np.argsort(lin, kind="stable")
    coords = np.unravel_index(np.arange(N, dtype=np.int64), shape)
    masks = []
    for k in order:
        m = np.ones(N, dtype=bool)
        for d in range(len(shape)):
            c = coords[d] + offsets[k][d]
            m &= (c >= 0) & (c < shape[d])
        masks.append(m)
    L = np.zeros(N, dtype=np.int64)
    for m in masks:
        L += m
    rp = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(L, out=rp[1:])
    nnz = int(rp[-1])
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    cursor = rp[:-1].copy()
    rows = np.arange(N, dtype=np.int64)
    for k, m in zip(order, masks):
        r = rows[m]
        pos = cursor[m]
        col[pos] = (r + lin[k]).astype(np.int32)
        val[pos] = value_fn(int(k), r, m)
        cursor[m] += 1
    return Csr(N, N, rp.astype(np.int32), col, val)


def _offsets(dim: int, kind: str):
    if kind == "star":          # 2*dim+1 point
        offs = [tuple([0] * dim)]
        for d in range(dim):
            for s in (-1, 1):
                o = [0] * dim
                o[d] = s
                offs.append(tuple(o))
        return offs
    grids = np.meshgrid(*[[-1, 0, 1]] * dim, indexing="ij")   # 3^dim point
    return [tuple(int(g.flat[i]) for g in grids) for i in range(3 ** dim)]


def laplace2d(nx: int, ny: int | None = None, diag: float = 4.0, off: float = -1.0) -> Csr:
    """5-point Laplacian on an ny x nx grid, row index i*nx + j."""
    ny = nx if ny is None else ny
    offs = _offsets(2, "star")
    return _stencil((ny, nx), offs, lambda k, r, m: diag if offs[k] == (0, 0) else off)


def stencil27_unit(n: int) -> Csr:
    """27-point stencil with 26 on the diagonal and -1 off it (n^3 grid)."""
    offs = _offsets(3, "box")
    return _stencil((n, n, n), offs, lambda k, r, m: 26.0 if offs[k] == (0, 0, 0) else -1.0)


def stencil27_weighted(n: int, rng: np.random.Generator) -> Csr:
    """27-point stencil on an n^3 grid with symmetric random couplings:
    w_pq = w_qp ~ U[0.5, 1.5], a_pq = -w_pq, a_pp = 1 + sum_q w_pq (strictly
    diagonally dominant, symmetric positive definite)."""
    shape = (n, n, n)
    N = n ** 3
    offs = _offsets(3, "box")
    strides = (n * n, n, 1)
    lin = [sum(o[d] * strides[d] for d in range(3)) for o in offs]
    pos_offs = sorted([k for k in range(len(offs)) if lin[k] > 0], key=lambda k: lin[k])
    weights = {k: rng.uniform(0.5, 1.5, N) for k in pos_offs}   # weight of edge (p, p+o)
    neg_of = {}
    for k in range(len(offs)):
        if lin[k] < 0:
            neg_of[k] = offs.index(tuple(-v for v in offs[k]))
    coords = np.unravel_index(np.arange(N, dtype=np.int64), shape)

    def valid(k):
        m = np.ones(N, dtype=bool)
        for d in range(3):
            c = coords[d] + offs[k][d]
            m &= (c >= 0) & (c < shape[d])
        return m

    diag = np.ones(N, dtype=np.float64)
    for k in sorted(range(len(offs)), key=lambda k: lin[k]):
        if lin[k] == 0:
            continue
        m = valid(k)
        r = np.nonzero(m)[0]
        w = weights[k][r] if lin[k] > 0 else weights[neg_of[k]][r + lin[k]]
        diag[r] += w

    def value_fn(k, r, m):
        if lin[k] == 0:
            return diag[r]
        if lin[k] > 0:
            return -weights[k][r]
        return -weights[neg_of[k]][r + lin[k]]

    return _stencil(shape, offs, value_fn)


def shifted_laplacian(kind: str, n_target: int, rng: np.random.Generator) -> Csr:
    """SPD shifted Laplacian: 2D 5-point on s x s (s = round(sqrt(n))) or 3D
    7-point on s^3 (s = round(cbrt(n))), Dirichlet, plus diag(d), d ~ U[0,1]."""
    if kind == "2d":
        s = max(2, int(round(np.sqrt(n_target))))
        shape, dim = (s, s), 2
    else:
        s = max(2, int(round(np.cbrt(n_target))))
        shape, dim = (s, s, s), 3
    N = int(np.prod(shape))
    d = rng.uniform(0.0, 1.0, N)
    offs = _offsets(dim, "star")
    centre = tuple([0] * dim)
    return _stencil(shape, offs,
                    lambda k, r, m: (2.0 * dim + d[r]) if offs[k] == centre else -1.0)


# --------------------------------------------------------------------------
# random-column matrices
# --------------------------------------------------------------------------

def distinct_columns(L: np.ndarray, n_cols: int, rng: np.random.Generator):
    """Row pointers and per-row sorted, distinct, uniformly random columns
    for row lengths L (each L_r <= n_cols)."""
    L = np.asarray(L, dtype=np.int64)
    n = L.shape[0]
    if np.any(L > n_cols):
        raise ValueError("row longer than the number of columns")
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(L, out=rp[1:])
    nnz = int(rp[-1])
    col = np.empty(nnz, dtype=np.int64)
    dense = np.nonzero(L * 4 > n_cols)[0]
    sparse_mask = np.ones(n, dtype=bool)
    sparse_mask[dense] = False
    for r in dense:                      # nearly full rows: draw without replacement
        col[rp[r]:rp[r + 1]] = np.sort(rng.choice(n_cols, int(L[r]), replace=False))
    sel_rows = np.nonzero(sparse_mask)[0]
    if sel_rows.size:
        Ls = L[sel_rows]
        row_of = np.repeat(sel_rows, Ls)
        pos = _positions(rp, sel_rows, Ls)
        c = rng.integers(0, n_cols, pos.shape[0])
        while True:
            key = row_of * n_cols + c
            order = np.argsort(key, kind="stable")
            ks = key[order]
            dup = np.nonzero(ks[1:] == ks[:-1])[0] + 1
            if dup.size == 0:
                break
            c[order[dup]] = rng.integers(0, n_cols, dup.size)
        col[pos] = c[order]          # rows keep their order; columns sorted
    return rp.astype(np.int32), col.astype(np.int32)


def _positions(rp, rows, Ls):
    starts = rp[rows]
    base = np.repeat(starts - np.concatenate([[0], np.cumsum(Ls)[:-1]]), Ls)
    return base + np.arange(int(Ls.sum()), dtype=np.int64)


def random_csr(L, n_cols: int, rng_struct, rng_val, lo=-1.0, hi=1.0) -> Csr:
    rp, col = distinct_columns(L, n_cols, rng_struct)
    val = rng_val.uniform(lo, hi, col.shape[0])
    return Csr(len(L), n_cols, rp, col, val)


def powerlaw(n: int, alpha: float, lmax: int, rng_struct, rng_val) -> Csr:
    """Row lengths clip(Zipf(alpha), 1, lmax) (clipped, not resampled), distinct
    uniform-random columns, values U[-1, 1]."""
    L = np.clip(rng_struct.zipf(alpha, n), 1, min(lmax, n)).astype(np.int64)
    return random_csr(L, n, rng_struct, rng_val)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def workload_laplace64():
    """2D 5-point Laplacian on 64x64 (n=4096, 20224 nnz), 4 / -1; x U[-1,1]."""
    s, v, xr = streams(0)
    A = laplace2d(64)
    return A, uniform_vector(A.n_cols, xr)


def workload_powerlaw(n: int = 1_000_000):
    """n rows, lengths clip(Zipf(2.0), 1, 10^4), values U[-1,1]; x U[-1,1]."""
    s, v, xr = streams(1)
    A = powerlaw(n, 2.0, 10_000, s, v)
    return A, uniform_vector(A.n_cols, xr)


def workload_stencil27(n: int = 128):
    """27-point stencil on n^3 with symmetric U[0.5,1.5] couplings; x U[-1,1]."""
    s, v, xr = streams(2)
    A = stencil27_weighted(n, v)
    return A, uniform_vector(A.n_cols, xr)


def workload_mixed(side: int = 64):
    """Rows of two kinds in one square matrix of n = 2*side^3 rows: the first
    side^3 rows are a 27-point stencil on a side^3 grid (regular rows, columns
    in the first half), the rest power-law rows (clip(Zipf(2.0), 1, 10^4),
    distinct uniform columns over all n) -- a matrix whose regularity
    changes between regions of rows; x U[-1,1]."""
    s, v, xr = streams(6)
    St = stencil27_weighted(side, v)
    m = St.n_rows
    n = 2 * m
    L = np.clip(s.zipf(2.0, m), 1, 10_000).astype(np.int64)
    P = random_csr(L, n, s, v)
    rp = np.concatenate([St.rp, St.rp[-1] + P.rp[1:]]).astype(np.int32)
    col = np.concatenate([St.col, P.col]).astype(np.int32)
    val = np.concatenate([St.val, P.val])
    A = Csr(n, n, rp, col, val)
    return A, uniform_vector(n, xr)


def batch_member(k: int, n_lo: float = 1e3, n_hi: float = 2e5):
    """Matrix k of the mixed batch: n log-uniform in [n_lo, n_hi]; even k has
    U{5..50} nonzeros per row, odd k clip(Zipf(2.2), 1, min(5000, n))."""
    s, v, xr = streams(3, k)
    n = int(round(np.exp(s.uniform(np.log(n_lo), np.log(n_hi)))))
    if k % 2 == 0:
        L = s.integers(5, 51, n)
        L = np.minimum(L, n)
    else:
        L = np.clip(s.zipf(2.2, n), 1, min(5000, n)).astype(np.int64)
    A = random_csr(L, n, s, v)
    return A, uniform_vector(n, xr)


def workload_batch(count: int = 256, n_lo: float = 1e3, n_hi: float = 2e5):
    return [batch_member(k, n_lo, n_hi) for k in range(count)]


def serve_pool_matrix(i: int, n_lo: float = 1e4, n_hi: float = 1e6):
    """Matrix i of the serving pool: 2D or 3D (50/50) shifted Laplacian with n
    log-uniform in [n_lo, n_hi]."""
    s, v, xr = streams(4, i)
    kind = "2d" if s.uniform() < 0.5 else "3d"
    n = int(round(np.exp(s.uniform(np.log(n_lo), np.log(n_hi)))))
    A = shifted_laplacian(kind, n, v)
    return A, kind
