"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these compares the oracle with itself: each check uses the paper's
worked example, a closed form, brute force, an invariant of the format, an
independent library routine (numpy, scipy, fractions) or an error bound.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U64 = 2.0 ** -53


def gamma(n, u=U64):
    return n * u / (1.0 - n * u)


def csr_from_rows(rows, n_cols):
    """rows: list of lists of (col, val)."""
    rp = np.zeros(len(rows) + 1, dtype=np.int32)
    cols, vals = [], []
    for i, r in enumerate(rows):
        for c, v in r:
            cols.append(c)
            vals.append(v)
        rp[i + 1] = len(cols)
    return rp, np.array(cols, dtype=np.int32), np.array(vals, dtype=np.float64)


def fig3_matrix():
    rows = [[(i, float(i + 1))] for i in range(7)] + [[(j, float(10 + j)) for j in range(8)]]
    return csr_from_rows(rows, 8)


# ---------------------------------------------------------------------------
# Worked example of Fig. 3 (Sec. 3)
# ---------------------------------------------------------------------------

def test_fig3_worked_example(ora):
    g = json.load(open(os.path.join(GOLDEN, "fig3_example.json")))
    paper, reading = g["stated_by_paper"], g["reading"]
    rp, col, val = fig3_matrix()
    L = np.diff(rp)
    T = paper["threads"]
    # one thread per row: chunk size = longest row, artificial zeros
    one = paper["one_thread_per_row"]
    assert L.max() == one["chunk_size"]
    assert len(L) * one["chunk_size"] - L.sum() == one["artificial_zeros"]
    # adaptive distribution
    c, t = ora.chunk_size(L, T)
    ad = paper["adaptive"]
    assert c == ad["chunk_size"]
    assert t[-1] == ad["threads_on_last_row"]
    assert T - t.sum() == ad["free_threads"]
    assert t.sum() * c - L.sum() == ad["artificial_zeros"]
    # full conversion under the readings
    a = ora.convert(rp, col, val, T, reading["desired_chunk_size"])
    assert a.n_groups == 1
    assert a.groups[0].tolist() == [0, 8, 0, 2]
    assert a.tm.tolist() == reading["threads_mapping_inclusive"]
    assert a.n_slots == reading["slots"]
    assert int((a.columns == -1).sum()) == reading["artificial_zeros_in_all_slots"]
    mapped = [a.columns[j * T + k] for k in range(a.tm[-1]) for j in range(c)]
    assert sum(1 for v in mapped if v == -1) == reading["artificial_zeros_in_mapped_chunks"]


def test_fig3_with_desired_chunk_size_one(ora):
    rp, col, val = fig3_matrix()
    a = ora.convert(rp, col, val, 12, 1)
    # D*T = 12: rows 0..6 (7 nonzeros) fit, row 7 (8 more) opens a new group
    assert a.groups.tolist() == [[0, 7, 0, 1], [7, 1, 12, 1]]
    assert a.tm.tolist() == [1, 2, 3, 4, 5, 6, 7, 8]


# ---------------------------------------------------------------------------
# Step 2 (chunk size) against brute force over all thread distributions
# ---------------------------------------------------------------------------

def brute_force_chunk(L, T):
    best = None
    for t in itertools.product(range(1, T + 1), repeat=len(L)):
        if sum(t) > T:
            continue
        m = max(max(-(-l // ti) for l, ti in zip(L, t)), 1)
        best = m if best is None else min(best, m)
    return best


def test_chunk_size_is_optimal_by_brute_force(ora):
    checked = 0
    for T in range(1, 8):
        for n in range(1, min(T, 4) + 1):
            for L in itertools.product(range(0, 7), repeat=n):
                c, t = ora.chunk_size(L, T)
                assert c == brute_force_chunk(L, T), (L, T)
                assert all(ti >= 1 for ti in t) and sum(t) <= T
                assert all(-(-l // ti) <= c for l, ti in zip(L, t))
                # minimal allocation for that chunk size
                assert all(ti == max(1, -(-l // c)) for l, ti in zip(L, t))
                checked += 1
    assert checked > 5000


# ---------------------------------------------------------------------------
# Closed-form layouts
# ---------------------------------------------------------------------------

def test_uniform_rows_give_sliced_ellpack_layout(ora):
    """Uniform row length L with desiredChunkSize = L: groups of T rows, one
    chunk per row, chunk size L -> the column-major ELLPACK slice of Sec. 2."""
    rng = np.random.default_rng(5)
    n, Lr, T = 300, 5, 64
    A = synth.random_csr(np.full(n, Lr), 1000, rng, rng)
    a = ora.convert(A.rp, A.col, A.val, T, Lr)
    assert a.n_groups == -(-n // T)
    for r in range(n):
        for e in range(Lr):
            slot = (r // T) * Lr * T + e * T + (r % T)
            assert a.columns[slot] == A.col[A.rp[r] + e]
            assert a.values[slot] == A.val[A.rp[r] + e]
    assert np.all(a.groups[:, 3] == Lr)


def test_diagonal_matrix(ora):
    n, T = 200, 64
    d = np.arange(1, n + 1, dtype=np.float64) * 0.37
    rp = np.arange(n + 1, dtype=np.int32)
    col = np.arange(n, dtype=np.int32)
    a = ora.convert(rp, col, d, T, 1)
    assert np.all(a.groups[:, 3] == 1)
    for g in a.groups:
        assert a.tm[g[0]:g[0] + g[1]].tolist() == list(range(1, g[1] + 1))
    x = np.random.default_rng(1).uniform(-1, 1, n)
    y = ora.argcsr_spmv(a, x)
    assert np.array_equal(y, d * x)          # one product per row: bitwise
    assert np.array_equal(ora.csr_spmv(rp, col, d, x), d * x)


def test_single_long_row(ora):
    """One row of 1000 nonzeros, T = 64: chunk 16, 63 chunks, last one holds 8."""
    L, T = 1000, 64
    rp = np.array([0, L], dtype=np.int32)
    col = np.arange(L, dtype=np.int32)
    val = np.ones(L)
    a = ora.convert(rp, col, val, T, 1)
    assert a.groups.tolist() == [[0, 1, 0, 16]]
    assert a.tm.tolist() == [63]
    last_chunk = [a.columns[j * T + 62] for j in range(16)]
    assert sum(1 for v in last_chunk if v != -1) == 8
    assert all(a.columns[j * T + 63] == -1 for j in range(16))     # one free chunk


def test_empty_matrix_and_empty_rows(ora):
    n, T = 150, 64
    rp = np.zeros(n + 1, dtype=np.int32)
    col = np.zeros(0, dtype=np.int32)
    val = np.zeros(0)
    a = ora.convert(rp, col, val, T, 1)
    assert a.n_groups == -(-n // T)
    assert np.all(a.groups[:, 3] == 1) and np.all(a.columns == -1)
    assert np.all(a.values == 0)
    x = np.ones(n)
    assert np.all(ora.argcsr_spmv(a, x) == 0) and np.all(ora.csr_spmv(rp, col, val, x) == 0)
    # zero rows
    a0 = ora.convert(np.zeros(1, dtype=np.int32), col, val, T, 1)
    assert a0.n_groups == 0 and a0.n_slots == 0


# ---------------------------------------------------------------------------
# Invariants of the format on random matrices
# ---------------------------------------------------------------------------

def check_invariants(A, a, T, D):
    n = A.n_rows
    L = A.row_lengths()
    G = a.n_groups
    # I1 groups contiguous, covering all rows in order
    assert a.groups[0, 0] == 0 if n else G == 0
    for g in range(G - 1):
        assert a.groups[g, 0] + a.groups[g, 1] == a.groups[g + 1, 0]
    if G:
        assert a.groups[-1, 0] + a.groups[-1, 1] == n
    # I2 sizes; I3 offsets
    assert np.all((a.groups[:, 1] >= 1) & (a.groups[:, 1] <= T))
    off = np.concatenate([[0], np.cumsum(a.groups[:, 3].astype(np.int64) * T)])
    assert np.array_equal(a.groups[:, 2], off[:-1]) and a.n_slots == off[-1]
    seen = np.zeros(A.nnz, dtype=np.int64)
    for g in range(G):
        f, s, o, c = (int(v) for v in a.groups[g])
        tm = a.tm[f:f + s].astype(np.int64)
        t = np.diff(np.concatenate([[0], tm]))
        # I4 strictly increasing, <= T, at least one chunk per row
        assert np.all(t >= 1) and tm[-1] <= T
        Lg = L[f:f + s]
        # I8 group nonzero budget unless a single row; I9 maximal
        assert Lg.sum() <= D * T or s == 1
        if f + s < n:
            assert s + 1 > T or Lg.sum() + L[f + s] > D * T
        # I10 chunk size minimal and allocation minimal
        need = lambda cc: int(np.maximum(1, -(-Lg // cc)).sum())
        assert need(c) <= T and (c == 1 or need(c - 1) > T)
        assert np.array_equal(t, np.maximum(1, -(-Lg // c)))
        # I5/I6/I7 every entry exactly once, valid before padding, padding (0,-1)
        for l in range(s):
            r = f + l
            b = 0 if l == 0 else int(tm[l - 1])
            for k in range(b, int(tm[l])):
                vals_seen = False
                for j in range(c):
                    slot = o + j * T + k
                    e = (k - b) * c + j
                    if e < L[r]:
                        assert not vals_seen
                        assert a.columns[slot] == A.col[A.rp[r] + e]
                        assert a.values[slot] == A.val[A.rp[r] + e]
                        seen[A.rp[r] + e] += 1
                    else:
                        vals_seen = True
                        assert a.columns[slot] == -1 and a.values[slot] == 0
        for k in range(int(tm[-1]), T):          # free chunks
            for j in range(c):
                assert a.columns[o + j * T + k] == -1
    assert np.all(seen == 1)


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(
    lengths=st.lists(st.integers(0, 40), min_size=0, max_size=90),
    T=st.sampled_from([1, 2, 3, 5, 8, 12, 16, 64]),
    D=st.integers(1, 6),
    seed=st.integers(0, 2 ** 31),
)
def test_invariants_random(ora, lengths, T, D, seed):
    rng = np.random.default_rng(seed)
    L = np.array(lengths, dtype=np.int64)
    A = synth.random_csr(L, 64, rng, rng) if len(L) else synth.Csr(
        0, 64, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    a = ora.convert(A.rp, A.col, A.val, T, D)
    check_invariants(A, a, T, D)
    rp, col, val = ora.argcsr_to_csr(a, A.nnz)
    assert np.array_equal(rp, A.rp) and np.array_equal(col, A.col)
    assert np.array_equal(val.view(np.uint64), A.val.view(np.uint64))


def test_invariants_powerlaw_sample(ora):
    s, v, _ = synth.streams(101)
    A = synth.powerlaw(3000, 2.0, 500, s, v)
    for T, D in [(64, 1), (64, 4), (128, 1), (256, 2)]:
        a = ora.convert(A.rp, A.col, A.val, T, D)
        check_invariants(A, a, T, D)


def test_round_trip_bit_exact_large(ora):
    A, _ = synth.workload_powerlaw(200_000)
    for T, D in [(64, 1), (256, 2)]:
        a = ora.convert(A.rp, A.col, A.val, T, D)
        rp, col, val = ora.argcsr_to_csr(a, A.nnz)
        assert np.array_equal(rp, A.rp) and np.array_equal(col, A.col)
        assert np.array_equal(val.view(np.uint64), A.val.view(np.uint64))


# ---------------------------------------------------------------------------
# SpMV: dense matvec, closed forms, exact rationals, library routine
# ---------------------------------------------------------------------------

def test_dense_matvec_small_integers_bitwise(ora):
    rng = np.random.default_rng(7)
    for n in [1, 2, 7, 33, 64]:
        for m in [1, 5, 64]:
            M = rng.integers(-9, 10, (n, m)).astype(np.float64)
            M[rng.random((n, m)) < 0.6] = 0
            x = rng.integers(-9, 10, m).astype(np.float64)
            rows = [[(j, M[i, j]) for j in range(m) if M[i, j] != 0] for i in range(n)]
            rp, col, val = csr_from_rows(rows, m)
            ref = M @ x
            assert np.array_equal(ora.csr_spmv(rp, col, val, x), ref)
            for T, D in [(1, 1), (4, 2), (12, 2), (64, 1)]:
                a = ora.convert(rp, col, val, T, D)
                assert np.array_equal(ora.argcsr_spmv(a, x), ref)


def laplace5_closed_form(nx, u):
    """y = A u for the 5-point stencil (4 / -1, Dirichlet): y = 4u - sum of the
    in-grid neighbours = -Laplacian_h(u) + sum of u at the missing neighbours."""
    y = np.zeros(nx * nx)
    for i in range(nx):
        for j in range(nx):
            v = 4 * u(i, j)
            for di, dj in [(-1, 0), (1, 0), (0, -1), (0, 1)]:
                if 0 <= i + di < nx and 0 <= j + dj < nx:
                    v -= u(i + di, j + dj)
            y[i * nx + j] = v
    return y


def test_laplace5_polynomials(ora):
    nx = 64
    A = synth.laplace2d(nx)
    assert A.nnz == 20224
    for u in [lambda i, j: 1.0, lambda i, j: float(i * i + j * j), lambda i, j: float(i * j + 3 * i)]:
        x = np.array([u(k // nx, k % nx) for k in range(nx * nx)])
        want = laplace5_closed_form(nx, u)
        # interior: the discrete Laplacian of i^2 + j^2 is exactly 4
        assert np.array_equal(ora.csr_spmv(A.rp, A.col, A.val, x), want)
        for T, D in [(64, 1), (64, 5), (128, 1), (256, 4)]:
            a = ora.convert(A.rp, A.col, A.val, T, D)
            assert np.array_equal(ora.argcsr_spmv(a, x), want)
    # u = i^2 + j^2: interior rows give exactly -4
    x = np.array([float((k // nx) ** 2 + (k % nx) ** 2) for k in range(nx * nx)])
    y = ora.csr_spmv(A.rp, A.col, A.val, x).reshape(nx, nx)
    assert np.all(y[1:-1, 1:-1] == -4.0)
    # u = 1: number of missing neighbours
    y1 = ora.csr_spmv(A.rp, A.col, A.val, np.ones(nx * nx)).reshape(nx, nx)
    assert y1[0, 0] == 2 and y1[0, 5] == 1 and y1[5, 5] == 0


def test_stencil27_unit_closed_form(ora):
    n = 12
    A = synth.stencil27_unit(n)
    i = np.arange(n ** 3) // (n * n)
    x = (i * i).astype(np.float64)
    y = ora.csr_spmv(A.rp, A.col, A.val, x).reshape(n, n, n)
    assert np.all(y[1:-1, 1:-1, 1:-1] == -18.0)       # -sum of d_i^2 over 26 neighbours
    y0 = ora.csr_spmv(A.rp, A.col, A.val, np.ones(n ** 3)).reshape(n, n, n)
    assert np.all(y0[1:-1, 1:-1, 1:-1] == 0.0)
    a = ora.convert(A.rp, A.col, A.val, 64, 27)
    assert np.array_equal(ora.argcsr_spmv(a, x).reshape(n, n, n), y)


def test_weighted_stencil_row_sums_to_one(ora):
    s, v, _ = synth.streams(2)
    A = synth.stencil27_weighted(16, v)
    y = ora.csr_spmv(A.rp, A.col, A.val, np.ones(A.n_cols))
    L = A.row_lengths()
    absum = np.abs(A.val)
    bound = gamma(L) * np.add.reduceat(absum, A.rp[:-1]) * 2
    assert np.all(np.abs(y - 1.0) <= bound)
    # symmetric, dominant
    M = sp.csr_matrix((A.val, A.col, A.rp), shape=(A.n_rows, A.n_cols))
    assert abs(M - M.T).max() == 0


def exact_row(A, x, r):
    s = Fraction(0)
    for k in range(A.rp[r], A.rp[r + 1]):
        s += Fraction(A.val[k]) * Fraction(x[A.col[k]])
    return s


def test_exact_rational_rows(ora):
    cases = [synth.workload_powerlaw(100_000), synth.workload_stencil27(20)]
    for A, x in cases:
        y = ora.csr_spmv(A.rp, A.col, A.val, x)
        L = A.row_lengths()
        rows = list(np.argsort(-L)[:20]) + list(np.random.default_rng(3).integers(0, A.n_rows, 60))
        for r in rows:
            ex = exact_row(A, x, r)
            abs_sum = sum(abs(A.val[k] * x[A.col[k]]) for k in range(A.rp[r], A.rp[r + 1]))
            err = abs(Fraction(y[r]) - ex)
            assert err <= Fraction(gamma(int(L[r])) * abs_sum * 1.0000001), r


def test_matches_scipy_within_bound(ora):
    A, x = synth.workload_powerlaw(50_000)
    M = sp.csr_matrix((A.val, A.col, A.rp), shape=(A.n_rows, A.n_cols))
    y_sp = M @ x
    y = ora.csr_spmv(A.rp, A.col, A.val, x)
    absum = np.abs(M) @ np.abs(x)
    L = A.row_lengths()
    assert np.all(np.abs(y - y_sp) <= 2 * gamma(np.maximum(L, 1)) * absum)
    # the OpenMP row split does not change a single bit
    assert np.array_equal(ora.csr_spmv(A.rp, A.col, A.val, x, n_threads=4), y)


def test_argcsr_order_matches_csr_definition(ora):
    A, x = synth.workload_powerlaw(100_000)
    y = ora.csr_spmv(A.rp, A.col, A.val, x)
    absum = np.add.reduceat(np.abs(A.val * x[A.col]), A.rp[:-1]) * (A.row_lengths() > 0)
    for T, D in [(64, 1), (128, 2), (256, 1)]:
        a = ora.convert(A.rp, A.col, A.val, T, D)
        ya = ora.argcsr_spmv(a, x)
        assert np.all(np.abs(ya - y) <= 1e-12 * absum)


def test_csr_check(ora):
    rp, col, val = fig3_matrix()
    assert ora.csr_check(8, 8, rp, col) == 0
    bad = col.copy()
    bad[3] = -1
    assert ora.csr_check(8, 8, rp, bad) != 0
    bad[3] = 8
    assert ora.csr_check(8, 8, rp, bad) != 0
    rp2 = rp.copy()
    rp2[3], rp2[4] = rp2[4], rp2[3]
    assert ora.csr_check(8, 8, rp2, col) != 0


def test_slot_overflow_is_reported(ora):
    """Rows of 65 nonzeros at blockDim 64, desiredChunkSize 1: each row is a
    group of its own with chunk size 2, i.e. 128 slots; 17M such rows need
    more than 2^31 - 1 slots although the CSR input itself fits int32."""
    n, L, T = 17_000_000, 65, 64
    rp = (np.arange(n + 1, dtype=np.int64) * L).astype(np.int32)
    rc, G, S = ora.sizes(rp, T, 1)
    assert S == n * 128 and rc == -2


# ---------------------------------------------------------------------------
# Reduced-precision rounding (nearest, ties to even, directly from FP64)
# ---------------------------------------------------------------------------

def special_doubles(rng):
    v = list(rng.uniform(-1, 1, 3000)) + list(rng.normal(0, 1e3, 1000))
    v += list(np.ldexp(rng.uniform(0.5, 1, 500), rng.integers(-150, 130, 500)))
    v += [0.0, -0.0, 1.0, -1.0, 65504.0, 65519.99, 65520.0, 70000.0, 6e-8, 5.96e-8, 2.98e-8,
          2.0 ** -24, 2.0 ** -25, 2.0 ** -25 * 1.0000001, 3.0 * 2.0 ** -26, 1e-300, 3.4e38, 3.39e38,
          1 + 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -40, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -11,
          1 + 2.0 ** -11 + 2.0 ** -45, 1 + 3 * 2.0 ** -11, float(np.finfo(np.float32).max)]
    return np.array(v, dtype=np.float64)


def test_f16_rounding_matches_numpy(ora):
    v = special_doubles(np.random.default_rng(11))
    got = ora.round_array(v, ora.F16)
    want = v.astype(np.float16).view(np.uint16)       # numpy rounds double -> half directly
    assert np.array_equal(got, want)


def nearest_check(v, bits, decode, neighbours):
    """bits is a correct round-to-nearest-even of v: no neighbour is closer,
    and at a tie the chosen value has an even significand."""
    got = Fraction(decode(bits))
    d = abs(Fraction(v) - got)
    for nb in neighbours(bits):
        val = decode(nb)
        if math.isinf(val) or math.isnan(val):
            continue
        dn = abs(Fraction(v) - Fraction(val))
        assert d < dn or (d == dn and (bits & 1) == 0), (v, bits, nb)


def test_bf16_rounding_is_nearest_even(ora):
    v = special_doubles(np.random.default_rng(12))
    L = ora.lib()
    for x in v:
        b = ora.round_bf16(x)
        if math.isinf(L.ora_bf16_value(b)):
            assert abs(x) >= 3.3961e38
            continue
        nearest_check(x, b, L.ora_bf16_value, lambda q: [(q + 1) & 0xFFFF, (q - 1) & 0xFFFF])


def test_bf16_matches_torch_on_float32_exact_values(ora):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(13)
    f = rng.standard_normal(20000).astype(np.float32)
    f = np.concatenate([f, np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8], dtype=np.float32)])
    want = torch.from_numpy(f).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    got = ora.round_array(f.astype(np.float64), ora.BF16)
    assert np.array_equal(got, want)


def test_stored_values_round_trip(ora):
    v = special_doubles(np.random.default_rng(14))
    v = v[np.abs(v) < 60000]
    for dt, tol in [(ora.BF16, 2.0 ** -8), (ora.F16, 2.0 ** -11)]:   # unit roundoff
        back = ora.stored_as_f64(ora.round_array(v, dt), dt)
        normal = np.abs(v) > (1e-37 if dt == ora.BF16 else 6.2e-5)
        assert np.all(np.abs(back - v)[normal] <= tol * np.abs(v)[normal])


# ---------------------------------------------------------------------------
# Conjugate gradients: any x with true residual below tol is correct
# ---------------------------------------------------------------------------

def test_cg_true_residual(ora):
    for i in range(3):
        A, kind = synth.serve_pool_matrix(i, 2e3, 2e4)
        b = np.random.default_rng(i).uniform(-1, 1, A.n_rows)
        x, it, rel = ora.cg(A.rp, A.col, A.val, b, 1e-10, 5000)
        M = sp.csr_matrix((A.val, A.col, A.rp), shape=(A.n_rows, A.n_cols))
        true = np.linalg.norm(b - M @ x) / np.linalg.norm(b)
        assert true <= 1e-10 and abs(true - rel) <= 1e-12 and it > 0


# ---------------------------------------------------------------------------
# Row-grouped CSR (reading R9): the Sliced-ELLPACK-style storage the paper
# builds ARG-CSR from (Sec. 3) and compares it with (Sec. 5)
# ---------------------------------------------------------------------------

def test_rgcsr_fig3_one_thread_per_row(ora):
    """Sec. 3: with one thread per row the Fig. 3 matrix needs chunk size 8
    and 49 artificial zeros (golden file); block_dim = 8 maps exactly one
    thread to each row."""
    paper = json.load(open(os.path.join(GOLDEN, "fig3_example.json")))["stated_by_paper"]
    rp, col, val = fig3_matrix()
    a = ora.rg_convert(rp, col, val, paper["rows"])
    one = paper["one_thread_per_row"]
    assert a.groups.tolist() == [[0, 8, 0, one["chunk_size"]]]
    assert int((a.columns == -1).sum()) == one["artificial_zeros"]
    assert a.tm.tolist() == list(range(1, 9))


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(T=st.sampled_from([1, 3, 8, 64]), k=st.integers(0, 9), n_blocks=st.integers(1, 5),
       tail=st.integers(0, 7))
def test_rgcsr_uniform_rows_closed_form(ora, T, k, n_blocks, tail):
    """Uniform row length k: element e of row r sits at
    floor(r/T)*max(k,1)*T + e*T + (r mod T) (ELLPACK per slice of T rows)."""
    n = n_blocks * T + min(tail, T - 1)
    rp = (np.arange(n + 1) * k).astype(np.int32)
    col = np.tile(np.arange(k), n).astype(np.int32)
    val = np.arange(n * k, dtype=np.float64) + 1.0        # value = 1 + CSR position
    a = ora.rg_convert(rp, col, val, T)
    w = max(k, 1)
    assert a.n_groups == -(-n // T) and a.n_slots == a.n_groups * w * T
    for r in range(n):
        for e in range(k):
            s = (r // T) * w * T + e * T + (r % T)
            assert a.columns[s] == e and a.values[s] == 1.0 + r * k + e
    assert int((a.columns >= 0).sum()) == n * k


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(lengths=st.lists(st.integers(0, 40), min_size=1, max_size=90),
       T=st.sampled_from([1, 2, 5, 16, 30]))
def test_rgcsr_equals_argcsr_with_unbounded_budget(ora, lengths, T):
    """When every slice is full, row-grouped CSR is what ARG-CSR's own
    steps give once the nonzero budget cannot bind (desired_chunk_size at
    least the longest row): groups of T rows, chunk size = the longest row
    (the greedy distribution leaves no thread free to split a row), one
    chunk per row.  Two independent code paths of the oracle."""
    n = len(lengths) - len(lengths) % T
    if n == 0:
        return
    rp = np.concatenate([[0], np.cumsum(lengths[:n])]).astype(np.int32)
    col = np.zeros(rp[-1], dtype=np.int32)
    val = np.arange(rp[-1], dtype=np.float64)
    rg = ora.rg_convert(rp, col, val, T)
    ar = ora.convert(rp, col, val, T, max(1, max(lengths[:n])))
    for f in ("groups", "tm", "columns", "values"):
        assert np.array_equal(getattr(rg, f), getattr(ar, f)), f


def test_rgcsr_partial_last_slice_keeps_one_chunk_per_row(ora):
    """n = T + 1 with a long last row: the second slice holds that row alone
    with chunk size = its length (ARG-CSR would spread it over the slice's
    free threads), and an all-empty slice has chunk size 1 (R9)."""
    T = 4
    rp, col, val = csr_from_rows([[(0, 1.0)]] * T + [[(j, 2.0) for j in range(10)]], 10)
    a = ora.rg_convert(rp, col, val, T)
    assert a.groups.tolist() == [[0, 4, 0, 1], [4, 1, 4, 10]]
    assert a.tm.tolist() == [1, 2, 3, 4, 1]
    assert ora.convert(rp, col, val, T, 100).groups[1, 3] == 3     # ARG: ceil(10 / 4)
    e = ora.rg_convert(np.zeros(6, dtype=np.int32), np.zeros(0, dtype=np.int32),
                       np.zeros(0), 4)
    assert e.groups.tolist() == [[0, 4, 0, 1], [4, 1, 4, 1]] and (e.columns == -1).all()


@settings(max_examples=40, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(lengths=st.lists(st.integers(0, 25), min_size=0, max_size=70),
       T=st.sampled_from([1, 4, 7, 64]), seed=st.integers(0, 2**31 - 1))
def test_rgcsr_roundtrip_and_spmv_is_csr_order(ora, lengths, T, seed):
    """Decoding the storage gives back the CSR matrix, and since each row is
    one chunk summed left to right, the SpMV is bitwise the sequential CSR
    sum (Sec. 2)."""
    rng = np.random.default_rng(seed)
    n = len(lengths)
    A = synth.random_csr(np.asarray(lengths, dtype=np.int64), 30, rng, rng)
    a = ora.rg_convert(A.rp, A.col, A.val, T)
    rp2, col2, val2 = ora.argcsr_to_csr(a, A.nnz)
    assert np.array_equal(rp2, A.rp) and np.array_equal(col2, A.col)
    assert np.array_equal(val2, A.val)
    x = rng.uniform(-1, 1, 30)
    y = ora.argcsr_spmv(a, x)
    yc = ora.csr_spmv(A.rp, A.col, A.val, x)
    assert np.array_equal(y.view(np.uint64), yc.view(np.uint64)) or n == 0


# ---------------------------------------------------------------------------
# desiredChunkSize per region of rows (reading R10: the region of a group's
# first row sets its nonzero limit)
# ---------------------------------------------------------------------------

def test_regions_hand_worked_example(ora):
    """T = 4, regions of 4 rows with D = 2 then 1 (limits 8 and 4 nonzeros),
    row lengths 3,3,3,3 | 2,2,2,2 | 1,1.  By hand: rows 0-1 (6; row 2 would
    make 9 > 8); rows 2-4 (8: the group opened in region 0 keeps its limit
    while it runs into region 1); rows 5-6 (4); rows 7-9 (4)."""
    L = [3, 3, 3, 3, 2, 2, 2, 2, 1, 1]
    rp = np.concatenate([[0], np.cumsum(L)]).astype(np.int32)
    col = np.zeros(rp[-1], dtype=np.int32)
    a = ora.convert_regions(rp, col, np.ones(rp[-1]), 4, 4, [2, 1, 1])
    assert a.groups[:, :2].tolist() == [[0, 2], [2, 3], [5, 2], [7, 3]]


def test_regions_group_keeps_its_limit_after_crossing(ora):
    """T = 4, regions of 4 rows with D = 2, 1, 1 (limits 8, 4, 4), row
    lengths 3,3,3,3 | 1,1,1,1 | 1,1.  The group opened at row 2 keeps the
    limit 8 of its first row's region after it runs into region 1, so it takes
    rows 2-5 (3+3+1+1 = 8, four rows); a limit taken from the row just added
    would close it after row 4.  Then rows 6-9 (4 nonzeros, four rows)."""
    L = [3, 3, 3, 3, 1, 1, 1, 1, 1, 1]
    rp = np.concatenate([[0], np.cumsum(L)]).astype(np.int32)
    col = np.zeros(rp[-1], dtype=np.int32)
    a = ora.convert_regions(rp, col, np.ones(rp[-1]), 4, 4, [2, 1, 1])
    assert a.groups[:, :2].tolist() == [[0, 2], [2, 4], [6, 4]]


@settings(max_examples=80, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(lengths=st.lists(st.integers(0, 60), min_size=0, max_size=120),
       T=st.sampled_from([1, 2, 5, 16, 64]), region_rows=st.integers(1, 40),
       seed=st.integers(0, 2**31 - 1))
def test_regions_groups_are_greedy_maximal(ora, lengths, T, region_rows, seed):
    """Brute-force statement of the rule: the groups partition the rows in
    order; a group opened at s holds at most T rows and at most D(s)*T
    nonzeros unless it is the single row s; and it cannot take one more row
    without breaking one of those limits."""
    rng = np.random.default_rng(seed)
    n = len(lengths)
    D = rng.integers(1, 5, max(1, -(-n // region_rows)))
    rp = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    a = ora.convert_regions(rp.astype(np.int32), np.zeros(rp[-1], dtype=np.int32),
                            np.ones(rp[-1]), T, region_rows, D)
    nxt = 0
    for first, size, _, _ in a.groups.tolist():
        assert first == nxt and size >= 1
        limit = int(D[first // region_rows]) * T
        e = first + size
        assert size <= T and (rp[e] - rp[first] <= limit or size == 1)
        if e < n:
            assert size + 1 > T or rp[e + 1] - rp[first] > limit
        nxt = e
    assert nxt == n


# ---------------------------------------------------------------------------
# staging of x for banded matrices (reading R11)
# ---------------------------------------------------------------------------

def _stage_example():
    """One group (T = 4, D = 18): rows with columns {0,1,2}, {5,9,10},
    {200..263} and {300}; chunk size 64, one chunk per row."""
    cols = [[0, 1, 2], [5, 9, 10], list(range(200, 264)), [300]]
    rp = np.cumsum([0] + [len(c) for c in cols]).astype(np.int32)
    col = np.concatenate(cols).astype(np.int32)
    return rp, col, np.ones(col.size)


def test_stage_hand_worked_example(ora):
    rp, col, val = _stage_example()
    a = ora.convert(rp, col, val, 4, 18)
    assert a.n_groups == 1 and a.groups[0, 3] == 64
    want = {
        # gap: (tile starts, tile lengths, {column: local index})
        0: ([0, 5, 9, 200, 300], [3, 1, 2, 64, 1], {0: 0, 2: 2, 5: 64, 9: 128, 10: 129,
                                                    200: 192, 263: 255, 300: 256}),
        2: ([0, 9, 200, 300], [6, 2, 64, 1], {0: 0, 5: 5, 9: 64, 10: 65, 200: 128,
                                              263: 191, 300: 192}),
        3: ([0, 200, 300], [11, 64, 1], {5: 5, 9: 9, 10: 10, 200: 64, 263: 127, 300: 128}),
        # the hole 11..199 (189 columns) stays open; 264..299 (36) is bridged
        100: ([0, 200, 264], [11, 64, 37], {0: 0, 9: 9, 200: 64, 263: 127, 300: 164}),
        # one window 0..300, cut every 64 columns: the local index is the column
        200: ([0, 64, 128, 192, 256], [64, 64, 64, 64, 45], {c: c for c in (0, 9, 200, 263, 300)}),
    }
    for gap, (starts, lens, loc) in want.items():
        st = ora.stage(a, gap, 16)
        assert list(st.tile_ptr) == [0, len(starts)], gap
        assert list(st.tile_start) == starts and list(st.tile_len) == lens, gap
        pos = {int(c): int(l) for c, l in zip(a.columns, st.local) if c >= 0}
        for c, l in loc.items():
            assert pos[c] == l, (gap, c)
        assert np.all(st.local[a.columns < 0] == 0xFFFF)
        assert np.array_equal(ora.unstage(a, st), a.columns)
    assert ora.stage(a, 0, 4) == ora.STAGE_TOO_MANY_TILES          # needs 5 tiles


def test_stage_laplace_closed_form(ora):
    """5-point Laplacian on a 64x64 grid, T = 64, D = 5: group i is grid line
    i and reads lines i-1, i, i+1 whole, one tile each (gap 0); column k of
    line L has local index 64*(L - max(i-1, 0)) + k."""
    s = 64
    A = synth.laplace2d(s, s)
    a = ora.convert(A.rp, A.col, A.val, s, 5)
    assert a.n_groups == s and np.all(a.groups[:, 1] == s)
    st = ora.stage(a, 0, 8)
    for i in range(s):
        lines = [L for L in (i - 1, i, i + 1) if 0 <= L < s]
        tb, te = st.tile_ptr[i], st.tile_ptr[i + 1]
        assert list(st.tile_start[tb:te]) == [64 * L for L in lines]
        assert np.all(st.tile_len[tb:te] == 64)
        off, c = a.groups[i, 2], a.groups[i, 3]
        sl = slice(off, off + c * s)
        cols, loc = a.columns[sl], st.local[sl]
        live = cols >= 0
        L, k = cols[live] // s, cols[live] % s
        assert np.array_equal(loc[live], 64 * (L - max(i - 1, 0)) + k)
        assert np.all(loc[~live] == 0xFFFF)


def _stage_by_occupancy(a, gap):
    """The same tiles from a different formulation: an occupancy array over
    each group's column range, holes of at most `gap` filled where a present
    column lies on both sides, runs of the result cut every 64 columns."""
    tiles = []
    T = a.block_dim
    for g in range(a.n_groups):
        off, c = a.groups[g, 2], a.groups[g, 3]
        cols = a.columns[off:off + c * T]
        cols = cols[cols >= 0]
        out = []
        if cols.size:
            lo, hi = cols.min(), cols.max()
            occ = np.zeros(hi - lo + 1, dtype=bool)
            occ[cols - lo] = True
            present = np.nonzero(occ)[0]
            for p, q in zip(present[:-1], present[1:]):
                if q - p - 1 <= gap:
                    occ[p:q] = True
            edges = np.diff(np.concatenate([[0], occ.astype(np.int8), [0]]))
            for s0, e0 in zip(np.nonzero(edges == 1)[0], np.nonzero(edges == -1)[0]):
                for t in range(s0, e0, 64):
                    out.append((int(lo + t), int(min(64, e0 - t))))
        tiles.append(out)
    return tiles


def test_stage_matches_occupancy_definition(ora):
    rng = np.random.default_rng(17)
    for trial in range(40):
        n = int(rng.integers(1, 300))
        n_cols = int(rng.integers(1, 2000))
        band = int(rng.integers(1, 200))
        L = rng.integers(0, 12, n)
        rows = []
        for r in range(n):
            centre = int(r * n_cols / max(n, 1))
            lo, hi = max(0, centre - band), min(n_cols, centre + band + 1)
            k = min(int(L[r]), hi - lo)
            rows.append(np.sort(rng.choice(np.arange(lo, hi), k, replace=False)))
        rp = np.cumsum([0] + [len(x) for x in rows]).astype(np.int32)
        col = np.concatenate(rows).astype(np.int32) if rp[-1] else np.zeros(0, np.int32)
        T = int(rng.choice([1, 5, 64, 128]))
        D = int(rng.choice([1, 2, 8]))
        gap = int(rng.choice([0, 1, 3, 17]))
        a = ora.convert(rp, col, np.ones(col.size), T, D)
        st = ora.stage(a, gap, 1023)
        want = _stage_by_occupancy(a, gap)
        assert list(np.diff(st.tile_ptr)) == [len(t) for t in want], trial
        flat = [t for ts in want for t in ts]
        assert list(zip(st.tile_start.tolist(), st.tile_len.tolist())) == flat, trial
        assert np.array_equal(ora.unstage(a, st), a.columns), trial
        # a local index addresses a column inside its tile
        for g in range(a.n_groups):
            off, c = a.groups[g, 2], a.groups[g, 3]
            loc = st.local[off:off + c * T]
            live = loc != 0xFFFF
            q = loc[live] // 64
            assert np.all(q < np.diff(st.tile_ptr)[g])
            assert np.all(loc[live] % 64 < st.tile_len[st.tile_ptr[g] + q])
