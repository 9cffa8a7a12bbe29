"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Conversion must be bit-exact (groups, threads mapping, columns, value bits).
FP64 SpMV must satisfy |y_gpu - y_oracle| <= 1e-12 * sum_j |a_ij x_j| per
row (exact where that sum is 0).  Reduced-precision SpMV (FP32 accumulation)
is checked against the FP64 oracle evaluated on the stored (rounded) values
with the worst-case bound gamma_{L+1}(2^-24) * sum_j |a_ij x_j|.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from conftest import gpu_available
from helpers import U32, abs_row_sums, gamma, powerlaw_sample, scaled_error

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ac():
    import paper_1203_5737_amd as ac
    ac._lib.lib()          # raises if the HIP library is not built
    return ac


def announce(msg):
    print(f"\n[gpu] {msg}", flush=True)


def compare_conversion(ac, A, T, D, dtype, device_grouping=False, fmt=0, keep_plan=False):
    announce(f"convert n={A.n_rows} nnz={A.nnz} T={T} D={D} dtype={dtype} "
             f"device_grouping={device_grouping} format={fmt} keep_plan={keep_plan}")
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
    if device_grouping:
        assert ac.plan_device(dev.row_ptr, T, D, fmt=fmt) == ac.plan(A.rp, T, D, fmt)
    M = ac.convert(dev, T, D, dtype, device_grouping=device_grouping, fmt=fmt,
                   keep_plan=keep_plan)
    if fmt == ac.FORMAT_RG:
        ref = oracle.rg_convert(A.rp, A.col, A.val, T, dtype)
    else:
        ref = oracle.convert(A.rp, A.col, A.val, T, D, dtype)
    assert M.n_groups == ref.n_groups and M.n_slots == ref.n_slots
    assert np.array_equal(M.groups.cpu().numpy(), ref.groups)
    assert np.array_equal(M.threads_mapping.cpu().numpy(), ref.tm)
    assert np.array_equal(M.columns.cpu().numpy(), ref.columns)
    gv = M.values.cpu()
    gbits = gv.view(torch.int64 if dtype == 0 else torch.int32 if dtype == 1 else torch.int16)
    rbits = ref.values.view(np.int64 if dtype == 0 else np.int32 if dtype == 1 else np.int16)
    assert np.array_equal(gbits.numpy(), rbits)
    # launch schedule: ascending indices of the groups with long chunk loops
    want_heavy = np.nonzero(ref.groups[:, 3] > M.heavy_chunk)[0]
    assert M.n_heavy == len(want_heavy)
    if M.n_heavy:
        assert np.array_equal(M.heavy_groups.cpu().numpy(), want_heavy)
    return dev, M, ref


def fig3():
    rp = np.array([0, 1, 2, 3, 4, 5, 6, 7, 15], dtype=np.int32)
    col = np.array(list(range(7)) + list(range(8)), dtype=np.int32)
    val = np.array([1, 2, 3, 4, 5, 6, 7] + [10 + j for j in range(8)], dtype=np.float64)
    return synth.Csr(8, 8, rp, col, val)


# ---------------------------------------------------------------------------
# conversion: bit-exact
# ---------------------------------------------------------------------------

def test_convert_fig3_any_block_dim(ac):
    compare_conversion(ac, fig3(), 12, 2, oracle.F64)
    compare_conversion(ac, fig3(), 12, 1, oracle.F64)
    compare_conversion(ac, fig3(), 3, 1, oracle.F32)


@pytest.mark.parametrize("T,D", [(64, 1), (64, 5), (128, 1), (256, 4), (100, 2)])
def test_convert_laplace64(ac, T, D):
    A, _ = synth.workload_laplace64()
    compare_conversion(ac, A, T, D, oracle.F64)


@pytest.mark.parametrize("dtype", [0, 1, 2, 3])
def test_convert_dtypes_bit_exact(ac, dtype):
    A, _ = powerlaw_sample(40_000, seed=1)
    # include values that stress rounding: ties, subnormal and overflow range
    rng = np.random.default_rng(5)
    special = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -11, 65520.0, 70000.0, 1e-7,
                        3e-8, 2.0 ** -25, 1e-300, 3.4e38, -(1 + 2 ** -8), 0.0, -0.0, 1e39,
                        1e-40, -2.5e-39, 1.2e-38, 6.1e-5, -6.0e-5])
    A.val[: special.size] = special
    A.val[special.size:2000] = rng.normal(0, 1e4, 2000 - special.size)
    for T, D in [(64, 1), (256, 2)]:
        compare_conversion(ac, A, T, D, dtype)


@pytest.mark.parametrize("dtype", [0, 1, 2, 3])
def test_convert_long_rows_bit_exact(ac, dtype):
    """Many short rows keep the mean chunk small, so rows of a few hundred to
    tens of thousands of elements have chunks longer than the fill's LDS stage
    and are filled by the long-row pass: single-row groups, several blocks of
    64 chunks, step counts that are not a multiple of the tile, and long rows
    at the start, middle and end of the matrix."""
    rng = np.random.default_rng(17)
    lengths = rng.integers(0, 6, 30_000)
    for pos, L in [(0, 20_000), (5, 300), (777, 1025), (12_345, 4097), (20_000, 65_537),
                   (29_999, 2_500)]:
        lengths[pos] = L
    rp = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int32)
    nnz = int(rp[-1])
    n_cols = 70_000
    col = np.concatenate([np.sort(rng.choice(n_cols, L, replace=False)) for L in lengths]).astype(np.int32)
    val = rng.uniform(-1, 1, nnz)
    A = synth.Csr(len(lengths), n_cols, rp, col, val)
    for T, D in [(64, 1), (100, 1), (256, 2), (1000, 1)]:
        compare_conversion(ac, A, T, D, dtype)


@pytest.mark.parametrize("T,D", [(64, 1), (64, 2), (64, 4), (128, 1), (256, 1), (7, 3), (1000, 1)])
def test_convert_powerlaw(ac, T, D):
    A, _ = powerlaw_sample(60_000, seed=2)
    compare_conversion(ac, A, T, D, oracle.F64)


def test_convert_edge_cases(ac):
    rng = np.random.default_rng(9)
    # empty rows mixed in, a 10^4 row, a row of 1000 (chunk 16 at T=64)
    L = rng.integers(0, 5, 3000)
    L[::7] = 0
    L[100] = 10_000
    L[2000] = 1000
    A = synth.random_csr(L, 20_000, rng, rng)
    for T, D in [(64, 1), (128, 3), (256, 1)]:
        compare_conversion(ac, A, T, D, oracle.F64)
    # every row empty
    E = synth.Csr(500, 10, np.zeros(501, np.int32), np.zeros(0, np.int32), np.zeros(0))
    compare_conversion(ac, E, 64, 1, oracle.F64)
    # a single row
    compare_conversion(ac, synth.random_csr(np.array([1000]), 1000, rng, rng), 64, 1, oracle.F64)


def test_convert_rejects_bad_input(ac):
    A, _ = synth.workload_laplace64()
    col = A.col.copy()
    col[77] = A.n_cols           # out of range
    dev = ac.to_device_csr(A.rp, col, A.val, A.n_cols, DEV)
    with pytest.raises(ac.ArgCsrError) as e:
        ac.convert(dev, 64, 1)
    assert e.value.code == ac._lib.EINVAL
    col[77] = -1                 # the padding marker is never a real column
    dev = ac.to_device_csr(A.rp, col, A.val, A.n_cols, DEV)
    with pytest.raises(ac.ArgCsrError):
        ac.convert(dev, 64, 1)


def test_convert_validates_every_column_position(ac):
    """Every column index is checked as the fill stages it: a bad index at
    the start, the middle or the end of the array is found, for every
    alignment of the array's start."""
    rng = np.random.default_rng(23)
    L = rng.integers(0, 9, 500)
    A = csr_from_lengths(L, 300, 23)
    nnz = A.nnz
    for shift in range(4):
        for pos in sorted({0, 1, 2, 3, 4, 5, nnz // 2, nnz - 5, nnz - 4, nnz - 3, nnz - 2, nnz - 1}):
            for bad in (A.n_cols, -1, -(2 ** 31), 2 ** 31 - 1):
                col = A.col.copy()
                col[pos] = bad
                padded = torch.zeros(nnz + 4, dtype=torch.int32, device=DEV)
                padded[shift:shift + nnz] = torch.from_numpy(col).to(DEV)
                dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
                dev.col = padded[shift:shift + nnz]       # a view 4*shift bytes past alignment
                with pytest.raises(ac.ArgCsrError) as e:
                    ac.convert(dev, 32, 2)
                assert e.value.code == ac._lib.EINVAL, (shift, pos, bad)
        padded = torch.zeros(nnz + 4, dtype=torch.int32, device=DEV)
        padded[shift:shift + nnz] = torch.from_numpy(A.col).to(DEV)
        dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
        dev.col = padded[shift:shift + nnz]
        M = ac.convert(dev, 32, 2)                            # every index valid
        ref = oracle.convert(A.rp, A.col, A.val, 32, 2)
        assert np.array_equal(M.columns.cpu().numpy(), ref.columns)


def test_convert_validates_columns_of_long_rows(ac):
    """The chunks of rows longer than the fill's stage are moved tile by tile
    by fill_long_kernel, which checks their columns itself: a bad index at
    the tile and chunk boundaries of two long rows (in groups of their own,
    chunk sizes 79 and 24, the last chunk of the second one short) is found,
    and the matrix without it converts to the oracle's columns."""
    rng = np.random.default_rng(31)
    L = rng.integers(0, 6, 400)
    L[10] = 5000          # alone in its group at T=64, D=1: 64 chunks of 79
    L[200] = 1500         # 64 chunks of 24
    A = csr_from_lengths(L, 6000, 31)
    for row, c in ((10, 79), (200, 24)):
        s0 = int(A.rp[row])
        picks = {0, 1, 15, 16, 17, c - 1, c, c + 15, 31 * c + 16, int(L[row]) - 1}
        for off in sorted(p for p in picks if p < int(L[row])):
            col = A.col.copy()
            col[s0 + off] = -1 if off % 2 else A.n_cols
            dev = ac.to_device_csr(A.rp, col, A.val, A.n_cols, DEV)
            with pytest.raises(ac.ArgCsrError) as e:
                ac.convert(dev, 64, 1)
            assert e.value.code == ac._lib.EINVAL, (row, off)
    M = ac.convert(ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV), 64, 1)
    ref = oracle.convert(A.rp, A.col, A.val, 64, 1)
    assert np.array_equal(M.columns.cpu().numpy(), ref.columns)


# ---------------------------------------------------------------------------
# conversion step 1 on the device (binary lifting): identical groups
# ---------------------------------------------------------------------------

def csr_from_lengths(L, n_cols, seed):
    rng = np.random.default_rng(seed)
    return synth.random_csr(np.asarray(L, dtype=np.int64), n_cols, rng, rng)


def test_device_grouping_fig3_and_laplace(ac):
    for T in (1, 2, 3, 5, 12, 100):
        for D in (1, 2, 3):
            compare_conversion(ac, fig3(), T, D, oracle.F64, device_grouping=True)
    A, _ = synth.workload_laplace64()
    for T, D in [(64, 1), (64, 5), (128, 1), (100, 2), (1024, 1)]:
        compare_conversion(ac, A, T, D, oracle.F64, device_grouping=True)


@pytest.mark.parametrize("T,D", [(64, 1), (128, 2), (256, 1), (7, 3), (1000, 1)])
def test_device_grouping_powerlaw(ac, T, D):
    A, _ = powerlaw_sample(300_000, seed=31)
    compare_conversion(ac, A, T, D, oracle.F64, device_grouping=True)


def test_device_grouping_edge_cases(ac):
    """Empty rows only (groups of T rows), every row over the budget (one
    row per group), alternating empty and long rows, one row, and sizes
    around powers of two (the number of jump levels)."""
    cases = [
        ([0], 5, 64, 1), ([300], 400, 64, 1), ([0] * 5000, 10, 64, 1),
        ([200] * 3000, 300, 64, 1), ([0, 500] * 800, 600, 64, 2),
        ([1] * 1023, 50, 1, 1), ([3] * 4097, 50, 64, 1),
    ]
    rng = np.random.default_rng(40)
    for n in (255, 256, 257, 1023, 1024, 1025, 65536, 65537):
        cases.append((rng.integers(0, 9, n), 100, int(rng.choice([1, 16, 64, 256])),
                      int(rng.integers(1, 4))))
    for i, (L, n_cols, T, D) in enumerate(cases):
        compare_conversion(ac, csr_from_lengths(L, n_cols, 41 + i), T, D, oracle.F64,
                           device_grouping=True)


def test_device_grouping_random(ac):
    rng = np.random.default_rng(42)
    for i in range(30):
        n = int(rng.integers(1, 3000))
        L = rng.integers(0, int(rng.choice([3, 30, 300])), n)
        L[rng.integers(0, n, 3)] = rng.integers(0, 4000, 3)
        T = int(rng.choice([1, 3, 64, 128, 256, 1000]))
        D = int(rng.integers(1, 6))
        A = csr_from_lengths(L, 5000, 100 + i)
        dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
        assert ac.plan_device(dev.row_ptr, T, D) == ac.plan(A.rp, T, D), (i, T, D)
        M = ac.convert(dev, T, D, device_grouping=True)
        ref = oracle.convert(A.rp, A.col, A.val, T, D)
        assert np.array_equal(M.groups.cpu().numpy(), ref.groups), (i, T, D)
        assert np.array_equal(M.threads_mapping.cpu().numpy(), ref.tm)
        assert np.array_equal(M.columns.cpu().numpy(), ref.columns)


def test_device_grouping_with_kept_plan(ac):
    """argcsr_plan_device_keep + argcsr_convert_planned (steps 1-3 once, kept
    on the device): the same bytes as the oracle."""
    A, _ = powerlaw_sample(200_000, seed=35)
    for T, D, dt in [(64, 1, oracle.F64), (128, 2, oracle.F32), (7, 3, oracle.F16),
                     (1000, 1, oracle.BF16)]:
        compare_conversion(ac, A, T, D, dt, device_grouping=True, keep_plan=True)
    compare_conversion(ac, csr_from_lengths([0, 500] * 300, 600, 77), 64, 2, oracle.F64,
                       device_grouping=True, keep_plan=True)
    compare_conversion(ac, csr_from_lengths([0] * 3000, 10, 78), 64, 1, oracle.F64,
                       device_grouping=True, keep_plan=True)
    compare_conversion(ac, fig3(), 8, 0, oracle.F64, device_grouping=True, fmt=ac.FORMAT_RG,
                       keep_plan=True)


def test_convert_planned_rejects_another_matrix(ac):
    """A device plan converts only the matrix it was made for: out's sizes or
    parameters that differ from the plan's are refused before any write."""
    import ctypes
    L = ac._lib
    A, _ = powerlaw_sample(20_000, seed=36)
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
    g, s, h = ctypes.c_int32(0), ctypes.c_int64(0), ctypes.c_int32(0)
    plan = ctypes.c_void_p(0)
    s_ = ac._stream(None)
    ac.check(L.lib().argcsr_plan_device_keep(A.n_rows, ac._ptr(dev.row_ptr), 64, 1, 0,
                                             ctypes.byref(g), ctypes.byref(s), ctypes.byref(h),
                                             ctypes.byref(plan), s_), "plan")
    try:
        assert (g.value, s.value, h.value) == ac.plan(A.rp, 64, 1)
        M = ac.convert(dev, 64, 1)
        for field, bad in [("n_slots", s.value + 64), ("block_dim", 128),
                           ("desired_chunk_size", 2), ("n_groups", g.value - 1)]:
            d = M.desc()
            setattr(d, field, bad)
            rc = L.lib().argcsr_convert_planned(plan, A.n_cols, ac._ptr(dev.row_ptr),
                                                ac._ptr(dev.col), ac._ptr(dev.val),
                                                ctypes.byref(d), s_)
            assert rc == L.EINVAL, field
        # the right descriptor converts to the same bytes as argcsr_convert
        M2 = ac.convert(dev, 64, 1)
        d = M2.desc()
        M2.columns.fill_(0)
        ac.check(L.lib().argcsr_convert_planned(plan, A.n_cols, ac._ptr(dev.row_ptr),
                                                ac._ptr(dev.col), ac._ptr(dev.val),
                                                ctypes.byref(d), s_), "planned")
        for f in ("groups", "threads_mapping", "columns", "values", "heavy_groups"):
            assert torch.equal(getattr(M, f), getattr(M2, f)), f
    finally:
        L.lib().argcsr_device_plan_destroy(plan)


def test_device_grouping_rejects_bad_row_ptr(ac):
    for rp in ([1, 2, 3], [0, 3, 2, 4], [0, 2, 1]):
        rpd = torch.tensor(rp, dtype=torch.int32, device=DEV)
        with pytest.raises(ac.ArgCsrError) as e:
            ac.plan_device(rpd, 64, 1)
        assert e.value.code == ac._lib.EINVAL
    assert ac.plan_device(torch.zeros(1, dtype=torch.int32, device=DEV), 64, 1) == (0, 0, 0)


# ---------------------------------------------------------------------------
# row-grouped CSR (second storage format, same kernels)
# ---------------------------------------------------------------------------

def test_row_grouped_conversion_bit_exact(ac):
    compare_conversion(ac, fig3(), 8, 0, oracle.F64, fmt=ac.FORMAT_RG)
    A, _ = synth.workload_laplace64()
    for T in (64, 100, 256):
        compare_conversion(ac, A, T, 0, oracle.F64, fmt=ac.FORMAT_RG)
    Ap, _ = powerlaw_sample(100_000, seed=33)
    for T, dtype, dev_group in [(64, oracle.F64, False), (128, oracle.F32, True),
                                (256, oracle.BF16, False), (64, oracle.F16, True)]:
        compare_conversion(ac, Ap, T, 0, dtype, device_grouping=dev_group, fmt=ac.FORMAT_RG)
    for i, (L, T) in enumerate([([0] * 300, 64), ([5] * 129 + [2000], 64), ([3, 0, 700] * 50, 7)]):
        compare_conversion(ac, csr_from_lengths(L, 2500, 60 + i), T, 0, oracle.F64,
                           device_grouping=bool(i % 2), fmt=ac.FORMAT_RG)


def test_row_grouped_spmv(ac):
    A, x = powerlaw_sample(60_000, seed=34)
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
    for T in (64, 128, 256):
        M = ac.convert(dev, T, 0, fmt=ac.FORMAT_RG)
        assert M.format == ac.FORMAT_RG
        check_f64(A, x, gpu_spmv(ac, M, x))
        M32 = ac.convert(dev, T, 0, ac.F32, fmt=ac.FORMAT_RG)
        check_reduced(A, x, gpu_spmv(ac, M32, x.astype(np.float32)), oracle.F32)


# ---------------------------------------------------------------------------
# desiredChunkSize per region of rows (reading R10)
# ---------------------------------------------------------------------------

def compare_regions(ac, A, T, region_rows, D, dtype=0, device_grouping=False):
    announce(f"regions n={A.n_rows} T={T} region_rows={region_rows} device={device_grouping}")
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
    M = ac.convert(dev, T, 0, dtype, region_rows=region_rows, region_desired=D,
                   device_grouping=device_grouping)
    ref = oracle.convert_regions(A.rp, A.col, A.val, T, region_rows, D, dtype)
    assert np.array_equal(M.groups.cpu().numpy(), ref.groups)
    assert np.array_equal(M.threads_mapping.cpu().numpy(), ref.tm)
    assert np.array_equal(M.columns.cpu().numpy(), ref.columns)
    gv = M.values.cpu()
    gbits = gv.view(torch.int64 if dtype == 0 else torch.int32 if dtype == 1 else torch.int16)
    rbits = ref.values.view(np.int64 if dtype == 0 else np.int32 if dtype == 1 else np.int16)
    assert np.array_equal(gbits.numpy(), rbits)
    return dev, M


def test_regions_conversion_and_spmv(ac):
    A, x = synth.workload_mixed(16)
    D = ac.choose_region_desired(A.rp, 512)
    assert D.min() == 1 and D.max() == 27
    for T, dev_group, dtype in [(64, False, 0), (128, True, 0), (256, False, 1), (64, True, 2)]:
        dev, M = compare_regions(ac, A, T, 512, D, dtype, dev_group)
        if dtype == 0:
            check_f64(A, x, gpu_spmv(ac, M, x))
    rng = np.random.default_rng(50)
    for i in range(6):
        L = rng.integers(0, int(rng.choice([4, 40])), int(rng.integers(100, 3000)))
        A2 = csr_from_lengths(L, 5000, 200 + i)
        region_rows = int(rng.integers(1, 700))
        D2 = rng.integers(1, 9, -(-A2.n_rows // region_rows)).astype(np.int32)
        compare_regions(ac, A2, int(rng.choice([1, 64, 100, 256])), region_rows, D2,
                        device_grouping=bool(i % 2))


# ---------------------------------------------------------------------------
# SpMV
# ---------------------------------------------------------------------------

def gpu_spmv(ac, M, x):
    xd = torch.from_numpy(np.ascontiguousarray(x)).to(DEV)
    y = torch.full((M.n_rows,), float("nan"), dtype=ac.vector_dtype(M.dtype), device=DEV)
    ac.spmv(M, xd, y)
    return y.cpu().numpy().astype(np.float64)


def check_f64(A, x, y):
    y_ref = oracle.csr_spmv(A.rp, A.col, A.val, x)
    worst, zero_ok = scaled_error(y, y_ref, abs_row_sums(A.rp, A.col, A.val, x))
    assert zero_ok and worst <= 1e-12, worst
    return worst


def check_reduced(A, x, y, dtype):
    """y computed with values stored in `dtype`, x in FP32, FP32 accumulation."""
    stored = oracle.stored_as_f64(oracle.round_array(A.val, dtype), dtype)
    x32 = x.astype(np.float32).astype(np.float64)
    y_ref = oracle.csr_spmv(A.rp, A.col, stored, x32)
    scale = abs_row_sums(A.rp, A.col, stored, x32)
    L = np.diff(A.rp)
    d = np.abs(y - y_ref)
    bound = gamma(L + 1, U32) * scale
    assert np.all(d <= bound), float(np.max(d - bound))      # rows with scale 0: exact
    # storage error against the FP64 oracle on the original values (reported)
    y64 = oracle.csr_spmv(A.rp, A.col, A.val, x)
    s64 = abs_row_sums(A.rp, A.col, A.val, x)
    acc_err, _ = scaled_error(y, y_ref, scale)
    tot_err, _ = scaled_error(y, y64, s64)
    return acc_err, tot_err


def test_spmv_laplace64_closed_form_exact(ac):
    """5-point stencil on u = i^2 + j^2: every product and partial sum is a
    small integer, so the GPU result equals the closed form bit for bit."""
    A, _ = synth.workload_laplace64()
    n = 64
    i, j = np.divmod(np.arange(n * n), n)
    u = (i * i + j * j).astype(np.float64)
    want = 4 * u
    for di, dj in [(-1, 0), (1, 0), (0, -1), (0, 1)]:
        ok = (i + di >= 0) & (i + di < n) & (j + dj >= 0) & (j + dj < n)
        want[ok] -= u[((i + di) * n + j + dj)[ok]]
    for T, D in [(64, 1), (64, 5), (128, 1), (256, 4)]:
        for dtype in [0, 1, 2, 3]:
            dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
            M = ac.convert(dev, T, D, dtype)
            y = gpu_spmv(ac, M, u if dtype == 0 else u.astype(np.float32))
            assert np.array_equal(y, want), (T, D, dtype)


@pytest.mark.parametrize("T,D", [(64, 1), (64, 5), (128, 1), (256, 4)])
def test_spmv_laplace64_f64(ac, T, D):
    A, x = synth.workload_laplace64()
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
    M = ac.convert(dev, T, D)
    check_f64(A, x, gpu_spmv(ac, M, x))


@pytest.mark.parametrize("T,D", [(64, 1), (64, 4), (128, 1), (128, 2), (256, 1), (256, 2)])
def test_spmv_powerlaw_f64(ac, T, D):
    A, x = powerlaw_sample(80_000, seed=3)
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
    M = ac.convert(dev, T, D)
    check_f64(A, x, gpu_spmv(ac, M, x))


def test_spmv_edge_cases(ac):
    rng = np.random.default_rng(10)
    L = rng.integers(0, 4, 5000)
    L[::5] = 0
    L[17] = 10_000
    L[4000] = 64 * 64 + 3          # longer than one group's 64 chunks of 64
    A = synth.random_csr(L, 30_000, rng, rng)
    x = rng.uniform(-1, 1, A.n_cols)
    for T, D in [(64, 1), (128, 1), (256, 1), (256, 8)]:
        dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
        M = ac.convert(dev, T, D)
        y = gpu_spmv(ac, M, x)
        check_f64(A, x, y)
        assert np.all(y[L == 0] == 0)
    # all rows empty: y overwritten with zeros
    E = synth.Csr(300, 5, np.zeros(301, np.int32), np.zeros(0, np.int32), np.zeros(0))
    M = ac.convert(ac.to_device_csr(E.rp, E.col, E.val, 5, DEV), 64, 1)
    assert np.all(gpu_spmv(ac, M, np.ones(5)) == 0)


@pytest.mark.parametrize("dtype", [1, 2, 3])
def test_spmv_reduced_precision(ac, dtype):
    for A, x in [powerlaw_sample(50_000, seed=4), synth.workload_stencil27(24)]:
        dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
        for T, D in [(64, 1), (256, 2)]:
            M = ac.convert(dev, T, D, dtype)
            y = gpu_spmv(ac, M, x.astype(np.float32))
            acc_err, tot_err = check_reduced(A, x, y, dtype)
            announce(f"dtype={dtype} T={T} D={D}: accumulation err {acc_err:.2e}, "
                     f"total err vs FP64 {tot_err:.2e} (x sum|ax|)")


def test_spmv_heavy_schedule_on_and_off(ac):
    """Long rows: split over a workgroup (schedule) or one wave each (none)."""
    rng = np.random.default_rng(12)
    L = rng.integers(1, 6, 20_000)
    L[rng.integers(0, 20_000, 40)] = rng.integers(200, 10_001, 40)
    A = synth.random_csr(L, 50_000, rng, rng)
    x = rng.uniform(-1, 1, A.n_cols)
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
    for T in (64, 128, 256):
        M = ac.convert(dev, T, 1)
        assert M.n_heavy > 0
        check_f64(A, x, gpu_spmv(ac, M, x))
        M0 = ac.convert(dev, T, 1, schedule=False)
        assert M0.heavy_groups is None
        check_f64(A, x, gpu_spmv(ac, M0, x))


def test_concurrent_conversions_on_separate_streams(ac):
    """Conversions from several host threads, each on its own stream, at
    once: conversion scratch is stream-ordered per call, so every result is
    the oracle's."""
    import threading
    mats = [powerlaw_sample(40_000 + 7_000 * i, seed=70 + i)[0] for i in range(4)]
    refs = [oracle.convert(A.rp, A.col, A.val, 64, 1) for A in mats]
    devs = [ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV) for A in mats]
    errors = []

    def work(i):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                for rep in range(5):
                    M = ac.convert(devs[i], 64, 1, stream=st, device_grouping=bool(rep % 2))
                    st.synchronize()
                    if not (np.array_equal(M.groups.cpu().numpy(), refs[i].groups) and
                            np.array_equal(M.columns.cpu().numpy(), refs[i].columns)):
                        errors.append((i, rep))
        except Exception as e:  # noqa: BLE001 - reported below
            errors.append((i, repr(e)))

    threads = [threading.Thread(target=work, args=(i,)) for i in range(4)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors


def random_case(seed):
    """A seeded random matrix and conversion setting: row-length mix, block
    size, desiredChunkSize, storage type, format and where step 1 runs."""
    rng = np.random.default_rng([7771, seed])
    n = int(np.exp(rng.uniform(0, np.log(40_000))))
    mix = rng.choice(["uniform", "zipf", "constant", "sparse"])
    if mix == "uniform":
        L = rng.integers(0, int(rng.choice([2, 9, 60])), n)
    elif mix == "zipf":
        L = np.clip(rng.zipf(rng.uniform(1.6, 2.6), n), 1, 5000)
    elif mix == "constant":
        L = np.full(n, int(rng.integers(1, 40)))
    else:
        L = np.where(rng.random(n) < 0.7, 0, rng.integers(1, 6, n))
    for pos in rng.integers(0, n, int(rng.integers(0, 4))):   # a few long rows
        L[pos] = int(rng.integers(100, 20_000))
    n_cols = int(max(L.max(initial=0), 1) + rng.integers(1, 30_000))
    T = int(rng.choice([64, 128, 256]) if rng.random() < 0.6 else
            rng.choice([1, 2, 7, 32, 100, 512, 1000, 1024]))
    D = int(np.exp(rng.uniform(0, np.log(64))))
    dtype = int(rng.integers(0, 4))
    fmt = 1 if rng.random() < 0.2 else 0
    device_grouping = bool(rng.random() < 0.5)
    return csr_from_lengths(L, n_cols, 9000 + seed), T, D, dtype, fmt, device_grouping, rng


@pytest.mark.parametrize("part", range(4))
def test_random_sweep_conversion_and_spmv(ac, part):
    """40 seeded random cases (10 per part): the conversion bit-exact against
    the oracle (any block size) and y within the error bound of the storage
    type (block sizes the SpMV kernels take; the others are refused)."""
    from paper_1203_5737_amd import _lib
    for seed in range(10 * part, 10 * part + 10):
        A, T, D, dtype, fmt, dg, rng = random_case(seed)
        announce(f"sweep seed={seed}")
        dev, M, ref = compare_conversion(ac, A, T, D, dtype, device_grouping=dg, fmt=fmt)
        x = rng.uniform(-1, 1, A.n_cols)
        if T not in (64, 128, 256):
            with pytest.raises(_lib.ArgCsrError) as e:
                gpu_spmv(ac, M, x if dtype == 0 else x.astype(np.float32))
            assert e.value.code == _lib.EUNSUPPORTED
        elif dtype == 0:
            check_f64(A, x, gpu_spmv(ac, M, x))
        else:
            check_reduced(A, x, gpu_spmv(ac, M, x.astype(np.float32)), dtype)


def test_spmv_deterministic(ac):
    A, x = powerlaw_sample(100_000, seed=5)
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
    M = ac.convert(dev, 128, 1)
    y1, y2 = gpu_spmv(ac, M, x), gpu_spmv(ac, M, x)
    assert np.array_equal(y1.view(np.uint64), y2.view(np.uint64))


@pytest.mark.parametrize("V", [0, 1, 2, 8, 64])
def test_csr_baseline(ac, V):
    A, x = powerlaw_sample(30_000, seed=6)
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
    xd = torch.from_numpy(x).to(DEV)
    y = ac.csr_spmv(dev, xd, lanes_per_row=V).cpu().numpy()
    check_f64(A, x, y)
    vals32 = dev.val.to(torch.float32)
    y32 = ac.csr_spmv(dev, xd.float(), values=vals32, dtype=ac.F32, lanes_per_row=V)
    check_reduced(A, x, y32.cpu().numpy().astype(np.float64), oracle.F32)


# ---------------------------------------------------------------------------
# full-size workloads, in the launch configuration the benchmark times
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def powerlaw_full():
    return synth.workload_powerlaw()


@pytest.fixture(scope="module")
def stencil_full():
    return synth.workload_stencil27(128)


@pytest.mark.parametrize("T,D", [(64, 1), (128, 1), (256, 1)])   # fixed, tuned, fewest groups
def test_full_powerlaw_f64(ac, powerlaw_full, T, D):
    A, x = powerlaw_full
    dev, M, ref = compare_conversion(ac, A, T, D, oracle.F64)
    check_f64(A, x, gpu_spmv(ac, M, x))


def test_full_device_grouping(ac, powerlaw_full, stencil_full):
    compare_conversion(ac, powerlaw_full[0], 64, 1, oracle.F64, device_grouping=True)
    compare_conversion(ac, stencil_full[0], 128, 27, oracle.F32, device_grouping=True)
    torch.cuda.empty_cache()


def test_full_stencil_row_grouped(ac, stencil_full):
    A, x = stencil_full
    dev, M, ref = compare_conversion(ac, A, 128, 0, oracle.F64, fmt=ac.FORMAT_RG)
    check_f64(A, x, gpu_spmv(ac, M, x))
    del M, ref
    torch.cuda.empty_cache()


@pytest.mark.parametrize("T", [64, 128])
def test_full_powerlaw_f32(ac, powerlaw_full, T):
    A, x = powerlaw_full
    dev, M, ref = compare_conversion(ac, A, T, 1, oracle.F32)
    acc, tot = check_reduced(A, x, gpu_spmv(ac, M, x.astype(np.float32)), oracle.F32)
    announce(f"powerlaw FP32 T={T}: accumulation err {acc:.2e}, total {tot:.2e}")


@pytest.mark.parametrize("T", [64, 128])
def test_full_stencil_all_dtypes(ac, stencil_full, T):
    A, x = stencil_full
    dev, M, ref = compare_conversion(ac, A, T, 27, oracle.F64)
    check_f64(A, x, gpu_spmv(ac, M, x))
    del M, ref
    for dtype in (1, 2, 3):
        M = ac.convert(dev, T, 27, dtype)
        acc, tot = check_reduced(A, x, gpu_spmv(ac, M, x.astype(np.float32)), dtype)
        announce(f"stencil T={T} dtype={dtype}: accumulation err {acc:.2e}, total {tot:.2e}")
        del M
    torch.cuda.empty_cache()
