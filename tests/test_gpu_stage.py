"""GPU parity of the staging of x for banded matrices (reading R11 of the
oracle): the tile tables and 16-bit positions made by argcsr_stage_plan /
argcsr_stage must equal the oracle's staging bit for bit, and the staged SpMV
(x read from the group's tiles in LDS, or gathered through the tile table)
must give bitwise the y of the unstaged kernel -- the same products summed in
the same order -- which the other parity tests hold against the oracle; it
is also checked against the oracle's CSR definition here.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from conftest import gpu_available
from helpers import U32, abs_row_sums, gamma, row_ids, scaled_error

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

DEV = "cuda:0"
MAX_TILES = 64          # tiles one group may stage on the GPU


@pytest.fixture(scope="module")
def ac():
    import paper_1203_5737_amd as ac
    ac._lib.lib()
    return ac


def announce(msg):
    print(f"\n[gpu] {msg}", flush=True)


def banded(n, half_band, density, seed, n_cols=None, long_rows=()):
    """Rows i with a random subset of columns in [i - half_band, i + half_band]
    (the diagonal always present), values U[-1, 1]; rows listed in long_rows
    get every column of [i, i + 3000)."""
    rng = np.random.default_rng(seed)
    n_cols = n if n_cols is None else n_cols
    rows = []
    for i in range(n):
        if i in long_rows:
            c = np.arange(i, min(n_cols, i + 3000))
        else:
            lo, hi = max(0, i - half_band), min(n_cols, i + half_band + 1)
            span = np.arange(lo, hi)
            c = span[rng.random(span.size) < density]
            if i < n_cols:
                c = np.union1d(c, [i])
        rows.append(np.asarray(c, dtype=np.int32))
    rp = np.zeros(n + 1, dtype=np.int32)
    rp[1:] = np.cumsum([r.size for r in rows])
    col = np.concatenate(rows) if rows else np.zeros(0, np.int32)
    val = rng.uniform(-1.0, 1.0, col.size)
    return synth.Csr(n, n_cols, rp, col.astype(np.int32), val)


def vec(n, seed, dtype):
    x = np.random.default_rng(seed).uniform(-1.0, 1.0, n)
    return x if dtype == 0 else x.astype(np.float32).astype(np.float64)


def run_case(ac, A, T, D, dtype, gap, x64, check_oracle=True):
    announce(f"stage n={A.n_rows} nnz={A.nnz} T={T} D={D} dtype={dtype} gap={gap}")
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
    M = ac.convert(dev, T, D, dtype)
    ref = oracle.convert(A.rp, A.col, A.val, T, D, dtype)
    st_ref = oracle.stage(ref, gap, MAX_TILES)
    assert st_ref != oracle.STAGE_TOO_MANY_TILES
    Ms = ac.stage(M, gap=gap, lds=True)
    assert Ms.stage_max_tiles == st_ref.max_tiles()
    assert np.array_equal(Ms.tile_ptr.cpu().numpy(), st_ref.tile_ptr)
    assert np.array_equal(Ms.tile_start.cpu().numpy(), st_ref.tile_start)
    assert np.array_equal(Ms.tile_len.cpu().numpy(), st_ref.tile_len)
    assert np.array_equal(Ms.local.cpu().numpy().view(np.uint16), st_ref.local)
    vt = ac.vector_dtype(dtype)
    x = torch.from_numpy(x64).to(DEV).to(vt)
    y0 = ac.spmv(M, x)
    y1 = ac.spmv(Ms, x)
    Mg = ac.stage(M, gap=gap, lds=False, keep_columns=False)
    y2 = ac.spmv(Mg, x)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1), "staged (LDS) y differs from the unstaged y"
    assert torch.equal(y0, y2), "staged (gathered) y differs from the unstaged y"
    if check_oracle:
        y_ref = oracle.argcsr_spmv(ref, x64)
        scale = abs_row_sums(A.rp, A.col, A.val if dtype == 0 else
                             _stored_csr_values(A, ref, dtype), x64)
        if dtype == 0:
            bound = 1e-12
        else:
            bound = float(np.max(gamma(np.diff(A.rp) + 1, U32))) if A.nnz else 0.0
        worst, exact = scaled_error(y1.cpu().numpy().astype(np.float64), y_ref, scale)
        assert exact and worst <= bound, (worst, bound)
    return M, Ms


def _stored_csr_values(A, ref, dtype):
    """The rounded values in CSR order (the oracle's inverse conversion)."""
    rp, col, val = oracle.argcsr_to_csr(ref, A.nnz)
    assert np.array_equal(rp, A.rp) and np.array_equal(col, A.col)
    return val


@pytest.mark.parametrize("dtype", [0, 1, 2, 3])
def test_stage_laplace2d(ac, dtype):
    A = synth.laplace2d(64)
    x = vec(A.n_cols, 1, dtype)
    for T, D, gap in [(64, 1, 0), (64, 5, 3), (128, 5, 0), (256, 5, 62)]:
        run_case(ac, A, T, D, dtype, gap, x)


@pytest.mark.parametrize("dtype", [0, 1])
def test_stage_ragged_grid_and_stencil(ac, dtype):
    A = synth.laplace2d(200, 137)            # ragged: 27400 rows, not a multiple of T
    x = vec(A.n_cols, 2, dtype)
    for T, D, gap in [(64, 5, 0), (128, 1, 0), (256, 5, 200)]:
        run_case(ac, A, T, D, dtype, gap, x)
    s, v, xr = synth.streams(4242)
    B = synth.stencil27_weighted(24, v)
    xb = vec(B.n_cols, 3, dtype)
    for T, D, gap in [(64, 27, 0), (128, 27, 0), (128, 27, 100), (256, 27, 0)]:
        run_case(ac, B, T, D, dtype, gap, xb)


@pytest.mark.parametrize("seed", range(6))
def test_stage_random_banded(ac, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(300, 5000))
    A = banded(n, int(rng.integers(3, 300)), float(rng.uniform(0.05, 0.9)), seed)
    dtype = int(rng.integers(0, 4))
    T = int(rng.choice([64, 128, 256]))
    D = int(rng.choice([1, 2, 8]))
    gap = int(rng.choice([0, 1, 5, 64, 1000]))
    ref = oracle.convert(A.rp, A.col, A.val, T, D, dtype)
    if oracle.stage(ref, gap, MAX_TILES) == oracle.STAGE_TOO_MANY_TILES:
        # a draw with a group of more than 64 tiles: the GPU must refuse it too
        announce(f"stage beyond the tile limit n={A.n_rows} T={T} D={D} gap={gap}")
        M = ac.convert(ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV), T, D, dtype)
        with pytest.raises(ac.ArgCsrError) as e:
            ac.stage(M, gap=gap)
        assert e.value.code == ac._lib.EUNSUPPORTED
        return
    run_case(ac, A, T, D, dtype, gap, vec(A.n_cols, seed, dtype))


def test_stage_heavy_groups_and_empty_rows(ac):
    # long rows (3000 consecutive columns: 47 tiles) make heavy groups, split
    # over the waves of a workgroup; empty rows make padding-only chunks
    A = banded(6000, 20, 0.5, 11, long_rows=(100, 2500, 5990))
    rp = A.rp.copy()
    keep = np.ones(A.nnz, bool)
    for r in range(3000, 3200):                      # rows 3000..3199 emptied
        keep[rp[r]:rp[r + 1]] = False
    L = np.diff(rp)
    L[3000:3200] = 0
    rp2 = np.zeros_like(rp)
    rp2[1:] = np.cumsum(L)
    B = synth.Csr(A.n_rows, A.n_cols, rp2, A.col[keep], A.val[keep])
    for dtype in (0, 1):
        M, Ms = run_case(ac, B, 64, 1, dtype, 0, vec(B.n_cols, 5, dtype))
        assert M.n_heavy > 0


def test_stage_limits(ac):
    # 100 random columns over 10^5 per row: every group (one row) needs 100
    # one-column tiles, more than 64
    s, v, xr = synth.streams(77)
    A = synth.random_csr(np.full(2000, 100), 100_000, s, v)
    ref = oracle.convert(A.rp, A.col, A.val, 64, 1, 0)
    assert oracle.stage(ref, 0, MAX_TILES) == oracle.STAGE_TOO_MANY_TILES
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
    M = ac.convert(dev, 64, 1, 0)
    with pytest.raises(ac.ArgCsrError) as e:
        ac.stage(M, gap=0)
    assert e.value.code == ac._lib.EUNSUPPORTED
    # two columns 2^19 apart in every row: 2 tiles per group, but a span the
    # staging bitmap cannot hold (a limit of the GPU staging, not of the
    # format: the oracle stages it)
    n = 128
    rp = np.arange(0, 2 * n + 1, 2, dtype=np.int32)
    col = np.stack([np.zeros(n, np.int32), np.full(n, 1 << 19, np.int32)], 1).ravel()
    B = synth.Csr(n, (1 << 19) + 1, rp, col, np.ones(2 * n))
    refb = oracle.convert(B.rp, B.col, B.val, 64, 1, 0)
    assert oracle.stage(refb, 0, MAX_TILES).max_tiles() == 2
    Mb = ac.convert(ac.to_device_csr(B.rp, B.col, B.val, B.n_cols, DEV), 64, 1, 0)
    with pytest.raises(ac.ArgCsrError) as e:
        ac.stage(Mb, gap=0)
    assert e.value.code == ac._lib.EUNSUPPORTED
    # an empty matrix stages to nothing
    E = synth.Csr(0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    Me = ac.convert(ac.to_device_csr(E.rp, E.col, E.val, 0, DEV), 64, 1, 0)
    Mse = ac.stage(Me, gap=0)
    assert Mse.n_stage_tiles == 0


@pytest.mark.parametrize("dtype,T", [(0, 64), (0, 128), (1, 128), (2, 128), (3, 128)])
def test_full_stencil_staged(ac, dtype, T):
    """The 27-point stencil 128^3 at D=27 and the block sizes the benchmark
    stages it with (FP64 at T=64, the others at T=128; FP64 at T=128 too):
    staging bit-exact against the oracle, y bitwise the unstaged y."""
    A, x = synth.workload_stencil27(128)
    x64 = x if dtype == 0 else x.astype(np.float32).astype(np.float64)
    run_case(ac, A, T, 27, dtype, 0, x64, check_oracle=(dtype == 0))


def test_autotune_picks_staging_on_the_stencil(ac):
    """The autotuner times every ARG-CSR finalist with x staged as well.  On
    the 27-point stencil 128^3 with FP32 values staging wins by about a
    quarter (cold: ~71 us against ~92 us for the best unstaged layout), so it
    must be chosen; the tuned matrix, staged, gives bitwise the y of the same
    layout unstaged and stays within the FP32 bound of the CSR definition."""
    announce("autotune with staging, stencil 128^3 FP32")
    ac.autotune_clear_cache()
    A, x = synth.workload_stencil27(128)
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
    r = ac.autotune(dev, 1, n_finalists=3)
    announce(f"tuned {r}")
    assert r["n_timed"] == 3 and r["staged"] == 1 and r["format"] == ac.FORMAT_ARG
    M = ac.convert(dev, r["block_dim"], r["desired_chunk_size"], 1)
    Ms = ac.stage(M, 0, True)
    xd = torch.from_numpy(x).to(DEV, torch.float32)
    y0 = ac.spmv(M, xd)
    y1 = ac.spmv(Ms, xd)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1)
    x64 = x.astype(np.float32).astype(np.float64)
    v64 = A.val.astype(np.float32).astype(np.float64)   # FP32 storage rounds to nearest even
    y_ref = np.bincount(row_ids(A.rp), weights=v64 * x64[A.col], minlength=A.n_rows)
    bound = float(np.max(gamma(np.diff(A.rp) + 1, U32)))
    worst, exact = scaled_error(y1.cpu().numpy().astype(np.float64), y_ref,
                                abs_row_sums(A.rp, A.col, v64, x64))
    assert exact and worst <= bound, (worst, bound)
