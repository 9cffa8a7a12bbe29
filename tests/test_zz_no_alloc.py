"""argcsr_convert_noalloc, the conversion for callers that cannot allocate
device memory, against argcsr_convert: two calls in a row (the second with a
smaller matrix, so scratch left by the first must not leak into it), every
output array byte for byte equal to argcsr_convert's and to the oracle's, and
the SpMV of the result within the FP64 bound."""
import numpy as np
import pytest
import torch

import oracle
import synth
from conftest import gpu_available
from helpers import abs_row_sums, powerlaw_sample, scaled_error

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

DEV = "cuda:0"


def announce(msg):
    print(f"\n[gpu] {msg}", flush=True)


def same(a: torch.Tensor, b: torch.Tensor) -> bool:
    return a.shape == b.shape and bool(torch.equal(a.view(torch.uint8), b.view(torch.uint8)))


def check_pair(ac, A, T, D, dtype, x64):
    announce(f"noalloc n={A.n_rows} nnz={A.nnz} T={T} D={D} dtype={dtype}")
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
    Mn = ac.convert(dev, T, D, dtype, noalloc=True)
    M = ac.convert(dev, T, D, dtype)
    torch.cuda.synchronize()
    for f in ("groups", "threads_mapping", "columns", "values", "heavy_groups"):
        assert same(getattr(Mn, f), getattr(M, f)), f
    assert (Mn.n_heavy, Mn.heavy_chunk, Mn.nnz) == (M.n_heavy, M.heavy_chunk, M.nnz)
    ref = oracle.convert(A.rp, A.col, A.val, T, D, dtype)
    assert np.array_equal(Mn.groups.cpu().numpy(), ref.groups)
    assert np.array_equal(Mn.threads_mapping.cpu().numpy(), ref.tm)
    assert np.array_equal(Mn.columns.cpu().numpy(), ref.columns)
    if dtype == 0:
        x = torch.from_numpy(x64).to(DEV)
        y = ac.spmv(Mn, x).cpu().numpy()
        y_ref = oracle.csr_spmv(A.rp, A.col, A.val, x64)
        worst, exact = scaled_error(y, y_ref, abs_row_sums(A.rp, A.col, A.val, x64))
        assert exact and worst <= 1e-12


@pytest.fixture(scope="module")
def ac():
    import paper_1203_5737_amd as ac
    ac._lib.lib()
    return ac


def test_noalloc_matches_convert_twice_smaller_second(ac):
    # first the power-law workload at full size (long rows: the fill's
    # long-row list in the fixed scratch), then a much smaller stencil
    A, x = synth.workload_powerlaw()
    check_pair(ac, A, 64, 1, 0, x)
    B = synth.laplace2d(40, 33)
    xb = np.random.default_rng(3).uniform(-1, 1, B.n_cols)
    check_pair(ac, B, 64, 1, 0, xb)
    # and a mid-size power-law sample in a reduced type, then a tiny one
    C, xc = powerlaw_sample(50_000, seed=9)
    check_pair(ac, C, 128, 2, 1, xc)
    Dm = synth.laplace2d(5, 3)
    check_pair(ac, Dm, 64, 1, 3, np.ones(Dm.n_cols))


def test_noalloc_rejects_oversized_scratch_and_device_grouping(ac):
    A = synth.laplace2d(16)
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
    with pytest.raises(ValueError):
        ac.convert(dev, 64, 1, 0, noalloc=True, device_grouping=True)
    # a slot count whose long-row list would not fit the 16 MiB scratch is
    # refused before anything is touched (the sizes are the caller's claim)
    import ctypes
    L = ac._lib
    d = L.MatrixDesc()
    d.n_rows, d.n_cols, d.block_dim, d.desired_chunk_size = A.n_rows, A.n_cols, 64, 1
    d.n_groups, d.n_slots = 4, 2_000_000_000
    rc = L.lib().argcsr_convert_noalloc(A.n_rows, A.n_cols,
                                        A.rp.ctypes.data_as(ctypes.c_void_p), None, None, None,
                                        ctypes.byref(d), None)
    assert rc == L.EINVAL
    assert b"scratch" in L.lib().argcsr_last_error()
