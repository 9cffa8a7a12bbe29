"""GPU: the plain-CSR baselines (Sec. 2 definition) against the oracle --
the binned variant (rows grouped by length, a lane count per bin) must bin
every row once, in ascending order within its bin, sum a row of bin k < 7
bitwise as the uniform kernel with 2^k lanes per row does, and stay within
the FP64 bound (reduced types: gamma_{L+1}(2^-24)) everywhere."""
import numpy as np
import pytest
import torch

import oracle
import synth
from conftest import gpu_available
from helpers import powerlaw_sample
from test_gpu_parity import check_f64, check_reduced

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

DEV = "cuda:0"


@pytest.fixture(scope="module")
def ac():
    import paper_1203_5737_amd as ac
    ac._lib.lib()
    return ac


def bins_of(rp):
    """Bin of every row: the smallest k with L <= 2^k, 7 above 64."""
    L = np.diff(rp.astype(np.int64))
    k = np.zeros(L.shape, np.int64)
    for b in range(1, 8):
        k[L > (1 << (b - 1))] = b
    return k


def with_rows(A, lengths_at):
    """A copy of A with the given rows replaced by rows of given lengths
    (columns 0..L-1, values 1/(1+j))."""
    L = np.diff(A.rp).astype(np.int64)
    cols, vals = [], []
    for r in range(A.n_rows):
        if r in lengths_at:
            n = lengths_at[r]
            cols.append(np.arange(n, dtype=np.int32) % A.n_cols)
            vals.append(1.0 / (1.0 + np.arange(n)))
            L[r] = n
        else:
            cols.append(A.col[A.rp[r]:A.rp[r + 1]])
            vals.append(A.val[A.rp[r]:A.rp[r + 1]])
    rp = np.zeros(A.n_rows + 1, np.int32)
    rp[1:] = np.cumsum(L)
    return synth.Csr(A.n_rows, A.n_cols, rp, np.concatenate(cols).astype(np.int32),
                     np.concatenate(vals))


def stored_values(ac, A, dtype):
    """A's values rounded to the storage type as the oracle rounds them
    (nearest-even from FP64), as a device tensor of that type."""
    bits = oracle.round_array(A.val, dtype)
    t = torch.from_numpy(bits.view(np.int16) if bits.dtype == np.uint16 else bits)
    return t.view(ac.storage_dtype(dtype)).to(DEV)


def test_binning_is_a_stable_partition(ac):
    A, x = powerlaw_sample(50_000, seed=12)
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
    b = ac.csr_bins(dev)
    k = bins_of(A.rp)
    want = np.argsort(k, kind="stable").astype(np.int32)
    assert np.array_equal(b.rows.cpu().numpy(), want)
    counts = np.bincount(k, minlength=8)
    assert np.array_equal(b.bin_start, np.concatenate([[0], np.cumsum(counts)]))


@pytest.mark.parametrize("dtype", [0, 1, 2, 3])
def test_binned_matches_oracle_and_uniform_kernel(ac, dtype):
    A0, x = powerlaw_sample(40_000, seed=13)
    # rows of every bin, long rows for the workgroup bin, empty rows
    A = with_rows(A0, {5: 65, 6: 255, 7: 256, 8: 257, 9: 3000, 10: 0, 11: 0, 39_999: 64})
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
    bins = ac.csr_bins(dev)
    vt = ac.vector_dtype(dtype)
    xd = torch.from_numpy(x).to(DEV, vt)
    vals = dev.val if dtype == 0 else stored_values(ac, A, dtype)
    y = ac.csr_spmv_binned(dev, xd, bins, values=vals, dtype=dtype)
    yn = y.cpu().numpy().astype(np.float64)
    if dtype == 0:
        check_f64(A, x, yn)
    else:
        check_reduced(A, x, yn, dtype)
    k = bins_of(A.rp)
    for b in range(7):
        yu = ac.csr_spmv(dev, xd, values=vals, dtype=dtype, lanes_per_row=1 << b).cpu()
        rows = np.nonzero(k == b)[0]
        assert torch.equal(y.cpu()[rows], yu[rows]), f"bin {b}"


def test_binned_full_powerlaw_and_stencil(ac):
    for A, x in (synth.workload_powerlaw(), synth.workload_stencil27(64)):
        dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
        bins = ac.csr_bins(dev)
        y = ac.csr_spmv_binned(dev, torch.from_numpy(x).to(DEV), bins)
        check_f64(A, x, y.cpu().numpy())


def test_binned_edge_cases(ac):
    E = synth.Csr(0, 0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0))
    dev = ac.to_device_csr(E.rp, E.col, E.val, 0, DEV)
    b = ac.csr_bins(dev)
    assert list(b.bin_start) == [0] * 9
    # all rows empty
    Z = synth.Csr(300, 10, np.zeros(301, np.int32), np.zeros(0, np.int32), np.zeros(0))
    dz = ac.to_device_csr(Z.rp, Z.col, Z.val, 10, DEV)
    bz = ac.csr_bins(dz)
    y = ac.csr_spmv_binned(dz, torch.ones(10, dtype=torch.float64, device=DEV), bz)
    assert torch.count_nonzero(y).item() == 0
    # bins that do not cover the rows are refused
    bz.bin_start[8] = 299
    with pytest.raises(ac.ArgCsrError):
        ac.csr_spmv_binned(dz, torch.ones(10, dtype=torch.float64, device=DEV), bz)
