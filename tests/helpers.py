"""Shared helpers of the test suite (not product code)."""
import numpy as np

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def gamma(n, u):
    n = np.asarray(n, dtype=np.float64)
    return n * u / (1.0 - n * u)


def row_ids(rp):
    return np.repeat(np.arange(len(rp) - 1), np.diff(rp))


def abs_row_sums(rp, col, val, x):
    """sum_j |a_ij x_j| per row (0 for empty rows)."""
    n = len(rp) - 1
    return np.bincount(row_ids(rp), weights=np.abs(val * x[col]), minlength=n)


def scaled_error(y, y_ref, scale):
    """max_i |y_i - y_ref_i| / scale_i over rows with scale > 0, and whether
    rows with scale == 0 are exactly equal."""
    y = np.asarray(y, dtype=np.float64)
    d = np.abs(y - y_ref)
    nz = scale > 0
    exact_zero_rows = bool(np.all(d[~nz] == 0))
    worst = float(np.max(d[nz] / scale[nz])) if np.any(nz) else 0.0
    return worst, exact_zero_rows


def powerlaw_sample(n, seed=7, lmax=10_000):
    import synth
    s, v, xr = synth.streams(1000 + seed)
    A = synth.powerlaw(n, 2.0, lmax, s, v)
    return A, synth.uniform_vector(A.n_cols, xr)
