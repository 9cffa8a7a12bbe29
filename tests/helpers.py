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


def heavy_chunk_for(T, S, G):
    """The launch-schedule threshold (documented with argcsr_matrix.heavy_groups):
    at least 4 rounds of 8 loaded steps per lane, and 4x the mean chunk size."""
    by_rounds = {64: 32, 128: 16, 256: 8}.get(T)
    if by_rounds is None or G == 0:
        return by_rounds
    return max(by_rounds, 4 * (-(-S // (G * T))))


RUN_SLOTS = 512
RUN_HEAVY = 1


def runs_table(groups, n_slots, n_rows, heavy_chunk):
    """The run schedule documented with argcsr_run_info, from a group table
    (first_row, size, offset, chunk_size per row of `groups`): group g opens a
    run iff g == 0, g or g-1 is heavy, or its offset lies in another window of
    RUN_SLOTS slots than g-1's.  Rows of the result: first_group, offset,
    first_row, flags; the last row is the sentinel."""
    groups = np.asarray(groups, dtype=np.int64).reshape(-1, 4)
    hc = np.iinfo(np.int64).max if heavy_chunk is None else heavy_chunk
    out = []
    for g in range(groups.shape[0]):
        heavy = groups[g, 3] > hc
        if g == 0 or heavy or groups[g - 1, 3] > hc or \
                groups[g, 2] // RUN_SLOTS != groups[g - 1, 2] // RUN_SLOTS:
            out.append([g, groups[g, 2], groups[g, 0], RUN_HEAVY if heavy else 0])
    out.append([groups.shape[0], n_slots, n_rows, 0])
    return np.array(out, dtype=np.int64).reshape(-1, 4)
