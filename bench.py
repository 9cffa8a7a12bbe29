"""ARG-CSR SpMV benchmark on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload powerlaw|stencil27|laplace64|mixed|batch|serve]
                    [--dtype f64|f32|bf16|f16] [--block-dim T] [--desired-chunk-size D]
                    [--legs stencil27,batch,serve,ceilings | none]
                    [--warm] [--no-cpu-baseline] [--no-extras]

A step is one y = A x in ARG-CSR (argcsr_spmv) on a matrix converted once
beforehand (conversion time is reported separately).  Inputs are resident in
HBM when timing starts.  By default every step is preceded by a 1 GiB
read-modify-write "flush" (not timed) so that neither the L2s nor the 256 MB
Infinity Cache hold the matrix: the figure is HBM bandwidth, not cache
bandwidth.  Each launch is bracketed by HIP events on the stream it is
launched on; `value` is algorithmic bytes / mean launch time.

Algorithmic bytes per SpMV (the same for every format, so a GB/s ratio is a
speed-up):  nnz*(s_v + 4) + n_rows*(4 + s_y) + n_cols*s_x.

The default run (power-law workload) also carries, as sub-objects of its one
JSON line: the 27-point stencil in FP64/FP32/BF16/FP16 (`stencil27`), the
256-matrix batch in one hipGraph replay (`batch`), the request server under
Poisson arrivals with p50/p99 latency (`serve`), and measured ceilings of the
box (`ceilings`: the flush's copy bandwidth, a streaming read of the
matrix's format bytes, and the random gathers of its column stream).

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ARG-CSR SpMV GB/s (% HBM peak) vs plain CSR; served p50/p99 latency"
HBM_PEAK_GBPS = 8000.0
FLUSH_BYTES = 1 << 30
DTYPES = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}
DTYPE_NAMES = {v: k for k, v in DTYPES.items()}
VALUE_BYTES = {0: 8, 1: 4, 2: 2, 3: 2}
# Sources each measured kernel's HBM traffic depends on: the SpMV kernels;
# with staging of x, the staged kernel and the tile tables; in a batch, the
# batch kernel, its work queue and the member choices of the autotuner.
_CSRC = "paper_1203_5737_amd/csrc/"
SOURCE_SETS = {
    "spmv": [_CSRC + f for f in ("spmv_kernels.hpp", "spmv.hip", "values.hpp", "common.hpp",
                                 "schedule.hpp")],
}
SOURCE_SETS["staged"] = SOURCE_SETS["spmv"] + [_CSRC + f for f in ("spmv_staged.hpp", "stage.hpp",
                                                                   "stage.hip")]
SOURCE_SETS["batch"] = SOURCE_SETS["spmv"] + [_CSRC + f for f in ("batch.hip", "workqueue.hpp",
                                                                  "tune.cpp")]
KERNEL_SOURCES = list(dict.fromkeys(f for v in SOURCE_SETS.values() for f in v))
# (block_dim, desired_chunk_size) per workload unless given on the command line
DEFAULT_PARAMS = {"powerlaw": (64, 1), "stencil27": (128, 27), "laplace64": (64, 1),
                  "mixed": (64, 1)}
DEFAULT_REGION_ROWS = {"mixed": 4096}
# block_dim of the staged 27-point stencil per value type (x tiles in LDS,
# gap 0; a sweep of T in {64, 128, 256} and both ways of reading x on the
# MI355X picked these)
STAGED_STENCIL_T = {"f64": 64, "f32": 128, "bf16": 128, "f16": 128}
ALL_LEGS = ("stencil27", "batch", "serve", "ceilings")


def log(msg: str) -> None:
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash(kind: str = "") -> str:
    """Hash of the sources of one kernel kind (SOURCE_SETS), or of all."""
    h = hashlib.sha256()
    for f in SOURCE_SETS[kind] if kind else KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_kind(workload: str) -> str:
    """The source set a traffic record of `workload` depends on."""
    return ("staged" if workload.endswith("-staged") else
            "batch" if workload == "batch" else "spmv")


def load_workload(name: str):
    import synth
    if name == "powerlaw":
        A, x = synth.workload_powerlaw()
        desc = "power-law rows: n=1e6, L=clip(Zipf(2.0),1,1e4), distinct uniform columns, U[-1,1]"
    elif name == "stencil27":
        A, x = synth.workload_stencil27(128)
        desc = "3D 27-point stencil 128^3, symmetric U[0.5,1.5] couplings, diagonally dominant"
    elif name == "laplace64":
        A, x = synth.workload_laplace64()
        desc = "2D 5-point Laplacian 64x64"
    elif name == "mixed":
        A, x = synth.workload_mixed(64)
        desc = ("mixed regularity: 27-point stencil 64^3 rows, then 64^3 power-law rows "
                "(Zipf(2.0), clip 1e4), n=524288")
    else:
        raise SystemExit(f"unknown workload {name}")
    return A, x, desc


def useful_bytes(A, dtype: int) -> int:
    sv = VALUE_BYTES[dtype]
    sx = 8 if dtype == 0 else 4
    return A.nnz * (sv + 4) + A.n_rows * (4 + sx) + A.n_cols * sx


def format_bytes(M, dtype: int) -> int:
    sv = VALUE_BYTES[dtype]
    sx = 8 if dtype == 0 else 4
    return M.n_slots * (sv + 4) + 16 * M.n_groups + 4 * M.n_rows + sx * (M.n_rows + M.n_cols)


class Timer:
    """Times `fn` launches with HIP events on the current stream, optionally
    evicting the caches (1 GiB read-modify-write) before each launch.  The
    flushes themselves are timed too: their bandwidth (1 GiB read + 1 GiB
    written) is the copy ceiling of the box."""

    def __init__(self, torch, cold: bool):
        self.torch = torch
        self.cold = cold
        self.flush_buf = (torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device="cuda")
                          if cold else None)
        self.flush_ms = []

    def run(self, fn, steps: int):
        torch = self.torch
        ev = lambda: torch.cuda.Event(enable_timing=True)
        starts, ends = [ev() for _ in range(steps)], [ev() for _ in range(steps)]
        fstarts = [ev() for _ in range(steps)] if self.cold else []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            if self.cold:
                fstarts[i].record()
                self.flush_buf.add_(1.0)
            starts[i].record()
            fn()
            ends[i].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
        if self.cold:
            self.flush_ms += [f.elapsed_time(s) for f, s in zip(fstarts, starts)]
        return ms, wall

    def copy_ceiling(self):
        if not self.flush_ms:
            return None
        ms = float(np.median(self.flush_ms))
        return {"gbps": 2 * FLUSH_BYTES / (ms * 1e-3) / 1e9, "median_ms": ms,
                "n": len(self.flush_ms),
                "what": "1 GiB read + 1 GiB written by the untimed flush (torch add_), HIP events"}


def stats(ms):
    return {"mean_ms": float(ms.mean()), "median_ms": float(np.median(ms)),
            "p10_ms": float(np.percentile(ms, 10)), "p90_ms": float(np.percentile(ms, 90))}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_convert(A, T, D, region_rows, regions, budget_s: float = 6.0):
    """CSR -> ARG-CSR by the oracle (single-threaded C, FP64 values): median
    time of up to 3 conversions of the whole matrix within `budget_s`."""
    import oracle
    ts = []
    while len(ts) < 3 and sum(ts) < budget_s / 2:
        t0 = time.perf_counter()
        if regions is not None:
            oracle.convert_regions(A.rp, A.col, A.val, T, region_rows, regions)
        else:
            oracle.convert(A.rp, A.col, A.val, T, D)
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)) * 1e3, len(ts)


def cpu_baseline(A, x, B_useful, budget_s: float = 16.0):
    """The FP64 CSR oracle on this host's cores (OpenMP row split; identical
    result to the sequential oracle): the median of at least 5 reps, each a
    batch of full SpMVs, within about `budget_s` seconds; then the same
    single-threaded, as in the paper's sequential baseline."""
    import oracle
    threads = os.cpu_count() or 1
    oracle.csr_spmv(A.rp, A.col, A.val, x, threads)           # warm-up
    t0 = time.perf_counter()
    oracle.csr_spmv(A.rp, A.col, A.val, x, threads)
    one = max(time.perf_counter() - t0, 1e-6)
    reps = 7
    per_rep = int(max(1, min(20_000, budget_s * 0.6 / reps / one)))
    rep_ms = []
    for _ in range(reps):
        t0 = time.perf_counter()
        for _ in range(per_rep):
            oracle.csr_spmv(A.rp, A.col, A.val, x, threads)
        rep_ms.append((time.perf_counter() - t0) / per_rep * 1e3)
    mt = float(np.median(rep_ms))
    st_ms = []
    for _ in range(5):
        t0 = time.perf_counter()
        oracle.csr_spmv(A.rp, A.col, A.val, x, 1)
        st_ms.append((time.perf_counter() - t0) * 1e3)
        if sum(st_ms) > budget_s * 400:                        # 40% of the budget, in ms
            break
    st = float(np.median(st_ms))
    return {"value": B_useful / (mt * 1e-3) / 1e9, "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": f"full matrix; median of {reps} reps of {per_rep} SpMVs on {threads} threads "
                      f"(OpenMP row split), and median of {len(st_ms)} single-threaded SpMVs",
            "ms_per_spmv": mt, "rep_ms": rep_ms, "single_thread_gbps": B_useful / (st * 1e-3) / 1e9,
            "single_thread_ms": st, "cpu_model": cpu_model()}


def error_vs_fp64(A, x, y):
    """y from the GPU against y = A x computed here in FP64 with numpy (every
    row, original values and x): the largest row error scaled by the row's
    sum |a_ij x_j|, and the relative 2-norm error.  For reduced-precision
    storage this is the total error (value rounding, FP32 x and accumulation)."""
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.rp))
    prod = A.val * x[A.col]
    ref = np.bincount(rows, weights=prod, minlength=A.n_rows)
    scale = np.bincount(rows, weights=np.abs(prod), minlength=A.n_rows)
    d = np.abs(np.asarray(y, dtype=np.float64) - ref)
    live = scale > 0
    return {"max_scaled": float(np.max(d[live] / scale[live])) if live.any() else 0.0,
            "zero_rows_exact": bool(np.all(d[~live] == 0)),
            "rel_l2": float(np.linalg.norm(d) / max(np.linalg.norm(ref), 1e-300))}


def traffic_for(workload: str, dtype_name: str, T: int, D: int):
    """HBM bytes per launch measured by rocprofv3 FETCH_SIZE/WRITE_SIZE for
    the current sources of the kernel (None when absent or those sources have
    changed since the counters were taken)."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    want = f"{workload}/{dtype_name}/T{T}/D{D}"
    for line in open(path):
        f = line.split()
        # key  kernel_hash  fetch_bytes  write_bytes  (scaled, per launch)
        if (len(f) >= 4 and not line.startswith("#") and f[0] == want
                and f[1] == kernel_source_hash(traffic_kind(workload))):
            return int(f[2]) + int(f[3])
    return None


def best_csr(ac, timer, dev, xd, yd, vals, dtype, steps, lanes=(0, 1, 2, 4, 8, 16, 32, 64)):
    """Plain CSR on the same GPU with the best lanes-per-row of a sweep."""
    best = None
    for V in lanes:
        f = lambda V=V: ac.csr_spmv(dev, xd, yd, values=vals, dtype=dtype, lanes_per_row=V)
        timer.run(f, 3)
        t, _ = timer.run(f, max(10, steps // 5))
        if best is None or t.mean() < best[1].mean():
            best = (V, t)
    V, _ = best
    f = lambda: ac.csr_spmv(dev, xd, yd, values=vals, dtype=dtype, lanes_per_row=V)
    t, _ = timer.run(f, steps)
    return V, t


def binned_csr(ac, timer, dev, xd, yd, vals, dtype, steps):
    """Plain CSR with rows binned by length, a lane count per bin."""
    bins = ac.csr_bins(dev)
    f = lambda: ac.csr_spmv_binned(dev, xd, bins, yd, values=vals, dtype=dtype)
    timer.run(f, 3)
    t, _ = timer.run(f, steps)
    return t, [int(v) for v in np.diff(bins.bin_start)]


def f32_variant(A, x, dev, timer, torch, ac, steps):
    """The same matrix with FP32 values, x and y (T=128, D=1), against plain
    CSR in FP32, timed the same way."""
    B = useful_bytes(A, 1)
    M = ac.convert(dev, 128, 1, 1)
    xd = torch.from_numpy(x).to("cuda", torch.float32)
    yd = torch.empty(A.n_rows, dtype=torch.float32, device="cuda")
    f = lambda: ac.spmv(M, xd, yd)
    timer.run(f, 5)
    t, _ = timer.run(f, steps)
    vals = dev.val.to(torch.float32)
    V, c = best_csr(ac, timer, dev, xd, yd, vals, 1, max(10, steps // 2), (8, 16, 32, 64))
    cb, _ = binned_csr(ac, timer, dev, xd, yd, vals, 1, max(10, steps // 2))
    ac.spmv(M, xd, yd)
    err = error_vs_fp64(A, x, yd.cpu().numpy())
    gbps = B / (t.mean() * 1e-3) / 1e9
    return {"block_dim": 128, "desired_chunk_size": 1, "mean_ms": float(t.mean()),
            "gbps": gbps, "frac": gbps / HBM_PEAK_GBPS,
            "csr_gbps": B / (c.mean() * 1e-3) / 1e9,
            "csr_binned_gbps": B / (cb.mean() * 1e-3) / 1e9,
            "csr_lanes_per_row": V,
            "speedup_vs_csr": float(min(c.mean(), cb.mean()) / t.mean()),
            "error_vs_fp64": err}


# ---------------------------------------------------------------------------
# legs of the default run
# ---------------------------------------------------------------------------

def tuned_record(ac, dev, dtype, xd, yd, timer, steps):
    """What argcsr_autotune picks for the matrix (4 finalists timed cold by
    the tuner, each ARG-CSR finalist also with x staged), converted (and
    staged when chosen) and timed here the same way as the fixed choice."""
    r = ac.autotune(dev, dtype, n_finalists=4)
    M = ac.convert(dev, r["block_dim"], r["desired_chunk_size"], dtype, fmt=r["format"])
    if r["staged"]:
        M = ac.stage(M, 0, True)
    f = lambda: ac.spmv(M, xd, yd)
    timer.run(f, 3)
    t, _ = timer.run(f, steps)
    B = useful_bytes_of(dev, dtype)
    return stats(t) | {"block_dim": r["block_dim"], "desired_chunk_size": r["desired_chunk_size"],
                       "format": "row-grouped" if r["format"] else "ARG-CSR",
                       "x_staged": bool(r["staged"]),
                       "tuner_median_us": r["measured_us"], "model_us": r["model_us"],
                       "candidates_timed": r["n_timed"],
                       "gbps": B / (t.mean() * 1e-3) / 1e9}


def useful_bytes_of(dev, dtype: int) -> int:
    sv = VALUE_BYTES[dtype]
    sx = 8 if dtype == 0 else 4
    return dev.nnz * (sv + 4) + dev.n_rows * (4 + sx) + dev.n_cols * sx


def leg_stencil27(torch, ac, timer, steps):
    """27-point stencil 128^3 (T=128, D=27) in every value type, cold, with
    the error against FP64 and plain CSR (FP64) beside it."""
    A, x, desc = load_workload("stencil27")
    T, D = DEFAULT_PARAMS["stencil27"]
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, "cuda")
    out = {"workload": desc, "n_rows": A.n_rows, "nnz": A.nnz, "block_dim": T,
           "desired_chunk_size": D, "steps": steps}
    for name, dtype in DTYPES.items():
        log(f"stencil27 {name}")
        M = ac.convert(dev, T, D, dtype)
        vdt = ac.vector_dtype(dtype)
        xd = torch.from_numpy(x).to("cuda", vdt)
        yd = torch.empty(A.n_rows, dtype=vdt, device="cuda")
        f = lambda: ac.spmv(M, xd, yd)
        timer.run(f, 3)
        t, _ = timer.run(f, steps)
        B = useful_bytes(A, dtype)
        gbps = B / (t.mean() * 1e-3) / 1e9
        rec = stats(t) | {"gbps": gbps, "frac": gbps / HBM_PEAK_GBPS, "useful_bytes": B,
                          "padding_ratio": M.n_slots / A.nnz,
                          "traffic": traffic_for("stencil27", name, T, D),
                          "error_vs_fp64": error_vs_fp64(A, x, yd.cpu().numpy())}
        if dtype == 0:
            V, c = best_csr(ac, timer, dev, xd, yd, dev.val, 0, steps, (4, 8, 16, 32))
            cb, _ = binned_csr(ac, timer, dev, xd, yd, dev.val, 0, steps)
            rec["csr_gbps"] = B / (c.mean() * 1e-3) / 1e9
            rec["csr_binned_gbps"] = B / (cb.mean() * 1e-3) / 1e9
            rec["csr_lanes_per_row"] = V
            c = c if c.mean() <= cb.mean() else cb
            rec["speedup_vs_csr"] = float(c.mean() / t.mean())
            rec["tuned"] = tuned_record(ac, dev, dtype, xd, yd, timer, steps)
        # x staged per group in LDS, 16-bit positions instead of columns
        Ts = STAGED_STENCIL_T[name]
        if Ts != T:
            del M
            M = ac.convert(dev, Ts, D, dtype)
        Ms = ac.stage(M, gap=0, lds=True, keep_columns=False)
        fs = lambda: ac.spmv(Ms, xd, yd)
        timer.run(fs, 3)
        ts, _ = timer.run(fs, steps)
        gs = B / (ts.mean() * 1e-3) / 1e9
        rec["staged"] = stats(ts) | {
            "block_dim": Ts, "gap": 0, "x_in_lds": True, "gbps": gs, "frac": gs / HBM_PEAK_GBPS,
            "max_group_tiles": Ms.stage_max_tiles, "tiles": Ms.n_stage_tiles,
            "format_bytes_staged": Ms.n_slots * (VALUE_BYTES[dtype] + 2),
            "speedup_vs_plain": float(t.mean() / ts.mean()),
            "traffic": traffic_for("stencil27-staged", name, Ts, D),
            "error_vs_fp64": error_vs_fp64(A, x, yd.cpu().numpy())}
        if "csr_gbps" in rec:
            rec["staged"]["speedup_vs_csr"] = gs / max(rec["csr_gbps"], rec["csr_binned_gbps"])
        out[name] = rec
        del M, Ms, xd, yd
    del dev
    torch.cuda.empty_cache()
    return out


def batch_record(torch, ac, count, dtype, steps, warmup, cold=True, extras=True):
    """`count` matrices (n log-uniform in [1e3, 2e5], half U{5..50} nonzeros
    per row, half clip(Zipf(2.2), 1, min(5000, n))), (T, D, format) chosen
    per matrix by argcsr_autotune_member (the batch-throughput model); a step
    is ONE replay of the
    batch's hipGraph (queue reset + persistent kernel over all matrices'
    groups)."""
    import synth
    mats = synth.workload_batch(count)
    vdt = ac.vector_dtype(dtype)
    devs, Ms, xs, ys, tunes = [], [], [], [], []
    t0 = time.perf_counter()
    for A, x in mats:
        d = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, "cuda")
        # ranked by the batch-throughput model, not timed: a small matrix
        # timed alone favours more groups than it needs among 255 others
        r = ac.autotune_member(A.rp, dtype)
        tunes.append((r["block_dim"], r["desired_chunk_size"], r["from_cache"], r["format"]))
        Ms.append(ac.convert(d, r["block_dim"], r["desired_chunk_size"], dtype, fmt=r["format"]))
        devs.append(d)
        xs.append(torch.from_numpy(x).to("cuda", vdt))
        ys.append(torch.empty(A.n_rows, dtype=vdt, device="cuda"))
    setup_s = time.perf_counter() - t0
    log(f"batch: {count} matrices tuned and converted in {setup_s:.1f} s")
    B = sum(useful_bytes(A, dtype) for A, _ in mats)
    nnz = sum(A.nnz for A, _ in mats)
    batch = ac.Batch(Ms, xs, ys)
    timer = Timer(torch, cold=cold)
    run = lambda: batch.launch(graph=True)
    timer.run(run, warmup)
    ms, wall = timer.run(run, steps)
    gbps = B / (ms.mean() * 1e-3) / 1e9
    # every member against y = A x in FP64 (numpy), after the last replay
    errs = [error_vs_fp64(A, x, y.cpu().numpy()) for (A, x), y in zip(mats, ys)]
    rec = {"workload": f"batch of {count} matrices, n log-uniform [1e3,2e5], half U{{5..50}} "
                       "nnz/row, half clip(Zipf(2.2),1,min(5000,n)); (T, D) by the batch-member model "
                       "per matrix; one hipGraph replay per step",
           "n_mats": count, "n_rows": sum(A.n_rows for A, _ in mats), "nnz": nnz,
           "value_dtype": DTYPE_NAMES[dtype], "useful_bytes": B, "gbps": gbps,
           "frac": gbps / HBM_PEAK_GBPS, "steps": steps,
           "traffic": traffic_for("batch", DTYPE_NAMES[dtype], "auto", "auto"),
           "spmv": stats(ms) | {"gflops": 2 * nnz / (ms.mean() * 1e-3) / 1e9,
                                "wall_ms_per_step": wall * 1e3 / steps} | batch.info(),
           "error_vs_fp64": {"max_scaled": max(e["max_scaled"] for e in errs),
                             "max_rel_l2": max(e["rel_l2"] for e in errs),
                             "zero_rows_exact": all(e["zero_rows_exact"] for e in errs)},
           "setup_s": setup_s,
           "tuned": {(f"T{T}/RG" if fm else f"T{T}/D{D}"): sum(1 for t in tunes
                                                             if (t[0], t[1], t[3]) == (T, D, fm))
                     for T, D, fm in sorted({(t[0], t[1], t[3]) for t in tunes})}}
    if extras:
        loop = lambda: [ac.spmv(M, x, y) for M, x, y in zip(Ms, xs, ys)]
        timer.run(loop, 2)
        t, _ = timer.run(loop, max(5, steps // 4))
        rec["single_launch_loop"] = stats(t) | {"gbps": B / (t.mean() * 1e-3) / 1e9}
        vals = [d.val.to(ac.storage_dtype(dtype)) if dtype != 0 else d.val for d in devs]
        csr = lambda: [ac.csr_spmv(d, x, y, values=v, dtype=dtype)
                       for d, x, y, v in zip(devs, xs, ys, vals)]
        timer.run(csr, 2)
        t, _ = timer.run(csr, max(5, steps // 4))
        rec["csr_loop"] = stats(t) | {"gbps": B / (t.mean() * 1e-3) / 1e9}
        bins = [ac.csr_bins(d) for d in devs]
        binned = lambda: [ac.csr_spmv_binned(d, x, b, y, values=v, dtype=dtype)
                          for d, x, y, v, b in zip(devs, xs, ys, vals, bins)]
        timer.run(binned, 2)
        tb, _ = timer.run(binned, max(5, steps // 4))
        rec["csr_binned_loop"] = stats(tb) | {"gbps": B / (tb.mean() * 1e-3) / 1e9}
        rec["speedup_vs_csr_loop"] = (min(rec["csr_loop"]["mean_ms"],
                                          rec["csr_binned_loop"]["mean_ms"]) / float(ms.mean()))
    batch.close()
    del Ms, devs, xs, ys
    torch.cuda.empty_cache()
    return rec


def serve_record(ac, pool_size, n_requests, n_warm, rate, budget_gb, budget_frac, max_active,
                 cg_inner_per_step, n_check=16):
    """Open-loop serving: Poisson arrivals at `rate` req/s of SpMV and CG
    requests (50/50) on SPD shifted 2D/3D Laplacians with n log-uniform in
    [1e4, 1e6]; request matrix ~ Zipf(1.1) over a pool of `pool_size`
    matrices, each generated from its own seed (only the ones the request
    sequence names).  Every request is submitted as ADMIT (a no-op when the
    matrix is resident) followed by the SpMV or CG.  The device budget is
    `budget_gb`, or, when that is 0, `budget_frac` of the device footprint of
    the matrices the run uses, so that admissions have to evict.  Latency runs
    from the scheduled arrival to the result in host memory; a failed request
    counts as infinitely late."""
    from concurrent.futures import ThreadPoolExecutor
    import synth
    from paper_1203_5737_amd import serve
    rng = np.random.default_rng(np.random.SeedSequence([12035737, 4, 999999]))
    P = pool_size
    zipf_w = 1.0 / np.arange(1, P + 1) ** 1.1
    zipf_w /= zipf_w.sum()
    n_req = n_requests + n_warm
    mats = rng.choice(P, size=n_req, p=zipf_w)
    kinds = rng.random(n_req) < 0.5                      # True: CG
    gaps = rng.exponential(1.0 / rate, n_req)
    used = sorted(set(int(m) for m in mats))
    t0 = time.perf_counter()
    with ThreadPoolExecutor(8) as ex:
        pool = dict(zip(used, ex.map(lambda i: synth.serve_pool_matrix(i)[0], used)))
    gen_s = time.perf_counter() - t0
    log(f"serve: {len(used)} matrices generated in {gen_s:.1f} s")
    inputs = [rng.uniform(-1, 1, pool[m].n_rows) if cg else
              rng.uniform(-1, 1, pool[m].n_cols).astype(np.float32)
              for m, cg in zip(mats, kinds)]
    # device footprint of a resident matrix: groups, mapping, columns, FP64
    # and FP32 values, heavy list (the server's layout)
    T = 64
    foot = 0
    for m in used:
        A = pool[m]
        D = int(min(64, max(1, round(A.nnz / max(A.n_rows, 1)))))
        G, S, H = ac.plan(A.rp, T, D)
        foot += 16 * G + 4 * A.n_rows + 16 * S + 4 * max(H, 1)
    budget = int(budget_gb * (1 << 30)) if budget_gb > 0 else int(budget_frac * foot)
    srv = serve.Server(budget_bytes=budget, max_active=max_active, cg_tol=1e-10,
                       cg_inner_per_step=cg_inner_per_step)
    records = []
    tstart = time.monotonic_ns() + 50_000_000
    arrivals = tstart + np.cumsum(gaps * 1e9).astype(np.int64)
    for k in range(n_req):
        while time.monotonic_ns() < arrivals[k]:
            pass
        m = int(mats[k])
        A = pool[m]
        ta = srv.admit(m, A.rp, A.col, A.val, A.n_cols)
        if kinds[k]:
            t, out = srv.cg(m, inputs[k])
        else:
            t, out = srv.spmv(m, inputs[k], A.n_rows)
        records.append((t, ta, int(arrivals[k]), bool(kinds[k]), m, out))
    log(f"serve: {n_req} requests submitted")
    results = []
    for t, ta, arr, cg, m, out in records:
        r = srv.wait(t, 600.0)
        ra = srv.wait(ta, 600.0)
        cold = ra["status"] == 0 and ra["iterations"] == 1
        srv.release(ta)
        results.append((r, arr, cold, cg, m, out))
    wall = (max(r["t_done_ns"] for r, *_ in results) - tstart) * 1e-9
    st = srv.stats()
    srv.close()
    meas = results[n_warm:]

    def lat(xs):
        return np.array([(r["t_done_ns"] - arr) * 1e-6 if r["status"] == 0 else np.inf
                         for r, arr, *_ in xs])

    def pct(xs):
        a = lat(xs)
        return {"n": int(a.size), "p50_ms": float(np.percentile(a, 50)) if a.size else None,
                "p99_ms": float(np.percentile(a, 99)) if a.size else None}

    ok_idx = [k for k in range(n_warm, n_req) if results[k][0]["status"] == 0]
    ok = [results[k] for k in ok_idx]
    # a sample of the results checked here with numpy (CSR definition in
    # FP64): SpMV within the FP32 dot-product bound on the FP32-rounded
    # values, CG by its true residual
    check = {"spmv_checked": 0, "spmv_ok": 0, "cg_checked": 0, "cg_max_true_relres": 0.0}
    srng = np.random.default_rng(7)
    for k in [ok_idx[i] for i in srng.permutation(len(ok_idx))[:n_check]]:
        r, arr, cold, cg, m, out = results[k]
        A = pool[m]
        rows = np.repeat(np.arange(A.n_rows), np.diff(A.rp))
        inp = inputs[k]
        if cg:
            Ax = np.bincount(rows, weights=A.val * out[A.col], minlength=A.n_rows)
            rr = float(np.linalg.norm(inp - Ax) / np.linalg.norm(inp))
            check["cg_checked"] += 1
            check["cg_max_true_relres"] = max(check["cg_max_true_relres"], rr)
        else:
            v32 = A.val.astype(np.float32).astype(np.float64)
            xx = inp.astype(np.float64)
            prod = v32 * xx[A.col]
            ref = np.bincount(rows, weights=prod, minlength=A.n_rows)
            scale = np.bincount(rows, weights=np.abs(prod), minlength=A.n_rows)
            L = np.diff(A.rp) + 1
            u = 2.0 ** -24
            good = np.all(np.abs(out.astype(np.float64) - ref) <= L * u / (1 - L * u) * scale)
            check["spmv_checked"] += 1
            check["spmv_ok"] += int(good)
    warm = [x for x in meas if not x[2]]
    coldr = [x for x in meas if x[2]]
    sp_bytes = sum(useful_bytes(pool[m], 1) * (1 if not cg else max(1, r["iterations"]))
                   for r, _, _, cg, m, _ in ok)
    return {
        "workload": f"serving: Poisson {rate:g} req/s, 50% SpMV / 50% CG to 1e-10, pool of {P} SPD "
                    f"shifted 2D/3D Laplacians (n log-uniform [1e4,1e6], Zipf(1.1) popularity), "
                    f"budget {budget / (1 << 30):.2f} GiB"
                    + ("" if budget_gb > 0 else
                       f" = {budget_frac:g} x the {foot / (1 << 30):.2f} GiB device footprint of the "
                       f"{len(used)} matrices the requests use"),
        "requests": n_requests, "warm_up_requests": n_warm, "max_active": max_active,
        "cg_inner_per_step": cg_inner_per_step or 2,
        "p50_ms": pct(meas)["p50_ms"], "p99_ms": pct(meas)["p99_ms"],
        "latency": {"all": pct(meas), "warm": pct(warm), "cold": pct(coldr),
                    "spmv": pct([x for x in meas if not x[3]]),
                    "cg": pct([x for x in meas if x[3]])},
        "throughput_req_s": len(results) / wall,
        "aggregate_spmv_gbps_lower_bound": sp_bytes / wall / 1e9,
        "failed": len(meas) - len(ok),
        "cg_max_relres": max((r["relres"] for r, _, _, cg, _, _ in ok if cg), default=None),
        "cg_mean_iterations": float(np.mean([r["iterations"] for r, _, _, cg, _, _ in ok if cg] or [0])),
        "check": check,
        "pool_generation_s": gen_s, "matrices_used": len(used),
        "footprint_bytes": foot, "budget_bytes": budget,
        "server": st,
    }


def leg_ceilings(torch, ac, M, dtype, timer, steps):
    """Measured ceilings of the box for this matrix: a streaming read of its
    format bytes (values + columns, 16-byte loads) and the random gathers of
    its column stream alone (every column of the slots, x[column] summed,
    no values and no row sums), both cold like the SpMV."""
    out = {}
    sink = torch.empty(ac.PROBE_SINK_ELEMS, dtype=torch.float64, device="cuda")
    fb = M.n_slots * (VALUE_BYTES[dtype] + 4)
    f = lambda: (ac.probe_read(M.values, sink), ac.probe_read(M.columns, sink))
    timer.run(f, 3)
    t, _ = timer.run(f, steps)
    out["stream_read"] = {"gbps": fb / (t.mean() * 1e-3) / 1e9, "bytes": fb, **stats(t),
                          "what": "values and columns read once, 16-byte non-temporal loads"}
    x = torch.zeros(M.n_cols, dtype=ac.vector_dtype(dtype), device="cuda")
    g = lambda: ac.probe_gather(M.columns, x, sink)
    timer.run(g, 3)
    t, _ = timer.run(g, steps)
    n_g = M.nnz
    out["gather"] = {"gathers_per_s": n_g / (t.mean() * 1e-3), "gathers": n_g, **stats(t),
                     "column_bytes_gbps": 4 * M.n_slots / (t.mean() * 1e-3) / 1e9,
                     "what": "the column stream read and x[column] gathered and summed"}
    return out


# ---------------------------------------------------------------------------
# standalone workloads
# ---------------------------------------------------------------------------

def run_batch(args, torch, ac):
    dtype = DTYPES[args.dtype]
    rec = batch_record(torch, ac, args.batch_count, dtype, args.steps, args.warmup,
                       cold=not args.warm, extras=not args.no_extras)
    out = {"metric": METRIC, "value": round(rec["gbps"], 2), "unit": "GB/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": rec["spmv"]["mean_ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": args.dtype, "data": "synthetic",
           "config": {"workload": rec["workload"], "n_rows": rec["n_rows"], "nnz": rec["nnz"],
                      "value_dtype": args.dtype,
                      "timing": "warm" if args.warm else "cold (1 GiB flush before each step, untimed)"},
           "roofline": {"bound": "hbm", "achieved": round(rec["gbps"], 2), "peak": HBM_PEAK_GBPS,
                        "unit": "GB/s", "frac": round(rec["frac"], 4), "traffic": rec["traffic"]},
           "batch": rec, "kernel_hash": kernel_source_hash()}
    print(json.dumps(out))


def run_serve(args, torch, ac):
    rec = serve_record(ac, args.pool, args.requests, args.warm_requests, args.rate,
                       args.budget_gb, args.budget_frac, args.max_active, args.cg_inner_per_step)
    out = {"metric": METRIC, "value": rec["p50_ms"], "unit": "ms (p50 latency)", "n_gpus": 1,
           "steps": args.requests, "warmup": args.warm_requests,
           "ms_per_step": float(rec["latency"]["all"]["p50_ms"]), "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32 SpMV / f64 CG",
           "data": "synthetic", "config": {"workload": rec["workload"]}, "serve": rec}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="powerlaw")
    ap.add_argument("--dtype", default="f64", choices=list(DTYPES))
    ap.add_argument("--block-dim", type=int, default=None)
    ap.add_argument("--desired-chunk-size", type=int, default=None)
    ap.add_argument("--region-rows", type=int, default=None,
                    help="desiredChunkSize per region of this many rows (0: one D)")
    ap.add_argument("--legs", default=",".join(ALL_LEGS),
                    help="extra legs of the power-law run: comma list of "
                         f"{', '.join(ALL_LEGS)}, or 'none'")
    ap.add_argument("--warm", action="store_true", help="no cache flush between steps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the CSR and warm timings")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--rate", type=float, default=1000.0, help="serve: arrivals per second")
    ap.add_argument("--requests", type=int, default=2000, help="serve: measured requests")
    ap.add_argument("--warm-requests", type=int, default=200, help="serve: unmeasured first requests")
    ap.add_argument("--pool", type=int, default=512, help="serve: distinct matrices")
    ap.add_argument("--cg-inner-per-step", type=int, default=0,
                    help="serve: inner CG iterations a step may run (0 = the server's default)")
    ap.add_argument("--budget-gb", type=float, default=0.0,
                    help="serve: device memory budget (0: --budget-frac of the footprint used)")
    ap.add_argument("--budget-frac", type=float, default=0.4,
                    help="serve: budget as a fraction of the used matrices' device footprint")
    ap.add_argument("--max-active", type=int, default=64, help="serve: requests per step")
    ap.add_argument("--stage-gap", type=int, default=-1,
                    help="stage x per group with this window gap (-1: no staging)")
    ap.add_argument("--stage-lds", type=int, default=1,
                    help="staged SpMV reads x from LDS (1) or gathers it through the tile table (0)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_1203_5737_amd as ac

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    ac._lib.lib()                                    # fails loudly if not built
    if args.workload == "serve":
        return run_serve(args, torch, ac)
    if args.workload == "batch":
        if args.dtype == "f64" and "--dtype" not in sys.argv:
            args.dtype = "f32"                        # the batch workload is quoted in FP32
        return run_batch(args, torch, ac)
    legs = [] if args.legs in ("", "none") else args.legs.split(",")
    for leg in legs:
        if leg not in ALL_LEGS:
            raise SystemExit(f"unknown leg {leg}")
    if args.workload != "powerlaw":
        legs = [leg for leg in legs if leg == "ceilings"]
    dtype = DTYPES[args.dtype]
    T0, D0 = DEFAULT_PARAMS.get(args.workload, (64, 1))
    T = args.block_dim or T0
    D = args.desired_chunk_size or D0

    log(f"{args.workload}: generating")
    A, x, desc = load_workload(args.workload)
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, "cuda")
    torch.cuda.synchronize()
    log(f"{args.workload}: n={A.n_rows} nnz={A.nnz}; converting")
    region_rows = (args.region_rows if args.region_rows is not None
                   else DEFAULT_REGION_ROWS.get(args.workload, 0))
    regions = ac.choose_region_desired(A.rp, region_rows) if region_rows else None
    conv = lambda **kw: ac.convert(dev, T, D, dtype, region_rows=region_rows,
                                   region_desired=regions, **kw)

    # conversion (timed separately, host grouping included)
    t0 = time.perf_counter()
    M = conv()
    convert_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    M = conv()
    convert_ms = min(convert_ms, (time.perf_counter() - t0) * 1e3)
    # the same with conversion step 1 on the device (no host row_ptr pass)
    convert_device_ms = float("inf")
    for _ in range(2):
        t0 = time.perf_counter()
        Md = conv(device_grouping=True)
        convert_device_ms = min(convert_device_ms, (time.perf_counter() - t0) * 1e3)
        del Md

    vdt = ac.vector_dtype(dtype)
    xd = torch.from_numpy(x).to("cuda", vdt)
    yd = torch.empty(A.n_rows, dtype=vdt, device="cuda")
    B = useful_bytes(A, dtype)
    Bf = format_bytes(M, dtype)
    staging = None
    if args.stage_gap >= 0:
        M = ac.stage(M, gap=args.stage_gap, lds=bool(args.stage_lds))
        staging = {"gap": args.stage_gap, "x_in_lds": bool(args.stage_lds),
                   "max_group_tiles": M.stage_max_tiles, "tiles": M.n_stage_tiles}
    traffic_key = args.workload + ("-staged" if staging else "")

    timer = Timer(torch, cold=not args.warm)
    spmv = lambda: ac.spmv(M, xd, yd)
    log(f"{args.workload}: timing {args.steps} SpMVs")
    timer.run(spmv, args.warmup)
    ms, wall = timer.run(spmv, args.steps)
    mean_s = ms.mean() * 1e-3
    gbps = B / mean_s / 1e9

    out = {
        "metric": METRIC, "value": round(gbps, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": float(ms.mean()),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": desc, "n_rows": A.n_rows, "nnz": A.nnz, "block_dim": T,
                   "desired_chunk_size": D if regions is None else "per region",
                   "region_rows": region_rows or None, "value_dtype": args.dtype,
                   "timing": "warm" if args.warm else "cold (1 GiB flush before each step, untimed)"},
        "roofline": {"bound": "hbm", "achieved": round(gbps, 2), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBPS, 4),
                     "traffic": traffic_for(traffic_key, args.dtype, T, D)},
        "spmv": stats(ms) | {"gflops": 2 * A.nnz / mean_s / 1e9, "useful_bytes": B,
                             "format_bytes": Bf, "padding_ratio": M.n_slots / max(A.nnz, 1),
                             "n_groups": M.n_groups, "wall_ms_per_step": wall * 1e3 / args.steps},
        "convert_ms": convert_ms,
        "convert_device_grouping_ms": convert_device_ms,
        "kernel_hash": kernel_source_hash(),
        "error_vs_fp64": error_vs_fp64(A, x, yd.cpu().numpy()),
    }
    if staging:
        out["staging"] = staging

    if not args.no_extras:
        log("extras: warm, plain CSR, FP32, row-grouped")
        # the same SpMV without flushes (matrix may stay in the Infinity Cache)
        warm_ms, _ = Timer(torch, cold=False).run(spmv, args.steps)
        out["spmv_warm"] = stats(warm_ms) | {"gbps": B / (warm_ms.mean() * 1e-3) / 1e9}
        # plain CSR on the same GPU, same timing; best lanes-per-row of a sweep
        vals = dev.val if dtype == 0 else dev.val.to(ac.storage_dtype(dtype))
        V, t = best_csr(ac, timer, dev, xd, yd, vals, dtype, args.steps)
        csr_gbps = B / (t.mean() * 1e-3) / 1e9
        out["csr"] = stats(t) | {"gbps": csr_gbps, "lanes_per_row": V}
        tb, counts = binned_csr(ac, timer, dev, xd, yd, vals, dtype, args.steps)
        binned_gbps = B / (tb.mean() * 1e-3) / 1e9
        out["csr_binned"] = stats(tb) | {"gbps": binned_gbps, "rows_per_bin": counts}
        # against the better of the two plain-CSR kernels
        out["speedup_vs_csr"] = gbps / max(csr_gbps, binned_gbps)
        if dtype == 0 and args.workload == "powerlaw":
            out["f32"] = f32_variant(A, x, dev, timer, torch, ac, args.steps)
        if regions is None:
            log("extras: autotuned choice")
            out["tuned"] = tuned_record(ac, dev, dtype, xd, yd, timer, args.steps)
        if regions is not None:
            # the same matrix with one desiredChunkSize for every row
            out["uniform_desired"] = {}
            for Du in sorted({1, int(regions.max())}):
                Mu = ac.convert(dev, T, Du, dtype)
                f = lambda: ac.spmv(Mu, xd, yd)
                timer.run(f, 3)
                t, _ = timer.run(f, args.steps)
                out["uniform_desired"][f"D{Du}"] = stats(t) | {
                    "gbps": B / (t.mean() * 1e-3) / 1e9, "padding_ratio": Mu.n_slots / A.nnz}
                del Mu
            out["region_desired_histogram"] = {
                int(k): int(v) for k, v in zip(*np.unique(regions, return_counts=True))}
        # the second storage format (row-grouped CSR, one chunk per row) at the same T
        Mrg = ac.convert(dev, T, 0, dtype, fmt=ac.FORMAT_RG)
        f = lambda: ac.spmv(Mrg, xd, yd)
        timer.run(f, 3)
        t, _ = timer.run(f, args.steps)
        out["row_grouped"] = stats(t) | {"gbps": B / (t.mean() * 1e-3) / 1e9, "block_dim": T,
                                         "padding_ratio": Mrg.n_slots / max(A.nnz, 1)}
        del Mrg

    if "ceilings" in legs:
        log("ceilings")
        out["ceilings"] = leg_ceilings(torch, ac, M, dtype, timer, max(10, args.steps // 2))
    copy = timer.copy_ceiling()
    if copy:
        out.setdefault("ceilings", {})["copy"] = copy
        out["roofline"]["achievable_gbps"] = round(copy["gbps"], 1)
        out["roofline"]["frac_of_achievable"] = round(gbps / copy["gbps"], 4)

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(A, x, useful_bytes(A, 0))   # the oracle is FP64
        conv_ms, conv_reps = cpu_convert(A, T, D, region_rows, regions)
        out["cpu_baseline"]["convert_ms"] = conv_ms
        out["cpu_baseline"]["convert_sample"] = (f"whole matrix, T={T} D={D}, single thread, "
                                                 f"median of {conv_reps}")
    del M, dev, xd, yd
    torch.cuda.empty_cache()

    leg_steps = max(10, min(args.steps, 30))
    if "stencil27" in legs:
        log("leg: stencil27")
        out["stencil27"] = leg_stencil27(torch, ac, Timer(torch, cold=not args.warm), leg_steps)
    if "batch" in legs:
        log("leg: batch")
        out["batch"] = batch_record(torch, ac, args.batch_count, 1, leg_steps,
                                    max(2, args.warmup // 2), cold=not args.warm)
    if "serve" in legs:
        log("leg: serve")
        out["serve"] = serve_record(ac, args.pool, args.requests, args.warm_requests, args.rate,
                                    args.budget_gb, args.budget_frac, args.max_active,
                                    args.cg_inner_per_step)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
