"""ARG-CSR SpMV benchmark on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload powerlaw|stencil27|laplace64]
                    [--dtype f64|f32|bf16|f16] [--block-dim T] [--desired-chunk-size D]
                    [--warm] [--no-cpu-baseline] [--no-extras]

A step is one y = A x in ARG-CSR (argcsr_spmv) on a matrix converted once
beforehand (conversion time is reported separately).  Inputs are resident in
HBM when timing starts.  By default every step is preceded by a 1 GiB
read-modify-write "flush" (not timed) so that neither the L2s nor the 256 MB
Infinity Cache hold the matrix: the figure is HBM bandwidth, not cache
bandwidth.  Each SpMV launch is bracketed by HIP events on the stream it is
launched on; `value` is algorithmic bytes / mean launch time.

Algorithmic bytes per SpMV (the same for every format, so a GB/s ratio is a
speed-up):  nnz*(s_v + 4) + n_rows*(4 + s_y) + n_cols*s_x.

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
DTYPES = {"f64": 0, "f32": 1, "bf16": 2, "f16": 3}
VALUE_BYTES = {0: 8, 1: 4, 2: 2, 3: 2}
KERNEL_SOURCES = ["paper_1203_5737_amd/csrc/spmv_kernels.hpp", "paper_1203_5737_amd/csrc/spmv.hip",
                  "paper_1203_5737_amd/csrc/values.hpp", "paper_1203_5737_amd/csrc/common.hpp",
                  "paper_1203_5737_amd/csrc/schedule.hpp"]
# (block_dim, desired_chunk_size) per workload unless given on the command line
DEFAULT_PARAMS = {"powerlaw": (64, 1), "stencil27": (128, 27), "laplace64": (64, 1),
                  "mixed": (64, 1)}
DEFAULT_REGION_ROWS = {"mixed": 4096}


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


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
    evicting the caches (1 GiB read-modify-write) before each launch."""

    def __init__(self, torch, cold: bool):
        self.torch = torch
        self.cold = cold
        self.flush_buf = torch.empty(1 << 28, dtype=torch.float32, device="cuda") if cold else None

    def run(self, fn, steps: int):
        torch = self.torch
        starts = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        ends = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            if self.cold:
                self.flush_buf.add_(1.0)
            starts[i].record()
            fn()
            ends[i].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = np.array([s.elapsed_time(e) for s, e in zip(starts, ends)])
        return ms, wall


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


def cpu_baseline(A, x, B_useful, budget_s: float = 12.0):
    """The FP64 CSR oracle on this host's cores (OpenMP row split; identical
    result to the sequential oracle), on a bounded number of full SpMVs."""
    import oracle
    threads = os.cpu_count() or 1
    y = oracle.csr_spmv(A.rp, A.col, A.val, x, threads)       # warm-up
    t0 = time.perf_counter()
    oracle.csr_spmv(A.rp, A.col, A.val, x, threads)
    one = max(time.perf_counter() - t0, 1e-6)
    reps = int(max(3, min(100_000, (budget_s * 0.6) / one)))
    t0 = time.perf_counter()
    for _ in range(reps):
        oracle.csr_spmv(A.rp, A.col, A.val, x, threads)
    mt = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    st_reps = max(1, min(reps, int((budget_s * 0.4) / max(one * threads, 1e-6))))
    for _ in range(st_reps):
        oracle.csr_spmv(A.rp, A.col, A.val, x, 1)
    st = (time.perf_counter() - t0) / st_reps
    del y
    return {"value": B_useful / mt / 1e9, "unit": "GB/s", "cores": threads, "kind": "oracle",
            "sample": f"full matrix, {reps} SpMVs on {threads} threads (OpenMP row split) "
                      f"+ {st_reps} single-threaded",
            "ms_per_spmv": mt * 1e3, "single_thread_gbps": B_useful / st / 1e9,
            "single_thread_ms": st * 1e3, "cpu_model": cpu_model()}


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
    best = None
    for V in (8, 16, 32, 64):
        g = lambda V=V: ac.csr_spmv(dev, xd, yd, values=vals, dtype=1, lanes_per_row=V)
        timer.run(g, 3)
        c, _ = timer.run(g, max(10, steps // 5))
        if best is None or c.mean() < best[1].mean():
            best = (V, c)
    ac.spmv(M, xd, yd)
    err = error_vs_fp64(A, x, yd.cpu().numpy())
    return {"block_dim": 128, "desired_chunk_size": 1, "mean_ms": float(t.mean()),
            "gbps": B / (t.mean() * 1e-3) / 1e9, "csr_gbps": B / (best[1].mean() * 1e-3) / 1e9,
            "csr_lanes_per_row": best[0], "speedup_vs_csr": float(best[1].mean() / t.mean()),
            "error_vs_fp64": err}


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
    the current kernel source (None when absent or the kernel has changed)."""
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    if not os.path.exists(path):
        return None
    want = f"{workload}/{dtype_name}/T{T}/D{D}"
    for line in open(path):
        f = line.split()
        # key  kernel_hash  fetch_bytes  write_bytes  (scaled, per launch)
        if len(f) >= 4 and not line.startswith("#") and f[0] == want and f[1] == kernel_source_hash():
            return int(f[2]) + int(f[3])
    return None


def run_batch(args, torch, ac):
    """256 matrices (n log-uniform in [1e3, 2e5], half U{5..50} nonzeros per
    row, half clip(Zipf(2.2), 1, min(5000, n))), FP32 values, (T, D)
    autotuned per matrix; a step is ONE replay of the batch's hipGraph
    (queue reset + persistent kernel over all matrices' groups)."""
    import synth
    dtype = DTYPES[args.dtype]
    count = args.batch_count
    mats = synth.workload_batch(count)
    vdt = ac.vector_dtype(dtype)
    devs, Ms, xs, ys, tunes = [], [], [], [], []
    t0 = time.perf_counter()
    for A, x in mats:
        d = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, "cuda")
        r = ac.autotune(d, dtype, n_finalists=3)
        tunes.append((r["block_dim"], r["desired_chunk_size"], r["from_cache"], r["format"]))
        Ms.append(ac.convert(d, r["block_dim"], r["desired_chunk_size"], dtype, fmt=r["format"]))
        devs.append(d)
        xs.append(torch.from_numpy(x).to("cuda", vdt))
        ys.append(torch.empty(A.n_rows, dtype=vdt, device="cuda"))
    setup_s = time.perf_counter() - t0
    B = sum(useful_bytes(A, dtype) for A, _ in mats)
    nnz = sum(A.nnz for A, _ in mats)
    batch = ac.Batch(Ms, xs, ys)
    timer = Timer(torch, cold=not args.warm)
    run = lambda: batch.launch(graph=True)
    timer.run(run, args.warmup)
    ms, wall = timer.run(run, args.steps)
    mean_s = ms.mean() * 1e-3
    gbps = B / mean_s / 1e9
    out = {
        "metric": METRIC, "value": round(gbps, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": float(ms.mean()),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"batch of {count} matrices, n log-uniform [1e3,2e5], half U{{5..50}} "
                               "nnz/row, half clip(Zipf(2.2),1,min(5000,n)); one hipGraph replay "
                               "per step", "n_rows": sum(A.n_rows for A, _ in mats), "nnz": nnz,
                   "value_dtype": args.dtype,
                   "timing": "warm" if args.warm else "cold (1 GiB flush before each step, untimed)"},
        "roofline": {"bound": "hbm", "achieved": round(gbps, 2), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBPS, 4), "traffic": None},
        "spmv": stats(ms) | {"gflops": 2 * nnz / mean_s / 1e9, "useful_bytes": B,
                             "wall_ms_per_step": wall * 1e3 / args.steps} | batch.info(),
        "setup_s": setup_s,
        "tuned": {(f"T{T}/RG" if fm else f"T{T}/D{D}"): sum(1 for t in tunes
                                                          if (t[0], t[1], t[3]) == (T, D, fm))
                  for T, D, fm in sorted({(t[0], t[1], t[3]) for t in tunes})},
        "kernel_hash": kernel_source_hash(),
    }
    if not args.no_extras:
        loop = lambda: [ac.spmv(M, x, y) for M, x, y in zip(Ms, xs, ys)]
        timer.run(loop, 2)
        t, _ = timer.run(loop, max(5, args.steps // 4))
        out["single_launch_loop"] = stats(t) | {"gbps": B / (t.mean() * 1e-3) / 1e9}
        direct = lambda: batch.launch(graph=False)
        t, _ = timer.run(direct, max(5, args.steps // 4))
        out["batch_direct_launch"] = stats(t) | {"gbps": B / (t.mean() * 1e-3) / 1e9}
        vals = [d.val.to(ac.storage_dtype(dtype)) if dtype != 0 else d.val for d in devs]
        csr = lambda: [ac.csr_spmv(d, x, y, values=v, dtype=dtype) for d, x, y, v in zip(devs, xs, ys, vals)]
        timer.run(csr, 2)
        t, _ = timer.run(csr, max(5, args.steps // 4))
        out["csr_loop"] = stats(t) | {"gbps": B / (t.mean() * 1e-3) / 1e9}
        out["speedup_vs_csr_loop"] = out["csr_loop"]["mean_ms"] / float(ms.mean())
    batch.close()
    print(json.dumps(out))


def run_serve(args, torch, ac):
    """Open-loop serving: Poisson arrivals at --rate req/s of SpMV and CG
    requests (50/50) on a pool of SPD shifted 2D/3D Laplacians with n
    log-uniform in [1e4, 1e6]; request matrix ~ Zipf(1.1) over the pool.
    Latency runs from the scheduled arrival to the result in host memory."""
    import threading
    import synth
    from paper_1203_5737_amd import serve
    rng = np.random.default_rng(np.random.SeedSequence([12035737, 4, 999999]))
    P = args.pool
    pool = [synth.serve_pool_matrix(i)[0] for i in range(P)]
    zipf_w = 1.0 / np.arange(1, P + 1) ** 1.1
    zipf_w /= zipf_w.sum()
    n_req = args.requests + args.warm_requests
    mats = rng.choice(P, size=n_req, p=zipf_w)
    kinds = rng.random(n_req) < 0.5                      # True: CG
    gaps = rng.exponential(1.0 / args.rate, n_req)
    inputs = [rng.uniform(-1, 1, pool[m].n_rows) if cg else
              rng.uniform(-1, 1, pool[m].n_cols).astype(np.float32)
              for m, cg in zip(mats, kinds)]
    srv = serve.Server(budget_bytes=int(args.budget_gb * (1 << 30)), max_active=args.max_active,
                       cg_tol=1e-10, cg_inner_per_step=args.cg_inner_per_step)
    records = []
    t0 = time.monotonic_ns() + 50_000_000
    arrivals = t0 + np.cumsum(gaps * 1e9).astype(np.int64)
    for k in range(n_req):
        while time.monotonic_ns() < arrivals[k]:
            pass
        m = int(mats[k])
        A = pool[m]
        # ADMIT is a no-op for a resident matrix; it converts the matrix again
        # after an eviction.  Its result says whether it converted (cold).
        ta = srv.admit(m, A.rp, A.col, A.val, A.n_cols)
        if kinds[k]:
            t, _ = srv.cg(m, inputs[k])
        else:
            t, _ = srv.spmv(m, inputs[k], pool[m].n_rows)
        records.append((t, ta, int(arrivals[k]), bool(kinds[k]), m))
    results = []
    for t, ta, arr, cg, m in records:
        r = srv.wait(t, 600.0)
        cold = srv.wait(ta, 600.0)["iterations"] == 1
        srv.release(ta)
        results.append((r, arr, cold, cg, m))
    wall = (max(r["t_done_ns"] for r, *_ in results) - t0) * 1e-9
    stats = srv.stats()
    srv.close()
    meas = results[args.warm_requests:]
    ok = [x for x in meas if x[0]["status"] == 0]
    lat = lambda xs: np.array([(r["t_done_ns"] - arr) * 1e-6 for r, arr, *_ in xs])
    def pct(xs):
        a = lat(xs)
        return {"n": int(a.size), "p50_ms": float(np.percentile(a, 50)) if a.size else None,
                "p99_ms": float(np.percentile(a, 99)) if a.size else None}
    all_lat = lat(ok)
    sp_bytes = sum(useful_bytes(pool[m], 1) * (1 if not cg else max(1, r["iterations"]))
                   for r, _, _, cg, m in ok)
    out = {
        "metric": METRIC, "value": float(np.percentile(all_lat, 50)), "unit": "ms (p50 latency)",
        "n_gpus": 1, "steps": len(meas), "warmup": args.warm_requests,
        "ms_per_step": float(all_lat.mean()), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 SpMV / f64 CG", "data": "synthetic",
        "config": {"workload": f"serving: Poisson {args.rate:g} req/s, 50% SpMV / 50% CG to 1e-10, "
                               f"pool of {P} SPD shifted 2D/3D Laplacians, n log-uniform [1e4,1e6], "
                               f"Zipf(1.1) popularity, {args.budget_gb:g} GB budget",
                   "max_active": args.max_active,
                   "cg_inner_per_step": args.cg_inner_per_step or 2},
        "latency": {"all": pct(ok), "p99_ms": float(np.percentile(all_lat, 99)),
                    "warm": pct([x for x in ok if not x[2]]), "cold": pct([x for x in ok if x[2]]),
                    "spmv": pct([x for x in ok if not x[3]]), "cg": pct([x for x in ok if x[3]])},
        "throughput_req_s": len(results) / wall,
        "aggregate_spmv_gbps_lower_bound": sp_bytes / wall / 1e9,
        "failed": len(meas) - len(ok),
        "cg_max_relres": max((r["relres"] for r, _, _, cg, _ in ok if cg), default=None),
        "cg_mean_iterations": float(np.mean([r["iterations"] for r, _, _, cg, _ in ok if cg] or [0])),
        "server": stats,
    }
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
    ap.add_argument("--warm", action="store_true", help="no cache flush between steps")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the CSR and warm timings")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--rate", type=float, default=1000.0, help="serve: arrivals per second")
    ap.add_argument("--requests", type=int, default=2000, help="serve: measured requests")
    ap.add_argument("--warm-requests", type=int, default=200, help="serve: unmeasured first requests")
    ap.add_argument("--pool", type=int, default=64, help="serve: distinct matrices")
    ap.add_argument("--cg-inner-per-step", type=int, default=0,
                    help="serve: inner CG iterations a step may run (0 = the server's default)")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serve: device memory budget")
    ap.add_argument("--max-active", type=int, default=64, help="serve: requests per step")
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
    dtype = DTYPES[args.dtype]
    T0, D0 = DEFAULT_PARAMS.get(args.workload, (64, 1))
    T = args.block_dim or T0
    D = args.desired_chunk_size or D0

    A, x, desc = load_workload(args.workload)
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, "cuda")
    torch.cuda.synchronize()
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

    timer = Timer(torch, cold=not args.warm)
    spmv = lambda: ac.spmv(M, xd, yd)
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
                     "traffic": traffic_for(args.workload, args.dtype, T, D)},
        "spmv": stats(ms) | {"gflops": 2 * A.nnz / mean_s / 1e9, "useful_bytes": B,
                             "format_bytes": Bf, "padding_ratio": M.n_slots / max(A.nnz, 1),
                             "n_groups": M.n_groups, "wall_ms_per_step": wall * 1e3 / args.steps},
        "convert_ms": convert_ms,
        "convert_device_grouping_ms": convert_device_ms,
        "kernel_hash": kernel_source_hash(),
        "error_vs_fp64": error_vs_fp64(A, x, yd.cpu().numpy()),
    }

    if not args.no_extras:
        # the same SpMV without flushes (matrix may stay in the Infinity Cache)
        warm_ms, _ = Timer(torch, cold=False).run(spmv, args.steps)
        out["spmv_warm"] = stats(warm_ms) | {"gbps": B / (warm_ms.mean() * 1e-3) / 1e9}
        # plain CSR on the same GPU, same timing; best lanes-per-row of a sweep
        vals = dev.val if dtype == 0 else dev.val.to(ac.storage_dtype(dtype))
        best = None
        for V in (0, 1, 2, 4, 8, 16, 32, 64):
            f = lambda V=V: ac.csr_spmv(dev, xd, yd, values=vals, dtype=dtype, lanes_per_row=V)
            timer.run(f, 3)
            t, _ = timer.run(f, max(10, args.steps // 5))
            if best is None or t.mean() < best[1].mean():
                best = (V, t)
        V, t = best
        f = lambda: ac.csr_spmv(dev, xd, yd, values=vals, dtype=dtype, lanes_per_row=V)
        t, _ = timer.run(f, args.steps)
        csr_gbps = B / (t.mean() * 1e-3) / 1e9
        out["csr"] = stats(t) | {"gbps": csr_gbps, "lanes_per_row": V}
        out["speedup_vs_csr"] = gbps / csr_gbps
        if dtype == 0 and args.workload == "powerlaw":
            out["f32"] = f32_variant(A, x, dev, timer, torch, ac, args.steps)
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

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(A, x, useful_bytes(A, 0))   # the oracle is FP64
        conv_ms, conv_reps = cpu_convert(A, T, D, region_rows, regions)
        out["cpu_baseline"]["convert_ms"] = conv_ms
        out["cpu_baseline"]["convert_sample"] = (f"whole matrix, T={T} D={D}, single thread, "
                                                 f"median of {conv_reps}")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
