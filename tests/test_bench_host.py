"""CPU: the host logic of bench.py -- the one-GPU refusal, the byte count its
GB/s figures divide by, the error it states against FP64, and the lookup of
measured traffic by kernel source hash."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import synth  # noqa: E402


def test_more_than_one_gpu_is_refused():
    proc = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                          capture_output=True, text=True, timeout=120)
    assert proc.returncode != 0
    line = json.loads(proc.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_useful_bytes_formula():
    A = synth.Csr(3, 5, np.array([0, 2, 2, 5], np.int32), np.array([0, 4, 1, 2, 3], np.int32),
                  np.ones(5))
    # nnz*(s_v + 4) + n_rows*(4 + s_y) + n_cols*s_x
    assert bench.useful_bytes(A, 0) == 5 * 12 + 3 * 12 + 5 * 8
    assert bench.useful_bytes(A, 1) == 5 * 8 + 3 * 8 + 5 * 4
    assert bench.useful_bytes(A, 2) == bench.useful_bytes(A, 3) == 5 * 6 + 3 * 8 + 5 * 4


def test_error_vs_fp64():
    rng = np.random.default_rng(4)
    L = rng.integers(0, 5, 200)
    L[:3] = 0                                            # empty rows
    A = synth.random_csr(L, 300, rng, rng)
    x = rng.uniform(-1, 1, A.n_cols)
    y = np.array([sum(A.val[k] * x[A.col[k]] for k in range(A.rp[i], A.rp[i + 1]))
                  for i in range(A.n_rows)])
    e = bench.error_vs_fp64(A, x, y)
    assert e["zero_rows_exact"] and e["max_scaled"] <= 4e-16 and e["rel_l2"] <= 4e-16
    # one row off by a known amount: its scaled error is that amount / sum |a x|
    i = int(np.argmax(np.diff(A.rp)))
    scale = sum(abs(A.val[k] * x[A.col[k]]) for k in range(A.rp[i], A.rp[i + 1]))
    y2 = y.copy()
    y2[i] += 1e-3 * scale
    assert abs(bench.error_vs_fp64(A, x, y2)["max_scaled"] - 1e-3) < 1e-9
    y3 = y.copy()
    y3[0] = 1e-30                                        # an empty row must be exactly 0
    assert not bench.error_vs_fp64(A, x, y3)["zero_rows_exact"]


def test_traffic_is_used_only_for_the_current_kernel():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    kinds = {k: bench.kernel_source_hash(k) for k in bench.SOURCE_SETS}
    assert len(set(kinds.values()) | {h}) == len(kinds) + 1
    assert set(bench.KERNEL_SOURCES) == {f for v in bench.SOURCE_SETS.values() for f in v}
    path = os.path.join(ROOT, "profiles", "traffic.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    for key, kh, fetch, write in rows:
        wl, dt, T, D = key.split("/")
        num = lambda v: int(v) if v.isdigit() else v          # "auto": the tuner's choice
        got = bench.traffic_for(wl, dt, num(T[1:]), num(D[1:]))
        current = kinds[bench.traffic_kind(wl)]
        assert got == (int(fetch) + int(write) if kh == current else None)
    assert bench.traffic_for("powerlaw", "f64", 999, 1) is None
