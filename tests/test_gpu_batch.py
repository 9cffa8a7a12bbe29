"""GPU: many matrices in one persistent launch, its hipGraph, and the autotuner.

Every group of a batch is computed by the same routine as argcsr_spmv, so
each y_m must equal the single-matrix result bit for bit, and the oracle
within the usual tolerance."""
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


def small_batch(count, seed, n_hi=30_000):
    mats = [synth.batch_member(k, 1e3, n_hi) for k in range(count)]
    rng = np.random.default_rng(seed)
    # one member with very long rows so the batch has heavy items
    L = rng.integers(1, 6, 8000)
    L[rng.integers(0, 8000, 6)] = 6000
    A = synth.random_csr(L, 8000, rng, rng)
    mats.append((A, rng.uniform(-1, 1, 8000)))
    return mats


def convert_all(ac, mats, dtype, seed):
    rng = np.random.default_rng(seed)
    out = []
    for A, x in mats:
        T = int(rng.choice([64, 128, 256]))
        D = int(rng.choice([1, 2, 4, 0]))           # 0: row-grouped CSR
        dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
        M = ac.convert(dev, T, D, dtype, fmt=ac.FORMAT_ARG if D else ac.FORMAT_RG)
        xd = torch.from_numpy(x).to(DEV, ac.vector_dtype(dtype))
        out.append((A, x, M, xd))
    return out


@pytest.mark.parametrize("dtype", [0, 1])
def test_batch_equals_single_launches(ac, dtype):
    print(f"\n[gpu] batch dtype={dtype}", flush=True)
    mats = convert_all(ac, small_batch(24, 1), dtype, 2)
    vdt = ac.vector_dtype(dtype)
    singles = [ac.spmv(M, xd) for (_, _, M, xd) in mats]
    ys = [torch.full((M.n_rows,), float("nan"), dtype=vdt, device=DEV) for (_, _, M, _) in mats]
    b = ac.Batch([m[2] for m in mats], [m[3] for m in mats], ys)
    info = b.info()
    assert info["n_heavy"] > 0 and info["n_items"] > 0 and info["grid"] > 0
    for graph in (False, True):
        for y in ys:
            y.fill_(float("nan"))
        b.launch(graph=graph)
        torch.cuda.synchronize()
        for y, y1 in zip(ys, singles):
            assert torch.equal(y.view(torch.int64 if dtype == 0 else torch.int32),
                               y1.view(torch.int64 if dtype == 0 else torch.int32))
    for (A, x, M, _), y in zip(mats, ys):
        yh = y.cpu().numpy().astype(np.float64)
        if dtype == 0:
            check_f64(A, x, yh)
        else:
            check_reduced(A, x, yh, oracle.F32)
    b.close()


def test_batch_graph_replays_track_inputs(ac):
    """Replay the graph several times with eager work in between; each
    replay must reproduce the eager result for the current x."""
    print("\n[gpu] graph replays", flush=True)
    mats = convert_all(ac, small_batch(8, 3), 1, 4)
    ys = [torch.empty(M.n_rows, dtype=torch.float32, device=DEV) for (_, _, M, _) in mats]
    b = ac.Batch([m[2] for m in mats], [m[3] for m in mats], ys)
    junk = torch.randn(512, 512, device=DEV)
    for rep in range(5):
        for (_, _, _, xd) in mats:
            xd.mul_(-0.5 if rep % 2 else 1.25)       # new x in place
        junk = junk @ junk.T / 512.0                 # unrelated eager work
        eager = [ac.spmv(M, xd) for (_, _, M, xd) in mats]
        b.launch(graph=True)
        torch.cuda.synchronize()
        for y, ye in zip(ys, eager):
            assert torch.equal(y, ye), rep
    b.close()


def test_batch_rejects_mixed_dtypes(ac):
    mats = small_batch(2, 5)
    a = convert_all(ac, mats[:1], 0, 6)[0]
    c = convert_all(ac, mats[1:2], 1, 7)[0]
    with pytest.raises(ac.ArgCsrError) as e:
        ac.Batch([a[2], c[2]], [a[3], c[3]],
                 [torch.empty(a[2].n_rows, dtype=torch.float64, device=DEV),
                  torch.empty(c[2].n_rows, dtype=torch.float32, device=DEV)])
    assert e.value.code == ac._lib.EINVAL


def test_autotune_times_finalists(ac):
    print("\n[gpu] autotune", flush=True)
    ac.autotune_clear_cache()
    A, x = powerlaw_sample(200_000, seed=8)
    dev = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
    r = ac.autotune(dev, ac.F64, n_finalists=3)
    assert r["n_timed"] == 3 and r["measured_us"] > 0 and r["from_cache"] == 0
    assert r["block_dim"] in (64, 128, 256) and 24 <= r["n_candidates"] <= 30
    assert r["format"] in (ac.FORMAT_ARG, ac.FORMAT_RG)
    assert r["desired_chunk_size"] >= 1 or r["format"] == ac.FORMAT_RG
    r2 = ac.autotune(dev, ac.F64, n_finalists=3)
    assert r2["from_cache"] == 1 and r2["block_dim"] == r["block_dim"]
    M = ac.convert(dev, r["block_dim"], r["desired_chunk_size"], fmt=r["format"])
    y = ac.spmv(M, torch.from_numpy(x).to(DEV)).cpu().numpy()
    check_f64(A, x, y)


def test_full_batch_of_256_as_benchmarked(ac):
    """The 256-matrix batch the benchmark times (FP32, (T, D, format) chosen
    per matrix by the batch-member model, one hipGraph replay):
    every member within the FP32 bound of the oracle and bitwise equal to its
    own single launch."""
    print("\n[gpu] full batch of 256", flush=True)
    mats = synth.workload_batch(256)
    conv = []
    for A, x in mats:
        d = ac.to_device_csr(A.rp, A.col, A.val, A.n_cols, DEV)
        r = ac.autotune_member(A.rp, ac.F32)
        M = ac.convert(d, r["block_dim"], r["desired_chunk_size"], ac.F32, fmt=r["format"])
        conv.append((M, torch.from_numpy(x).to(DEV, torch.float32)))
        del d
    ys = [torch.full((M.n_rows,), float("nan"), dtype=torch.float32, device=DEV) for M, _ in conv]
    b = ac.Batch([M for M, _ in conv], [xd for _, xd in conv], ys)
    b.launch(graph=True)
    torch.cuda.synchronize()
    print(f"[gpu] batch info {b.info()}", flush=True)
    for (A, x), (M, xd), y in zip(mats, conv, ys):
        single = ac.spmv(M, xd)
        assert torch.equal(y.view(torch.int32), single.view(torch.int32))
        check_reduced(A, x, y.cpu().numpy().astype(np.float64), oracle.F32)
    b.close()
