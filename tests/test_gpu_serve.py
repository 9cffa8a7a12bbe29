"""GPU: the request server -- resident matrices under a budget, continuous
batching of SpMV and CG requests, mixed-precision CG to a 1e-10 true
relative residual, and results that are bitwise the same alone and in a mix.

CG is pinned the only way its result is fixed: any x whose true residual
|b - A x| / |b|, recomputed here with the FP64 oracle, is at most 1e-10."""
import numpy as np
import pytest

import oracle
import synth
from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def srv_mod():
    from paper_1203_5737_amd import _lib, serve
    _lib.lib()
    return serve


def pool(count, n_lo=2e3, n_hi=3e4):
    return [synth.serve_pool_matrix(i, n_lo, n_hi)[0] for i in range(count)]


def true_relres(A, x, b):
    r = b - oracle.csr_spmv(A.rp, A.col, A.val, x)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def spmv_ok(A, x32, y):
    stored = oracle.stored_as_f64(oracle.round_array(A.val, oracle.F32), oracle.F32)
    xx = x32.astype(np.float64)
    ref = oracle.csr_spmv(A.rp, A.col, stored, xx)
    L = np.diff(A.rp)
    scale = np.bincount(np.repeat(np.arange(A.n_rows), L), weights=np.abs(stored * xx[A.col]),
                        minlength=A.n_rows)
    u = 2.0 ** -24
    return bool(np.all(np.abs(y.astype(np.float64) - ref) <= (L + 1) * u / (1 - (L + 1) * u) * scale))


def run_requests(srv, mats, reqs):
    """reqs: list of (kind, matrix index, input); returns outputs and results."""
    tickets = []
    for kind, m, inp in reqs:
        if kind == "spmv":
            tickets.append(srv.spmv(m, inp, mats[m].n_rows))
        else:
            tickets.append(srv.cg(m, inp))
    outs, res = [], []
    for t, out in tickets:
        r = srv.wait(t, 120.0)
        assert r["status"] == 0, r
        outs.append(out.copy())
        res.append(r)
        srv.release(t)
    return outs, res


def make_requests(mats, count, seed):
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(count):
        m = int(rng.integers(0, len(mats)))
        if k % 2 == 0:
            reqs.append(("spmv", m, rng.uniform(-1, 1, mats[m].n_cols).astype(np.float32)))
        else:
            reqs.append(("cg", m, rng.uniform(-1, 1, mats[m].n_rows)))
    return reqs


def admit_all(srv, mats):
    for i, A in enumerate(mats):
        t = srv.admit(i, A.rp, A.col, A.val, A.n_cols)
        assert srv.wait(t, 120.0)["status"] == 0
        srv.release(t)


def test_serve_results_and_alone_vs_mix(srv_mod):
    print("\n[gpu] serve mix", flush=True)
    mats = pool(6)
    reqs = make_requests(mats, 24, 1)
    with srv_mod.Server(budget_bytes=1 << 30, max_active=32) as srv:
        admit_all(srv, mats)
        mix_out, mix_res = run_requests(srv, mats, reqs)          # all in flight together
        st = srv.stats()
        assert st["completed"] == 24 and st["steps"] > 0
    for (kind, m, inp), out, r in zip(reqs, mix_out, mix_res):
        if kind == "spmv":
            assert spmv_ok(mats[m], inp, out)
        else:
            assert r["relres"] <= 1e-10 and r["refinements"] >= 1 and r["iterations"] > 0
            assert true_relres(mats[m], out, inp) <= 1e-10
    print("[gpu] serve alone", flush=True)
    # one request at a time, and without pinned staging: inputs and results
    # go straight between the caller's memory and the device
    with srv_mod.Server(budget_bytes=1 << 30, max_active=1, staging_bytes=-1) as srv:
        admit_all(srv, mats)
        alone_out, alone_res = run_requests(srv, mats, reqs)
    for a, b, ra, rb in zip(mix_out, alone_out, mix_res, alone_res):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
        assert ra["iterations"] == rb["iterations"]


def test_serve_inner_iterations_per_step(srv_mod):
    """A step may run several inner CG iterations of a request; the cycle's
    stopping tests then run on the device after each one, and later
    iterations of a stopped request are skipped.  Results, iteration and
    refinement counts and residuals are bitwise those of one iteration per
    step, for 2, 3 and 8 per step, with cycles ended by the residual test
    (cg_max_inner 200) and by the count limit inside a step (cg_max_inner 13);
    and a solve cut off by cg_max_iter (ENOCONV) stops at the same iterate."""
    from paper_1203_5737_amd import _lib
    print("\n[gpu] serve inner iterations per step", flush=True)
    mats = pool(4)
    reqs = make_requests(mats, 12, 5)
    for max_inner in (200, 13):
        base = None
        for per_step in (1, 2, 3, 8):
            with srv_mod.Server(budget_bytes=1 << 30, max_active=16, cg_max_inner=max_inner,
                                cg_inner_per_step=per_step) as srv:
                admit_all(srv, mats)
                out, res = run_requests(srv, mats, reqs)
            got = ([o.view(np.uint8).copy() for o in out],
                   [(r["iterations"], r["refinements"], r["relres"]) for r in res])
            if base is None:
                base = got
                for (kind, m, inp), o in zip(reqs, out):
                    if kind == "cg":
                        assert true_relres(mats[m], o, inp) <= 1e-10, (max_inner, m)
                continue
            for a, b in zip(base[0], got[0]):
                assert np.array_equal(a, b), (max_inner, per_step)
            assert base[1] == got[1], (max_inner, per_step)
    cg_reqs = [(m, inp) for kind, m, inp in reqs if kind == "cg"]
    outs = []
    for per_step in (1, 3):
        with srv_mod.Server(budget_bytes=1 << 30, max_active=8, cg_max_iter=7,
                            cg_inner_per_step=per_step) as srv:
            admit_all(srv, mats)
            got = []
            for m, b in cg_reqs:
                t, x = srv.cg(m, b)
                r = srv.wait(t, 120.0)
                srv.release(t)
                assert r["status"] == _lib.ENOCONV and r["iterations"] == 7, r
                got.append((x.view(np.uint8).copy(), r["relres"]))
        outs.append(got)
    for (xa, ra), (xb, rb) in zip(*outs):
        assert np.array_equal(xa, xb) and ra == rb


@pytest.mark.parametrize("T", [128, 256])
def test_serve_block_sizes(srv_mod, T):
    """Servers converting with T = 128 and 256 (the multi-matrix SpMV has one
    instance per block size): SpMV on Laplacians and on a matrix with rows of
    up to 6000 entries (whole-workgroup heavy groups), within the FP32 bound,
    bitwise equal alone and in the mix; CG to 1e-10."""
    print(f"\n[gpu] serve T={T}", flush=True)
    mats = pool(3)
    rng = np.random.default_rng(11)
    L = np.clip(rng.zipf(1.8, 20_000), 1, 6000)
    mats.append(synth.random_csr(L, 20_000, np.random.default_rng(12), np.random.default_rng(13)))
    reqs = [("spmv", m, rng.uniform(-1, 1, mats[m].n_cols).astype(np.float32)) for m in (3, 0, 3, 1)]
    reqs += [("cg", m, rng.uniform(-1, 1, mats[m].n_rows)) for m in (0, 1, 2)]
    outs = []
    for max_active in (16, 1):
        with srv_mod.Server(budget_bytes=1 << 30, max_active=max_active, block_dim=T) as srv:
            admit_all(srv, mats)
            out, res = run_requests(srv, mats, reqs)
        outs.append(out)
        for (kind, m, inp), o, r in zip(reqs, out, res):
            if kind == "spmv":
                assert spmv_ok(mats[m], inp, o), (T, m)
            else:
                assert true_relres(mats[m], o, inp) <= 1e-10, (T, m)
    for a, b in zip(*outs):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


def test_serve_clients_on_several_threads(srv_mod):
    """Four client threads submit and wait at the same time (ctypes releases
    the GIL, so the calls overlap in the library); every result equals the
    one the same request gets when submitted alone."""
    import threading
    print("\n[gpu] serve threads", flush=True)
    mats = pool(4)
    per_thread = [make_requests(mats, 8, 100 + t) for t in range(4)]
    outs = [None] * 4
    errors = []
    with srv_mod.Server(budget_bytes=1 << 30, max_active=16) as srv:
        admit_all(srv, mats)

        def client(t):
            try:
                outs[t] = run_requests(srv, mats, per_thread[t])[0]
            except Exception as e:                  # noqa: BLE001 - reported below
                errors.append(repr(e))
        threads = [threading.Thread(target=client, args=(t,)) for t in range(4)]
        for th in threads:
            th.start()
        for th in threads:
            th.join(300)
        assert not errors, errors
        assert srv.stats()["completed"] == 32
    with srv_mod.Server(budget_bytes=1 << 30, max_active=1) as srv:
        admit_all(srv, mats)
        for t in range(4):
            alone = run_requests(srv, mats, per_thread[t])[0]
            for a, b in zip(outs[t], alone):
                assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


def test_serve_small_staging_falls_back(srv_mod):
    """A staging arena too small for most requests: those bypass it, the
    others go through it; results are the same as with ample staging."""
    print("\n[gpu] serve small staging", flush=True)
    mats = pool(4)
    reqs = make_requests(mats, 16, 7)
    outs = []
    for staging in (0, 64 << 10):
        with srv_mod.Server(budget_bytes=1 << 30, max_active=8, staging_bytes=staging) as srv:
            admit_all(srv, mats)
            outs.append(run_requests(srv, mats, reqs)[0])
    for a, b in zip(*outs):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


def test_serve_requests_join_while_others_run(srv_mod):
    print("\n[gpu] serve continuous", flush=True)
    mats = pool(3, 5e4, 8e4)
    rng = np.random.default_rng(2)
    with srv_mod.Server(budget_bytes=1 << 30, max_active=8) as srv:
        admit_all(srv, mats)
        first = [srv.cg(m, rng.uniform(-1, 1, mats[m].n_rows)) for m in range(3)]
        late = [srv.spmv(m, rng.uniform(-1, 1, mats[m].n_cols), mats[m].n_rows) for m in range(3)]
        r_late = [srv.wait(t, 120.0) for t, _ in late]
        r_first = [srv.wait(t, 120.0) for t, _ in first]
        assert all(r["status"] == 0 for r in r_late + r_first)
        # the SpMVs entered while the solves were still iterating and left first
        assert max(r["t_done_ns"] for r in r_late) < max(r["t_done_ns"] for r in r_first)
        assert min(r["t_start_ns"] for r in r_late) < min(r["t_done_ns"] for r in r_first)


def test_serve_shutdown_with_admissions_in_preparation(srv_mod):
    """Destroying the server right after submitting ADMITs of large matrices,
    whose host side the preparation thread is still doing (queued ones are
    abandoned, a running one is waited for, pinned staging is freed), ends
    cleanly, twice; a new server then admits and serves correctly."""
    print("\n[gpu] serve shutdown during preparation", flush=True)
    mats = pool(6, 2e5, 4e5)
    for _ in range(2):
        srv = srv_mod.Server(budget_bytes=1 << 30, max_active=4)
        for i, A in enumerate(mats):
            srv.admit(i, A.rp, A.col, A.val, A.n_cols)
        srv.spmv(0, np.ones(mats[0].n_cols, np.float32), mats[0].n_rows)
        srv.close()
    rng = np.random.default_rng(8)
    with srv_mod.Server(budget_bytes=1 << 30, max_active=4) as srv:
        admit_all(srv, mats[:2])
        x = rng.uniform(-1, 1, mats[1].n_cols).astype(np.float32)
        t, y = srv.spmv(1, x, mats[1].n_rows)
        assert srv.wait(t, 120.0)["status"] == 0
        assert spmv_ok(mats[1], x, y)


def test_serve_budget_eviction_and_errors(srv_mod):
    print("\n[gpu] serve budget", flush=True)
    from paper_1203_5737_amd import _lib
    mats = pool(4, 2e4, 2.5e4)
    big = synth.shifted_laplacian("2d", 600_000, np.random.default_rng(3))
    with srv_mod.Server(budget_bytes=6 << 20, max_active=4) as srv:    # ~2 matrices fit
        admit_all(srv, mats)                      # later admissions evict earlier ones
        st = srv.stats()
        assert st["evictions"] >= 1 and st["resident_bytes"] <= 6 << 20
        t = srv.admit(99, big.rp, big.col, big.val, big.n_cols)
        assert srv.wait(t)["status"] == _lib.EBUDGET
        t, _ = srv.cg(0, np.ones(mats[0].n_rows))   # matrix 0 was evicted
        assert srv.wait(t)["status"] == _lib.ENOTFOUND
        t = srv.admit(0, mats[0].rp, mats[0].col, mats[0].val, mats[0].n_cols)
        assert srv.wait(t)["status"] == 0
        t, x = srv.cg(0, np.ones(mats[0].n_rows))
        r = srv.wait(t)
        assert r["status"] == 0 and true_relres(mats[0], x, np.ones(mats[0].n_rows)) <= 1e-10
        rect = synth.random_csr(np.full(50, 3), 80, np.random.default_rng(4), np.random.default_rng(5))
        t = srv.admit(7, rect.rp, rect.col, rect.val, 80)
        assert srv.wait(t)["status"] == 0
        t, _ = srv.cg(7, np.ones(50))             # CG needs a square matrix
        assert srv.wait(t)["status"] == _lib.EINVAL
        t = srv.evict(7)
        assert srv.wait(t)["status"] == 0
        t = srv.evict(7)
        assert srv.wait(t)["status"] == _lib.ENOTFOUND
        with pytest.raises(_lib.ArgCsrError):
            srv.poll(123456789)
    with pytest.raises(_lib.ArgCsrError):
        srv_mod.Server(budget_bytes=1 << 20, max_active=0)


def test_serve_admissions_wait_under_memory_pressure(srv_mod):
    """A budget of 6 MiB, about half of the 11.6 MB the eight matrices take
    when all are resident (the largest needs 3.6 MB while it is converted),
    and every matrix is used: every request is preceded by its ADMIT (a no-op
    when resident), admissions must evict matrices that no running request
    uses and wait while running requests hold the memory, and every request
    completes, oracle-checked."""
    print("\n[gpu] serve memory pressure", flush=True)
    budget = 6 << 20
    mats = pool(8, 1e4, 3e4)
    reqs = make_requests(mats, 40, 21)
    assert len({m for _, m, _ in reqs}) == len(mats)
    with srv_mod.Server(budget_bytes=budget, max_active=4) as srv:
        tickets = []
        for kind, m, inp in reqs:
            A = mats[m]
            ta = srv.admit(m, A.rp, A.col, A.val, A.n_cols)
            if kind == "spmv":
                t, out = srv.spmv(m, inp, A.n_rows)
            else:
                t, out = srv.cg(m, inp)
            tickets.append((ta, t, out))
        for (kind, m, inp), (ta, t, out) in zip(reqs, tickets):
            ra, r = srv.wait(ta, 120.0), srv.wait(t, 120.0)
            assert ra["status"] == 0 and r["status"] == 0, (ra, r)
            if kind == "spmv":
                assert spmv_ok(mats[m], inp, out)
            else:
                assert true_relres(mats[m], out, inp) <= 1e-10
        st = srv.stats()
        assert st["failed"] == 0 and st["completed"] == len(reqs)
        assert st["evictions"] > 0 and st["resident_bytes"] <= budget


def test_serve_results_while_conversions_run(srv_mod):
    """Regression: a finished request's vectors return to the arena while the
    copy of its result is still queued on the scheduler's stream; a
    conversion on the converter's stream may get those blocks, so it must be
    ordered after that stream.  Many short SpMV requests finishing while
    admissions convert under a budget that forces reuse: every result is
    checked."""
    print("\n[gpu] serve results while conversions run", flush=True)
    mats = pool(12, 1e4, 4e4)
    rng = np.random.default_rng(77)
    reqs = []
    for k in range(160):
        m = int(rng.integers(0, len(mats)))
        reqs.append((m, rng.uniform(-1, 1, mats[m].n_cols).astype(np.float32)))
    with srv_mod.Server(budget_bytes=8 << 20, max_active=8) as srv:
        tickets = []
        for m, x in reqs:
            A = mats[m]
            ta = srv.admit(m, A.rp, A.col, A.val, A.n_cols)
            tickets.append((ta,) + srv.spmv(m, x, A.n_rows))
        for k, ((m, x), (ta, t, y)) in enumerate(zip(reqs, tickets)):
            ra, r = srv.wait(ta, 120.0), srv.wait(t, 120.0)
            assert ra["status"] == 0 and r["status"] == 0, (k, m, ra, r, srv.stats())
            assert spmv_ok(mats[m], x, y)
        assert srv.stats()["evictions"] > 0


def test_serve_rejects_wrong_vector_lengths(srv_mod):
    """SPMV and CG requests state the lengths of their buffers; a request
    whose lengths are not the resident matrix's fails with EINVAL."""
    import ctypes
    from paper_1203_5737_amd import _lib
    mats = pool(1)
    A = mats[0]
    with srv_mod.Server(budget_bytes=1 << 28, max_active=2) as srv:
        admit_all(srv, mats)
        t, _ = srv.spmv(0, np.zeros(A.n_cols + 1, np.float32), A.n_rows)
        assert srv.wait(t)["status"] == _lib.EINVAL
        t, _ = srv.spmv(0, np.zeros(A.n_cols, np.float32), A.n_rows - 1)
        assert srv.wait(t)["status"] == _lib.EINVAL
        t, _ = srv.cg(0, np.ones(A.n_rows - 3))
        assert srv.wait(t)["status"] == _lib.EINVAL
        # a request without lengths (as before they were required) is refused too
        x = np.zeros(A.n_cols, np.float32)
        y = np.zeros(A.n_rows, np.float32)
        req = _lib.Request(_lib.REQ_SPMV, 0, 0, 0, None, None, None,
                           x.ctypes.data_as(ctypes.c_void_p), y.ctypes.data_as(ctypes.c_void_p))
        tk = ctypes.c_uint64(0)
        _lib.check(_lib.lib().argcsr_server_submit(srv._h, ctypes.byref(req), ctypes.byref(tk)),
                   "submit")
        assert srv.wait(tk.value)["status"] == _lib.EINVAL
        t, y = srv.spmv(0, np.ones(A.n_cols, np.float32), A.n_rows)
        assert srv.wait(t)["status"] == 0 and spmv_ok(A, np.ones(A.n_cols, np.float32), y)


def test_serve_large_matrices_alone_and_in_mix(srv_mod):
    """Matrices above 524 288 rows (the CG kernels' per-request tile sums
    then take more than one pass of 256 tiles), as in the serving benchmark:
    SpMV within the FP32 bound, CG to a true 1e-10 residual with the FP64
    oracle, and each result bitwise the same alone and in the mix."""
    print("\n[gpu] serve large matrices", flush=True)
    rng = np.random.default_rng(31)
    mats = [synth.shifted_laplacian("2d", 700_000, np.random.default_rng(32)),
            synth.shifted_laplacian("3d", 614_125, np.random.default_rng(33)),
            synth.serve_pool_matrix(5, 1e4, 3e4)[0]]
    assert mats[0].n_rows > 524_288 and mats[1].n_rows > 524_288
    reqs = []
    for m in (0, 1, 2, 0, 1):
        reqs.append(("spmv", m, rng.uniform(-1, 1, mats[m].n_cols).astype(np.float32)))
        reqs.append(("cg", m, rng.uniform(-1, 1, mats[m].n_rows)))
    outs = []
    for max_active in (16, 1):
        with srv_mod.Server(budget_bytes=2 << 30, max_active=max_active) as srv:
            admit_all(srv, mats)
            out, res = run_requests(srv, mats, reqs)
        outs.append(out)
        for (kind, m, inp), o, r in zip(reqs, out, res):
            if kind == "spmv":
                assert spmv_ok(mats[m], inp, o), m
            else:
                assert r["relres"] <= 1e-10 and true_relres(mats[m], o, inp) <= 1e-10, m
    for a, b in zip(*outs):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


def test_serve_requests_pass_an_admission_in_progress(srv_mod):
    """Requests are taken in order per matrix: while a large ADMIT prepares
    and converts, ADMIT+SPMV pairs of a resident matrix submitted behind it
    start and finish, and the large matrix's own SPMV, submitted right after
    its ADMIT, still sees the ADMIT complete first.  Every result is checked."""
    print("\n[gpu] serve: requests pass an admission in progress", flush=True)
    small = pool(1, 2e4, 2.1e4)[0]
    big = synth.shifted_laplacian("3d", 1_000_000, np.random.default_rng(5))
    rng = np.random.default_rng(8)
    with srv_mod.Server(budget_bytes=1 << 30, max_active=16) as srv:
        admit_all(srv, [small])
        tb = srv.admit(1, big.rp, big.col, big.val, big.n_cols)
        xb = rng.uniform(-1, 1, big.n_cols).astype(np.float32)
        t_big, y_big = srv.spmv(1, xb, big.n_rows)
        pairs = []
        for _ in range(8):
            x = rng.uniform(-1, 1, small.n_cols).astype(np.float32)
            ta = srv.admit(0, small.rp, small.col, small.val, small.n_cols)
            pairs.append((ta, x) + srv.spmv(0, x, small.n_rows))
        rb, r_big = srv.wait(tb, 120.0), srv.wait(t_big, 120.0)
        assert rb["status"] == 0 and rb["iterations"] == 1      # converted here
        assert r_big["status"] == 0 and r_big["t_start_ns"] >= rb["t_done_ns"]
        assert spmv_ok(big, xb, y_big)
        done_before = 0
        for ta, x, t, y in pairs:
            ra, r = srv.wait(ta, 120.0), srv.wait(t, 120.0)
            assert ra["status"] == 0 and ra["iterations"] == 0 and r["status"] == 0
            assert spmv_ok(small, x, y)
            done_before += r["t_done_ns"] < rb["t_done_ns"]
        # the big matrix takes milliseconds to plan, stage and convert; the
        # small SpMVs behind it need a few steps each
        assert done_before == len(pairs), (done_before, rb)


def test_serve_random_sequences_keep_order_per_matrix(srv_mod):
    """Random sequences of ADMIT+SPMV/CG pairs, bare SPMVs and EVICTs over six
    matrices (two large enough that their admissions are still preparing or
    converting while later requests arrive) under a budget that forces
    evictions.  Whatever overtakes what: every SPMV/CG submitted right after
    its ADMIT succeeds and is checked against the oracle; a bare SPMV either
    succeeds (checked) or finds its matrix gone (ENOTFOUND), and finds it gone
    whenever an EVICT of that matrix succeeded after the matrix's last ADMIT
    (in submission order); EVICTs succeed or report ENOTFOUND/EBUSY."""
    print("\n[gpu] serve: random sequences", flush=True)
    from paper_1203_5737_amd import _lib
    rng = np.random.default_rng(2024)
    mats = pool(4, 1.5e4, 3e4) + [synth.shifted_laplacian(k, 150_000, np.random.default_rng(9 + i))
                                  for i, k in enumerate(("2d", "3d"))]
    with srv_mod.Server(budget_bytes=32 << 20, max_active=6) as srv:
        ops = []
        for _ in range(240):
            m = int(rng.integers(0, len(mats)))
            A = mats[m]
            u = rng.random()
            if u < 0.6:
                ta = srv.admit(m, A.rp, A.col, A.val, A.n_cols)
                if rng.random() < 0.5:
                    x = rng.uniform(-1, 1, A.n_cols).astype(np.float32)
                    ops.append(("pair-spmv", m, ta, x) + srv.spmv(m, x, A.n_rows))
                else:
                    b = rng.uniform(-1, 1, A.n_rows)
                    ops.append(("pair-cg", m, ta, b) + srv.cg(m, b))
            elif u < 0.85:
                x = rng.uniform(-1, 1, A.n_cols).astype(np.float32)
                ops.append(("bare-spmv", m, None, x) + srv.spmv(m, x, A.n_rows))
            else:
                ops.append(("evict", m, srv.evict(m), None, None, None))
        gone = {}                       # matrix -> an EVICT of it succeeded since its last ADMIT
        for kind, m, ta, inp, t, out in ops:
            A = mats[m]
            if kind == "evict":
                r = srv.wait(ta, 120.0)
                assert r["status"] in (0, _lib.ENOTFOUND, _lib.EBUSY), (kind, m, r)
                if r["status"] == 0:
                    gone[m] = True
                continue
            if ta is not None:
                ra = srv.wait(ta, 120.0)
                assert ra["status"] == 0, (kind, m, ra)
                gone[m] = False
            r = srv.wait(t, 120.0)
            if kind == "bare-spmv":
                if gone.get(m):
                    assert r["status"] == _lib.ENOTFOUND, (kind, m, r)
                    continue
                assert r["status"] in (0, _lib.ENOTFOUND), (kind, m, r)
                if r["status"] != 0:
                    continue
            else:
                assert r["status"] == 0, (kind, m, r)
            if kind == "pair-cg":
                assert true_relres(A, out, inp) <= 1e-10
            else:
                assert spmv_ok(A, inp, out)
        st = srv.stats()
        print(f"[gpu] serve random sequences: {st}", flush=True)
        assert st["evictions"] > 0, st
