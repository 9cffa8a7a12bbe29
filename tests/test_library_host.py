"""Host-side checks of libargcsr that need no GPU: the library loads, exports
every symbol the public header declares, its host planning (conversion step
1 and the step-2 slot count) agrees with the oracle, and it reports errors."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
           if f.endswith(".h")]


@pytest.fixture(scope="module")
def L():
    from paper_1203_5737_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1203_5737_amd import build
        build.build()
    return _lib.lib()


def declared_functions():
    names = set()
    for h in HEADERS:
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(argcsr_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert "argcsr_spmv" in names and "argcsr_convert" in names and len(names) >= 6
    from paper_1203_5737_amd import _lib
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, f"declared but not exported: {missing}"
    for n in names:
        assert hasattr(L, n)


def test_product_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_1203_5737_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "oracle.h" not in text, f
                assert "liboracle" not in text, f
    from paper_1203_5737_amd import _lib
    ldd = subprocess.run(["ldd", _lib.LIB_PATH], capture_output=True, text=True).stdout
    assert "oracle" not in ldd


def test_missing_library_fails_loudly(monkeypatch):
    from paper_1203_5737_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", "/nonexistent/libargcsr.so")
    with pytest.raises(ImportError):
        _lib.lib()


def plan(L, rp, T, D, fmt=0):
    rp = np.ascontiguousarray(rp, dtype=np.int32)
    g, s = ctypes.c_int32(0), ctypes.c_int64(0)
    rc = L.argcsr_plan(rp.shape[0] - 1, rp.ctypes.data_as(ctypes.c_void_p), T, D, fmt,
                       ctypes.byref(g), ctypes.byref(s), None)
    return rc, g.value, s.value


def test_plan_matches_oracle_on_workload_shapes(L, ora):
    A, _ = synth.workload_laplace64()
    Ap, _ = synth.workload_powerlaw(300_000)
    fig3 = np.array([0, 1, 2, 3, 4, 5, 6, 7, 15], dtype=np.int32)
    cases = [(fig3, 12, 2), (fig3, 12, 1), (A.rp, 64, 1), (A.rp, 64, 5), (A.rp, 256, 3),
             (Ap.rp, 64, 1), (Ap.rp, 64, 4), (Ap.rp, 128, 1), (Ap.rp, 256, 2), (Ap.rp, 7, 3)]
    for rp, T, D in cases:
        assert plan(L, rp, T, D) == ora.sizes(rp, T, D), (T, D)


@settings(max_examples=200, deadline=None)
@given(lengths=st.lists(st.integers(0, 300), min_size=0, max_size=200),
       T=st.integers(1, 300), D=st.integers(1, 40))
def test_plan_matches_oracle_random(L, ora, lengths, T, D):
    rp = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int32)
    assert plan(L, rp, T, D) == ora.sizes(rp, T, D)


@settings(max_examples=150, deadline=None)
@given(lengths=st.lists(st.integers(0, 300), min_size=0, max_size=200),
       T=st.integers(1, 300))
def test_plan_row_grouped_matches_oracle(L, ora, lengths, T):
    """Row-grouped CSR sizes (groups of T rows, chunk = longest row >= 1)."""
    rp = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int32)
    assert plan(L, rp, T, 0, 1) == ora.rg_sizes(rp, T)


@settings(max_examples=120, deadline=None)
@given(lengths=st.lists(st.integers(0, 120), min_size=0, max_size=200),
       T=st.sampled_from([1, 7, 64, 128]), region_rows=st.integers(1, 60),
       seed=st.integers(0, 2**31 - 1))
def test_plan_regions_matches_oracle(L, ora, lengths, T, region_rows, seed):
    import paper_1203_5737_amd as ac
    rng = np.random.default_rng(seed)
    rp = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int32)
    D = rng.integers(1, 9, max(1, -(-len(lengths) // region_rows))).astype(np.int32)
    rc, G, S = ora.sizes_regions(rp, T, region_rows, D)
    assert rc == 0
    assert ac.plan_regions(rp, T, region_rows, D)[:2] == (G, S)


def test_choose_region_desired_rule(L):
    """Regular regions (longest row <= 2 x mean) get their longest row,
    capped; irregular or empty regions get 1."""
    import paper_1203_5737_amd as ac
    lengths = [4, 5, 6, 5] + [1, 1, 1, 40] + [0, 0, 0, 0] + [27] * 4 + [100] * 2
    rp = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int32)
    assert ac.choose_region_desired(rp, 4, 64).tolist() == [6, 1, 1, 27, 64]
    assert ac.choose_region_desired(rp, 4, 16).tolist() == [6, 1, 1, 16, 16]
    assert ac.choose_region_desired(np.zeros(1, dtype=np.int32), 4).tolist() == []
    with pytest.raises(ac.ArgCsrError):
        ac.plan_regions(rp, 64, 4, [1, 1, 0, 1, 1])              # an entry < 1
    with pytest.raises(ac.ArgCsrError):
        ac.plan_regions(rp, 64, 0, [1])                          # region_rows < 1


def test_plan_errors(L):
    from paper_1203_5737_amd import _lib
    good = np.array([0, 2, 3], dtype=np.int32)
    assert plan(L, good, 0, 1)[0] == _lib.EINVAL
    assert plan(L, good, 64, 0)[0] == _lib.EINVAL
    assert plan(L, good, 64, 1, 2)[0] == _lib.EINVAL          # unknown format
    assert plan(L, good, 64, 0, 1)[0] == _lib.OK              # D plays no part for RgCSR
    assert plan(L, np.array([1, 2, 3], dtype=np.int32), 64, 1)[0] == _lib.EINVAL
    assert plan(L, np.array([0, 3, 2], dtype=np.int32), 64, 1)[0] == _lib.EINVAL
    assert b"decreases" in L.argcsr_last_error()
    # 17M rows of 65 nonzeros at T=64: every row alone with chunk size 2
    rp = (np.arange(17_000_001, dtype=np.int64) * 65).astype(np.int32)
    rc, G, S = plan(L, rp, 64, 1)
    assert rc == _lib.EOVERFLOW and S == 17_000_000 * 128
    assert plan(L, np.zeros(1, dtype=np.int32), 64, 1) == (0, 0, 0)


def test_gpu_entry_points_reject_bad_arguments_without_gpu(L):
    """Argument checks run before any HIP call, so they work on a CPU host."""
    from paper_1203_5737_amd import _lib
    d = _lib.MatrixDesc()
    d.block_dim, d.dtype, d.n_rows, d.n_cols = 96, 0, 10, 10
    assert L.argcsr_spmv(ctypes.byref(d), None, None, None) == _lib.EUNSUPPORTED
    d.block_dim, d.dtype = 64, 9
    assert L.argcsr_spmv(ctypes.byref(d), None, None, None) == _lib.EINVAL
    # x is gathered with 32-bit byte offsets: FP64 x of 2^29 columns is out of range
    d.dtype, d.n_cols = 0, 1 << 29
    assert L.argcsr_spmv(ctypes.byref(d), None, None, None) == _lib.EUNSUPPORTED
    d.dtype = 1                               # the same x in FP32 fits
    assert L.argcsr_spmv(ctypes.byref(d), None, None, None) == _lib.OK
    d.n_cols = 10
    assert L.argcsr_spmv(None, None, None, None) == _lib.EINVAL
    assert L.argcsr_csr_spmv(4, 4, 4, None, None, None, 0, 3, None, None, None) == _lib.EINVAL
    # server configuration: inner CG iterations per step outside 0..8
    h = ctypes.c_void_p(0)
    for per_step in (-1, 9):
        cfg = _lib.ServerConfig(1 << 20, 4, 0, 0, 0, 1e-10, 1e-5, 200, 5000, 0, per_step)
        assert L.argcsr_server_create(ctypes.byref(cfg), ctypes.byref(h)) == _lib.EINVAL
        assert not h.value


def heavy_chunk_for(T, S, G):
    """The launch-schedule threshold (documented with argcsr_matrix.heavy_groups):
    at least 4 rounds of 8 loaded steps per lane, and 4x the mean chunk size."""
    by_rounds = {64: 32, 128: 16, 256: 8}.get(T)
    if by_rounds is None or G == 0:
        return by_rounds
    return max(by_rounds, 4 * (-(-S // (G * T))))


def test_plan_heavy_count_matches_oracle_groups(L, ora):
    Ap, _ = synth.workload_powerlaw(200_000)
    A2, _ = synth.workload_stencil27(16)
    for A, T, D in [(Ap, 64, 1), (Ap, 128, 2), (Ap, 256, 1), (A2, 256, 27), (A2, 64, 1)]:
        rp = np.ascontiguousarray(A.rp, dtype=np.int32)
        g, s, h = ctypes.c_int32(0), ctypes.c_int64(0), ctypes.c_int32(0)
        assert L.argcsr_plan(rp.shape[0] - 1, rp.ctypes.data_as(ctypes.c_void_p), T, D, 0,
                             ctypes.byref(g), ctypes.byref(s), ctypes.byref(h)) == 0
        ref = ora.convert(A.rp, A.col, A.val, T, D)
        hc = heavy_chunk_for(T, ref.n_slots, ref.n_groups)
        assert h.value == int((ref.groups[:, 3] > hc).sum())


def test_autotune_model_ranking_on_host(L, ora):
    """With no finalists timed the autotuner returns the cost model's best
    pair; recompute the model from the oracle's sizes and compare."""
    import paper_1203_5737_amd as ac
    ac.autotune_clear_cache()
    for A, dt in [(synth.workload_powerlaw(100_000)[0], ac.F64),
                  (synth.workload_laplace64()[0], ac.F32)]:
        d = ac.DeviceCsr(A.n_rows, A.n_cols, A.rp, None, None, None)
        r = ac.autotune(d, dt, n_finalists=0)
        sv, sx = (8, 8) if dt == ac.F64 else (4, 4)
        best = None
        lengths = np.diff(A.rp.astype(np.int64))
        desired = [1, 2, 4, 8, 16, 32, 64]
        for extra in (int(lengths.max()), int((A.nnz + A.n_rows // 2) // A.n_rows)):
            if 1 <= extra <= 64 and extra not in desired:   # longest and mean row length
                desired.append(extra)
        for T in (64, 128, 256):
            for D in desired + [0]:                     # 0: row-grouped CSR at this T
                ref = (ora.convert(A.rp, A.col, A.val, T, D) if D
                       else ora.rg_convert(A.rp, A.col, A.val, T))
                G, S = ref.n_groups, ref.n_slots
                H = int((ref.groups[:, 3] > heavy_chunk_for(T, S, G)).sum())
                # the longest of: bytes at 5 TB/s, the groups' latency chains
                # (3 us per group, 0.15 us per 64-slot step, x4.5 for FP64) over
                # 8192 waves in flight, one group's chain; plus 2 ns per heavy group
                step = 0.15 * (4.5 if dt == ac.F64 else 1.0)
                nbytes = S * (sv + 4) + 16 * G + A.n_rows * (4 + sx) + A.n_cols * sx
                model = max(nbytes / 5e6, (3.0 * G + step * S / 64) / 8192.0,
                            3.0 + step * S / 64 / G) + 2e-3 * H
                if best is None or model < best[0]:
                    best = (model, T, D, 0 if D else 1)
        assert (r["block_dim"], r["desired_chunk_size"], r["format"]) == best[1:]
        assert abs(r["model_us"] - best[0]) < 1e-9 * max(1.0, best[0])
        assert r["n_candidates"] == 3 * (len(desired) + 1)
        assert r["n_timed"] == 0 and r["from_cache"] == 0 and r["staged"] == 0
        assert ac.autotune(d, dt, n_finalists=0)["from_cache"] == 1


def test_autotune_member_ranking_on_host(L, ora):
    """The batch-member choice is the minimum of the batch-throughput model
    over the same candidates; recompute the model from the oracle's sizes."""
    import paper_1203_5737_amd as ac
    ac.autotune_clear_cache()
    bw = {64: 5.25e6, 128: 4.9e6, 256: 4.0e6}             # bytes per us by block size
    for k, dt in [(1, ac.F32), (2, ac.F64), (5, ac.BF16)]:
        A = synth.batch_member(k, 1e3, 2e4)[0]
        r = ac.autotune_member(A.rp, dt)
        sv = {ac.F64: 8, ac.F32: 4, ac.BF16: 2}[dt]
        lengths = np.diff(A.rp.astype(np.int64))
        desired = [1, 2, 4, 8, 16, 32, 64]
        for extra in (int(lengths.max()), int((A.nnz + A.n_rows // 2) // A.n_rows)):
            if 1 <= extra <= 64 and extra not in desired:
                desired.append(extra)
        best = None
        for T in (64, 128, 256):
            for D in desired + [0]:
                ref = (ora.convert(A.rp, A.col, A.val, T, D) if D
                       else ora.rg_convert(A.rp, A.col, A.val, T))
                G, S = ref.n_groups, ref.n_slots
                cost = (S * (sv + 4) + 16 * G) / bw[T] + 3.5e-4 * G
                if best is None or cost < best[0]:
                    best = (cost, T, D, 0 if D else 1)
        assert (r["block_dim"], r["desired_chunk_size"], r["format"]) == best[1:]
        assert abs(r["model_us"] - best[0]) < 1e-9 * max(1.0, best[0])
        assert r["n_candidates"] == 3 * (len(desired) + 1)
        assert r["n_timed"] == 0 and r["measured_us"] < 0 and r["staged"] == 0
        assert ac.autotune_member(A.rp, dt)["from_cache"] == 1
    with pytest.raises(ac.ArgCsrError) as e:
        ac.autotune_member(np.array([0, 2, 1], np.int32), ac.F32)
    assert e.value.code == ac._lib.EINVAL


def test_probes_reject_bad_arguments(L):
    """The measurement probes validate their arguments on the host before
    any launch (no GPU call is made on these paths)."""
    from paper_1203_5737_amd import _lib
    assert L.argcsr_probe_read(None, -1, None, None) == _lib.EINVAL
    assert L.argcsr_probe_read(ctypes.c_void_p(16), 64, None, None) == _lib.EINVAL   # no sink
    assert L.argcsr_probe_read(ctypes.c_void_p(8), 64, ctypes.c_void_p(16), None) == _lib.EINVAL
    assert L.argcsr_probe_read(None, 0, None, None) == _lib.OK                        # nothing to read
    assert L.argcsr_probe_gather(None, 10, None, 5, 3, None, None) == _lib.EINVAL      # x_bytes
    assert L.argcsr_probe_gather(None, -1, None, 5, 8, None, None) == _lib.EINVAL
    assert L.argcsr_probe_gather(ctypes.c_void_p(16), 10, ctypes.c_void_p(16), 2**30, 8,
                                 ctypes.c_void_p(16), None) == _lib.EUNSUPPORTED
    assert L.argcsr_probe_gather(None, 0, None, 5, 4, None, None) == _lib.OK
    assert _lib.PROBE_SINK == 16384
    hdr = open(os.path.join(ROOT, "include", "argcsr.h")).read()
    assert "#define ARGCSR_PROBE_SINK 16384" in hdr


# -- packed FP32 ------------------------------------------------------------

LLVM_OBJDUMP = "/opt/rocm/llvm/bin/llvm-objdump"
PACKED_FP32 = re.compile(r"\bv_pk_(fma|add|mul)_f32\b")


def _device_asm(src_text, flags, tmp_path):
    from paper_1203_5737_amd import build
    src = tmp_path / "probe.hip"
    src.write_text(src_text)
    r = subprocess.run([build.HIPCC, *flags, "-S", "--cuda-device-only", str(src), "-o",
                        str(tmp_path / "probe.s")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return (tmp_path / "probe.s").read_text()


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="needs hipcc")
def test_build_flags_keep_packed_fp32_out(tmp_path):
    """The build's feature flag works on the device pass (the warning about it
    comes from the host pass): ordinary float2 code that hipcc -O3 turns into
    v_pk_fma_f32 without the flag gets none with the build's flags."""
    from paper_1203_5737_amd import build
    src = ("#include <hip/hip_runtime.h>\n"
           "__global__ void k(const float2* a, const float2* b, float2* c) {\n"
           "  int i = threadIdx.x + blockIdx.x * blockDim.x; float2 x = a[i], y = b[i];\n"
           "  c[i] = make_float2(x.x * y.x + 1.5f, x.y * y.y + 1.5f); }\n")
    plain = [f"--offload-arch={build.ARCH}", "-O3", "-x", "hip"]
    assert PACKED_FP32.search(_device_asm(src, plain, tmp_path)), "probe no longer packs"
    assert not PACKED_FP32.search(_device_asm(src, build.FLAGS, tmp_path))


@pytest.mark.skipif(not os.path.exists(LLVM_OBJDUMP), reason="needs llvm-objdump")
def test_built_library_has_no_packed_fp32(L, tmp_path):
    """No v_pk_{fma,add,mul}_f32 in the gfx950 code objects of the built
    library (disassembled from the offload bundles of libargcsr.so)."""
    import shutil
    from paper_1203_5737_amd import _lib
    lib = tmp_path / "lib.so"
    shutil.copy(_lib.LIB_PATH, lib)
    subprocess.run([LLVM_OBJDUMP, "--offloading", str(lib)], cwd=tmp_path, check=True,
                   capture_output=True)
    objs = sorted(p for p in tmp_path.iterdir() if "amdgcn" in p.name)
    assert objs, "no device code objects found"
    for o in objs:
        asm = subprocess.run([LLVM_OBJDUMP, "-d", "--mcpu=gfx950", str(o)], capture_output=True,
                             text=True).stdout
        assert "s_endpgm" in asm or not asm.strip()
        hit = PACKED_FP32.search(asm)
        assert not hit, f"{o.name}: {hit.group(0)}"
