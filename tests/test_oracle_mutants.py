"""The pins are strong enough: plant a plausible mistake in a copy of the
oracle (on the CPU), rebuild it, and check that at least one pin fails.

Each mutant is a one-token edit of oracle.c: a dropped term, a flipped sign,
an off-by-one index, a transposed layout, a wrong tie rule, the other reading
of an ambiguous passage.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
import test_oracle_pins as pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "oracle.c")

MUTANTS = {
    "grouping_keeps_overflowing_row": ("open_count + L > limit", "open_count > limit"),
    "grouping_row_limit_off_by_one": ("open_size + 1 > block_dim", "open_size > block_dim"),
    "greedy_gives_thread_to_smallest": ("if (fill > best_fill) { best_fill = fill; best = l; }",
                                        "if (best_fill < 0 || fill < best_fill) { best_fill = fill; best = l; }"),
    "chunk_size_may_be_zero": ("int64_t chunk = 1;", "int64_t chunk = 0;"),
    "threads_mapping_exclusive": ("running += t[l];\n            tm[first[g] + l] = running;",
                                  "tm[first[g] + l] = running;\n            running += t[l];"),
    "layout_row_major_chunks": ("const int64_t slot = offset + (int64_t)j * block_dim +\n                                         first_chunk + q;",
                                "const int64_t slot = offset + (int64_t)(first_chunk + q) * c + j;"),
    "chunks_interleaved": ("const int64_t e = (int64_t)q * c + j;", "const int64_t e = (int64_t)j * t[l] + q;"),
    "offset_forgets_block_dim": ("offset += (int64_t)c * block_dim;", "offset += (int64_t)c;"),
    "csr_drops_last_term": ("for (int64_t k = rp[i]; k < rp[i + 1]; k++)", "for (int64_t k = rp[i]; k + 1 < rp[i + 1]; k++)"),
    "csr_wrong_sign": ("sum = sum + val[k] * x[col[k]];", "sum = sum - val[k] * x[col[k]];"),
    "row_chunks_wrong_begin": ("const int32_t b = (r == first) ? 0 : tm[r - 1];",
                               "const int32_t b = (r == first) ? 0 : tm[r - 1] - 1;"),
    "row_chunks_stop_one_early": ("for (int32_t k = b; k < tm[r]; k++) {\n                for (int32_t j = 0; j < chunk; j++) {\n                    const int64_t s = (int64_t)offset + (int64_t)j * block_dim + k;\n                    if (columns[s] == -1) break;\n                    sum",
                                  "for (int32_t k = b; k + 1 < tm[r]; k++) {\n                for (int32_t j = 0; j < chunk; j++) {\n                    const int64_t s = (int64_t)offset + (int64_t)j * block_dim + k;\n                    if (columns[s] == -1) break;\n                    sum"),
    "chunk_sum_transposed_index": ("const int64_t s = (int64_t)offset + (int64_t)j * block_dim + k;\n                    if (columns[s] == -1) break;\n                    sum",
                                   "const int64_t s = (int64_t)offset + (int64_t)k * chunk + j;\n                    if (s >= (int64_t)offset + (int64_t)chunk * block_dim || columns[s] == -1) break;\n                    sum"),
    "rounding_ties_to_odd": ("fmod(k, 2.0) != 0.0", "fmod(k, 2.0) == 0.0"),
    "rounding_ties_away": ("frac > 0.5 ||", "frac >= 0.5 ||"),
    "rounding_no_subnormal_quantum": ("(ue < emin ? emin : ue) - man_bits", "ue - man_bits"),
    "f32_truncates": ("((float*)values)[slot] = (float)v;", "((float*)values)[slot] = nextafterf((float)v, 0.0f);"),
    "regions_limit_of_current_row": ("        if (open_size == 0)                  /* row r opens a group */",
                                     "        if (1)                  /* row r opens a group */"),
    "rg_width_may_be_zero": ("        const int64_t rows = (n_rows - first < block_dim) ? n_rows - first : block_dim;\n        int64_t w = 1;",
                             "        const int64_t rows = (n_rows - first < block_dim) ? n_rows - first : block_dim;\n        int64_t w = 0;"),
    "rg_layout_row_major": ("columns[offset + e * block_dim + l] = col[rp[r] + e];\n                store_value(values, dtype, offset + e * block_dim + l,",
                            "columns[offset + l * w + e] = col[rp[r] + e];\n                store_value(values, dtype, offset + l * w + e,"),
    "rg_mapping_exclusive": ("tm[r] = (int32_t)(l + 1);", "tm[r] = (int32_t)l;"),
    "stage_gap_strict": ("(int64_t)u[i + 1] - last - 1 <= gap", "(int64_t)u[i + 1] - last - 1 < gap"),
    "stage_tiles_of_63": ("for (int64_t t = start; t <= last; t += 64) {", "for (int64_t t = start; t <= last; t += 63) {"),
    "stage_local_window_packed": ("v = (uint16_t)(64 * q + (c - ts[q]));", "v = (uint16_t)(q + (c - ts[q]));"),
    "stage_tile_drops_last_column": ("tl[nt] = (int32_t)(last - t + 1 < 64 ? last - t + 1 : 64);",
                                     "tl[nt] = (int32_t)(last - t < 64 ? last - t : 64);"),
    "rg_slices_offset_by_one": ("groups[4 * g + 0] = (int32_t)first;", "groups[4 * g + 0] = (int32_t)first + (g > 0);"),
}

BATTERY = [
    pins.test_fig3_worked_example,
    pins.test_fig3_with_desired_chunk_size_one,
    pins.test_chunk_size_is_optimal_by_brute_force,
    pins.test_uniform_rows_give_sliced_ellpack_layout,
    pins.test_diagonal_matrix,
    pins.test_single_long_row,
    pins.test_empty_matrix_and_empty_rows,
    pins.test_dense_matvec_small_integers_bitwise,
    pins.test_laplace5_polynomials,
    pins.test_f16_rounding_matches_numpy,
    pins.test_bf16_rounding_is_nearest_even,
    pins.test_invariants_powerlaw_sample,
    pins.test_regions_hand_worked_example,
    pins.test_regions_group_keeps_its_limit_after_crossing,
    pins.test_regions_groups_are_greedy_maximal,
    pins.test_rgcsr_fig3_one_thread_per_row,
    pins.test_rgcsr_uniform_rows_closed_form,
    pins.test_rgcsr_equals_argcsr_with_unbounded_budget,
    pins.test_rgcsr_partial_last_slice_keeps_one_chunk_per_row,
    pins.test_rgcsr_roundtrip_and_spmv_is_csr_order,
    pins.test_stage_hand_worked_example,
    pins.test_stage_laplace_closed_form,
    pins.test_stage_matches_occupancy_definition,
]


def f32_battery(ora):
    rng = np.random.default_rng(3)
    v = rng.uniform(-1, 1, 1000)
    rp = np.arange(1001, dtype=np.int32)
    a = ora.convert(rp, np.arange(1000, dtype=np.int32), v, 64, 1, ora.F32)
    assert np.array_equal(a.values[a.columns >= 0], v.astype(np.float32))


BATTERY.append(f32_battery)


def run_battery(ora):
    failures = []
    for fn in BATTERY:
        try:
            fn(ora)
        except Exception as e:                     # noqa: BLE001 - any failure counts
            failures.append(f"{fn.__name__}: {type(e).__name__}")
    return failures


def test_unmutated_oracle_passes_battery():
    assert run_battery(oracle) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor not unique/found: {name}"
    (tmp_path / "oracle.h").write_text(open(SRC.replace(".c", ".h")).read())
    (tmp_path / "oracle.c").write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-o", str(so), str(tmp_path / "oracle.c"), "-lm"], check=True)
    # run the battery in a child process: a mutant may also crash outright
    # (e.g. divide by a zero chunk size), which counts as caught.  The
    # property-based pins draw a fixed sequence of examples there, so whether
    # a mutant is caught does not depend on the run.
    code = (
        "import ctypes, sys; sys.path[:0] = [%r, %r]\n"
        "from hypothesis import settings\n"
        "settings.register_profile('fixed', derandomize=True, database=None)\n"
        "settings.load_profile('fixed')\n"
        "import oracle, test_oracle_mutants as m\n"
        "oracle._lib = oracle._bind(ctypes.CDLL(%r))\n"
        "print('START', flush=True)\n"
        "f = m.run_battery(oracle)\n"
        "print(f)\n"
        "sys.exit(1 if f else 0)\n"
    ) % (os.path.dirname(os.path.dirname(SRC)), os.path.dirname(__file__), str(so))
    proc = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=600)
    assert "START" in proc.stdout, proc.stderr[-2000:]          # the harness itself worked
    assert proc.returncode != 0, f"mutant {name} survived every pin: {proc.stdout[-500:]}"
