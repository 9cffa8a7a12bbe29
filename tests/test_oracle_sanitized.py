"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU):
conversion, inverse, both SpMV forms, rounding, staging and CG on random inputs,
including empty rows and matrices, must run without any sanitizer report."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

static unsigned long long s = 88172645463325252ull;
static unsigned rnd(void) { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return (unsigned)s; }

int main(void) {
  for (int rep = 0; rep < 300; rep++) {
    int n = rnd() % 200, ncol = 1 + rnd() % 300, T = 1 + rnd() % 70, D = 1 + rnd() % 5;
    int *rp = malloc(sizeof(int) * (n + 1));
    rp[0] = 0;
    for (int i = 0; i < n; i++) rp[i + 1] = rp[i] + (rnd() % 7 == 0 ? 0 : (int)(rnd() % 12));
    if (rep % 50 == 0 && n > 0) rp[n] = rp[n - 1] + 400;          /* one long row */
    int nnz = rp[n];
    int *col = malloc(sizeof(int) * (nnz + 1));
    double *val = malloc(sizeof(double) * (nnz + 1)), *x = malloc(sizeof(double) * ncol);
    for (int k = 0; k < nnz; k++) { col[k] = rnd() % ncol; val[k] = (double)(rnd() % 2001) / 1000.0 - 1.0; }
    for (int j = 0; j < ncol; j++) x[j] = (double)(rnd() % 2001) / 1000.0 - 1.0;
    if (ora_csr_check(n, ncol, nnz, rp, col) != ORA_OK) return 1;
    int G; long long S64; int64_t S;
    if (ora_argcsr_sizes(n, rp, T, D, &G, &S) != ORA_OK) return 2;
    S64 = S;
    int dt = rnd() % 4, bytes = dt == 0 ? 8 : dt == 1 ? 4 : 2;
    int *groups = malloc(sizeof(int) * 4 * (G + 1)), *tm = malloc(sizeof(int) * (n + 1));
    int *cols = malloc(sizeof(int) * (S64 + 1));
    void *vals = malloc((size_t)bytes * (S64 + 1));
    if (ora_argcsr_convert(n, rp, col, val, T, D, dt, groups, tm, cols, vals) != ORA_OK) return 3;
    double *v64 = malloc(sizeof(double) * (S64 + 1)), *y1 = malloc(sizeof(double) * (n + 1)),
           *y2 = malloc(sizeof(double) * (n + 1)), *val2 = malloc(sizeof(double) * (nnz + 1));
    ora_decode_array(S64, vals, dt, v64);
    ora_argcsr_spmv(G, groups, tm, cols, v64, T, x, y1);
    ora_csr_spmv(n, rp, col, val, x, y2, 1 + rep % 3);
    int *rp2 = malloc(sizeof(int) * (n + 1)), *col2 = malloc(sizeof(int) * (nnz + 1));
    if (ora_argcsr_to_csr(n, G, groups, tm, cols, v64, T, rp2, col2, val2) != nnz) return 4;
    if (n > 0 && memcmp(rp, rp2, sizeof(int) * (n + 1)) != 0) return 5;
    {   /* staging of x: sizing pass, filling pass, inverse */
      int *tp = malloc(sizeof(int) * (G + 1));
      int gap = (int)(rnd() % 5);
      int64_t nt = ora_stage(G, groups, cols, T, gap, 1023, tp, NULL, NULL, 0, NULL);
      if (nt >= 0) {
        int *ts = malloc(sizeof(int) * (nt + 1)), *tl = malloc(sizeof(int) * (nt + 1));
        uint16_t *loc = malloc(sizeof(uint16_t) * (S64 + 1));
        int *back = malloc(sizeof(int) * (S64 + 1));
        if (ora_stage(G, groups, cols, T, gap, 1023, tp, ts, tl, nt, loc) != nt) return 10;
        ora_unstage(G, groups, T, tp, ts, loc, back);
        if (S64 > 0 && memcmp(back, cols, sizeof(int) * S64) != 0) return 11;
        free(ts); free(tl); free(loc); free(back);
      }
      free(tp);
    }
    ora_round_array(nnz, val, 2, vals);
    {   /* row-grouped CSR in the same arrays, decoded back */
      int RG; int64_t RS;
      if (ora_rgcsr_sizes(n, rp, T, &RG, &RS) != ORA_OK) return 7;
      int *rgroups = malloc(sizeof(int) * 4 * (RG + 1)), *rcols = malloc(sizeof(int) * (RS + 1));
      double *rvals = malloc(sizeof(double) * (RS + 1));
      if (ora_rgcsr_convert(n, rp, col, val, T, 0, rgroups, tm, rcols, rvals) != ORA_OK) return 8;
      if (ora_argcsr_to_csr(n, RG, rgroups, tm, rcols, rvals, T, rp2, col2, val2) != nnz) return 9;
      free(rgroups); free(rcols); free(rvals);
    }
    free(rp); free(col); free(val); free(x); free(groups); free(tm); free(cols); free(vals);
    free(v64); free(y1); free(y2); free(val2); free(rp2); free(col2);
  }
  /* CG on a small SPD tridiagonal system */
  int n = 50, rp[51], col[148]; double val[148], b[50], xs[50], rel;
  int k = 0; rp[0] = 0;
  for (int i = 0; i < n; i++) {
    if (i > 0) { col[k] = i - 1; val[k++] = -1.0; }
    col[k] = i; val[k++] = 2.5;
    if (i < n - 1) { col[k] = i + 1; val[k++] = -1.0; }
    rp[i + 1] = k; b[i] = 1.0;
  }
  ora_cg(n, rp, col, val, b, xs, 1e-10, 500, &rel);
  if (!(rel <= 1e-10)) return 6;
  puts("sanitized ok");
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_ubsan(tmp_path):
    src = tmp_path / "drv.c"
    src.write_text(DRIVER)
    exe = tmp_path / "drv"
    odir = os.path.join(ROOT, "oracle")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fopenmp",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", odir, str(src), os.path.join(odir, "oracle.c"), "-o", str(exe), "-lm"],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "sanitized ok" in r.stdout, (r.returncode, r.stderr[-3000:])
