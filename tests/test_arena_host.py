"""CPU: the serving loop's device-budget sub-allocator (host bookkeeping only),
built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer and run
against a cell-map model of the same range.

After every operation the model checks that live blocks never overlap, that
the free list is exactly the maximal free runs (fully coalesced), that the
bytes in use add up, and that each allocation takes the smallest free run that
fits, the lowest such offset on ties, or fails exactly when no run fits."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1203_5737_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <vector>
#include "arena.hpp"

using argcsr::RangeAllocator;
using argcsr::kAlign;

static unsigned long long s = 0x9E3779B97F4A7C15ull;
static unsigned rnd() { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return unsigned(s); }

struct Model {
  std::vector<int> owner;                 // per kAlign cell: -1 free, else block id
  size_t cells_for(size_t bytes) const { return (bytes == 0 ? 1 : (bytes + kAlign - 1) / kAlign); }
  // smallest free run >= need, lowest offset on ties; returns cell index or -1
  long best(size_t need) const {
    long best_at = -1; size_t best_len = 0;
    for (size_t i = 0; i < owner.size();) {
      if (owner[i] != -1) { ++i; continue; }
      size_t j = i;
      while (j < owner.size() && owner[j] == -1) ++j;
      const size_t len = j - i;
      if (len >= need && (best_at < 0 || len < best_len)) { best_at = long(i); best_len = len; }
      i = j;
    }
    return best_at;
  }
  size_t runs() const {
    size_t r = 0;
    for (size_t i = 0; i < owner.size(); ++i)
      if (owner[i] == -1 && (i == 0 || owner[i - 1] != -1)) ++r;
    return r;
  }
};

int main() {
  for (int rep = 0; rep < 200; ++rep) {
    const size_t cells = rep == 0 ? 0 : 1 + rnd() % 300;
    RangeAllocator a;
    a.reset(cells * kAlign);
    Model m;
    m.owner.assign(cells, -1);
    std::vector<std::pair<size_t, size_t>> live;   // (offset, cells)
    int next_id = 0;
    for (int op = 0; op < 400; ++op) {
      if (live.empty() || rnd() % 3 != 0) {
        const size_t bytes = rnd() % 5 == 0 ? 0 : rnd() % (kAlign * (1 + rnd() % 40));
        const size_t need = m.cells_for(bytes);
        const long want = m.best(need);
        const size_t got = a.alloc(bytes);
        if (want < 0) {
          if (got != RangeAllocator::kNone) { std::printf("alloc should fail\n"); return 1; }
          continue;
        }
        if (got != size_t(want) * kAlign) {
          std::printf("best fit: got %zu want %ld\n", got, want * long(kAlign));
          return 2;
        }
        for (size_t c = 0; c < need; ++c) {
          if (m.owner[want + c] != -1) { std::printf("overlap\n"); return 3; }
          m.owner[want + c] = next_id;
        }
        ++next_id;
        live.push_back({got, need});
      } else {
        const size_t k = rnd() % live.size();
        a.release(live[k].first);
        for (size_t c = 0; c < live[k].second; ++c) m.owner[live[k].first / kAlign + c] = -1;
        live[k] = live.back();
        live.pop_back();
        if (rnd() % 4 == 0) a.release(cells * kAlign + 7);   // unknown offset: ignored
      }
      size_t used = 0;
      for (auto& b : live) used += b.second * kAlign;
      if (a.in_use() != used) { std::printf("in_use %zu vs %zu\n", a.in_use(), used); return 4; }
      if (a.free_blocks() != m.runs()) { std::printf("not coalesced\n"); return 5; }
    }
    for (auto& b : live) a.release(b.first);
    if (a.in_use() != 0 || a.free_blocks() != (cells ? 1u : 0u)) { std::printf("drain\n"); return 6; }
  }
  std::puts("arena ok");
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_range_allocator_against_model(tmp_path):
    src = tmp_path / "arena_drv.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "arena_drv"
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", CSRC, str(src), "-o", str(exe)],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "arena ok" in r.stdout, (r.returncode, r.stdout, r.stderr[-3000:])
