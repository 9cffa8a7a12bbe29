"""CPU: the serving loop's parallel host copy (CSR arrays into pinned
staging, on up to four threads beside the grouping), built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer: over random layouts of up to
five segments -- empty ones, tiny ones, sizes that are no multiple of the
piece size, totals from 0 to ~40 MB -- every destination byte equals its
source, the bytes just outside each destination are untouched, and the
number of threads is min(4, ceil(total / 8 MiB))."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1203_5737_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdint>
#include <vector>
#include "hostcopy.hpp"

using argcsr::CopySeg;
static unsigned long long s = 0x2545F4914F6CDD1Dull;
static unsigned long long rnd() { s ^= s << 13; s ^= s >> 7; s ^= s << 17; return s; }

int main() {
  const size_t kGuard = 64;
  for (int trial = 0; trial < 60; ++trial) {
    const int n_segs = int(rnd() % 6);
    std::vector<std::vector<char>> src(n_segs), dst(n_segs);
    std::vector<CopySeg> segs;
    size_t total = 0;
    for (int k = 0; k < n_segs; ++k) {
      size_t n;
      switch (rnd() % 4) {
        case 0: n = 0; break;
        case 1: n = rnd() % 97; break;
        case 2: n = rnd() % (3u << 20); break;
        default: n = (rnd() % 12) * ((size_t(1) << 20) + 13) + rnd() % 4099; break;
      }
      src[k].resize(n);
      for (size_t i = 0; i < n; ++i) src[k][i] = char(rnd());
      dst[k].assign(n + 2 * kGuard, char(0x5A));
      segs.push_back(CopySeg{dst[k].data() + kGuard, src[k].data(), n});
      total += n;
    }
    std::vector<std::thread> th = argcsr::start_copy(segs.data(), n_segs);
    const size_t want = std::min<size_t>(argcsr::kCopyThreads,
                                         (total + argcsr::kCopyPiece - 1) / argcsr::kCopyPiece);
    if (th.size() != want) { std::printf("threads %zu want %zu\n", th.size(), want); return 2; }
    for (auto& t : th) t.join();
    for (int k = 0; k < n_segs; ++k) {
      const size_t n = src[k].size();
      for (size_t i = 0; i < kGuard; ++i)
        if (dst[k][i] != char(0x5A) || dst[k][kGuard + n + i] != char(0x5A)) {
          std::printf("guard %d\n", k); return 3;
        }
      for (size_t i = 0; i < n; ++i)
        if (dst[k][kGuard + i] != src[k][i]) { std::printf("byte %d %zu\n", k, i); return 4; }
    }
  }
  std::puts("hostcopy ok");
  return 0;
}
"""


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_parallel_host_copy(tmp_path):
    src = tmp_path / "hostcopy_drv.cpp"
    src.write_text(DRIVER)
    exe = tmp_path / "hostcopy_drv"
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-pthread", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", CSRC, str(src), "-o", str(exe)],
                   check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "hostcopy ok" in r.stdout, (r.returncode, r.stdout, r.stderr[-3000:])
