// Parallel host copy of a few (destination, source, length) segments:
// the serving loop's preparation thread copies a matrix's CSR arrays into
// pinned staging with it while it groups the rows.  Host code only.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <thread>
#include <vector>

namespace argcsr {

// Host copies of up to kCopyThreads threads, each over a contiguous share
// of the bytes of `segs` (pieces of at least kCopyPiece bytes); the caller
// joins the returned threads.  Nothing to copy: no threads.
struct CopySeg {
  char* dst;
  const char* src;
  size_t n;
};
constexpr int kCopyThreads = 4;
constexpr size_t kCopyPiece = size_t(8) << 20;

inline std::vector<std::thread> start_copy(const CopySeg* segs, int n_segs) {
  size_t total = 0;
  for (int k = 0; k < n_segs; ++k) total += segs[k].n;
  const int n_threads =
      int(std::min<size_t>(kCopyThreads, (total + kCopyPiece - 1) / kCopyPiece));
  std::vector<std::thread> threads;
  std::vector<CopySeg> all(segs, segs + n_segs);
  for (int t = 0; t < n_threads; ++t) {
    const size_t lo = total * size_t(t) / size_t(n_threads);
    const size_t hi = total * size_t(t + 1) / size_t(n_threads);
    auto copy = [all, lo, hi] {
      size_t base = 0;                       // offset of the segment in the whole
      for (const CopySeg& c : all) {
        const size_t a = std::max(lo, base), b = std::min(hi, base + c.n);
        if (a < b) std::memcpy(c.dst + (a - base), c.src + (a - base), b - a);
        base += c.n;
      }
    };
    try {
      threads.emplace_back(copy);
    } catch (...) {                          // no thread to be had: copy this share here
      copy();
    }
  }
  return threads;
}

}  // namespace argcsr
