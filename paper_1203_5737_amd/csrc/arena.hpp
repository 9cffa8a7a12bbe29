// Best-fit sub-allocator with coalescing over one contiguous range (the
// serving loop's device memory budget).  Host-only bookkeeping: it hands out
// offsets inside [0, capacity); the caller maps them onto its allocation.
#pragma once

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>

namespace argcsr {

constexpr size_t kAlign = 256;

class RangeAllocator {
 public:
  static constexpr size_t kNone = ~size_t(0);

  void reset(size_t capacity) {
    capacity_ = capacity;
    in_use_ = 0;
    free_.clear();
    used_.clear();
    if (capacity > 0) free_[0] = capacity;
  }
  // Offset of a block of at least `bytes` (rounded up to kAlign), or kNone.
  size_t alloc(size_t bytes) {
    bytes = (std::max<size_t>(bytes, 1) + kAlign - 1) / kAlign * kAlign;
    auto best = free_.end();
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes && (best == free_.end() || it->second < best->second)) best = it;
    if (best == free_.end()) return kNone;
    const size_t off = best->first, len = best->second;
    free_.erase(best);
    if (len > bytes) free_[off + bytes] = len - bytes;
    used_[off] = bytes;
    in_use_ += bytes;
    return off;
  }
  // Returns a block to the free list, merging with free neighbours.  Unknown
  // offsets are ignored.
  void release(size_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t start = off, len = u->second;
    in_use_ -= len;
    used_.erase(u);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
  }
  size_t in_use() const { return in_use_; }
  size_t capacity() const { return capacity_; }
  size_t free_blocks() const { return free_.size(); }

 private:
  size_t capacity_ = 0, in_use_ = 0;
  std::map<size_t, size_t> free_;   // offset -> length
  std::map<size_t, size_t> used_;   // offset -> length
};

}  // namespace argcsr
