// First-fit allocator of integer ranges in [0, cap), used by the serving
// engine for time rows and combine ids.  Host-only C++ (no HIP), so the unit
// test builds it with the host compiler alone.
#pragma once

#include <iterator>
#include <map>

namespace dsmc {

class RangeAlloc {
 public:
  void reset(int cap) {
    free_.clear();
    if (cap > 0) free_[0] = cap;
  }
  // Start of the first free range of at least len units, or -1.
  int alloc(int len) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= len) {
        const int start = it->first, rem = it->second - len;
        free_.erase(it);
        if (rem) free_[start + len] = rem;
        return start;
      }
    }
    return -1;
  }
  // Return [start, start + len); adjacent free ranges are merged.
  void release(int start, int len) {
    if (len <= 0) return;
    auto it = free_.emplace(start, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  // Free ranges (start -> length), for tests.
  const std::map<int, int>& free_ranges() const { return free_; }

 private:
  std::map<int, int> free_;
};

}  // namespace dsmc
