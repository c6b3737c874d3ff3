// arena.hpp -- first-fit allocator of partition-row ranges in a fixed arena
// (host only).  A serving context keeps one arena per tier; a source's filter
// for output l takes one contiguous range of rows per tier, so the tail
// workgroups stream it as one run.  Free ranges are kept sorted by start and
// merged with their neighbours on release.
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace rta {

class RowArena {
 public:
  void reset(int64_t capacity) {
    cap_ = capacity > 0 ? capacity : 0;
    used_ = 0;
    free_.clear();
    if (cap_ > 0) free_[0] = cap_;
  }
  int64_t capacity() const { return cap_; }
  int64_t used() const { return used_; }
  int64_t largest_free() const {
    int64_t m = 0;
    for (const auto& f : free_) m = f.second > m ? f.second : m;
    return m;
  }

  // Lowest-addressed free range of at least n rows; returns its start, or -1
  // when no free range is large enough (n < 1 is an error: -1).
  int64_t alloc(int64_t n) {
    if (n < 1) return -1;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const int64_t start = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[start + n] = len - n;
      used_ += n;
      return start;
    }
    return -1;
  }

  // Return [start, start+n) to the arena.  Returns false (and changes
  // nothing) if the range is outside the arena or overlaps a free range.
  bool release(int64_t start, int64_t n) {
    if (n < 1 || start < 0 || start + n > cap_) return false;
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first < start + n) return false;
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second > start) return false;
    }
    int64_t s = start, len = n;
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        s = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && next->first == start + n) {
      len += next->second;
      free_.erase(next);
    }
    free_[s] = len;
    used_ -= n;
    return true;
  }

  const std::map<int64_t, int64_t>& free_ranges() const { return free_; }

 private:
  int64_t cap_ = 0, used_ = 0;
  std::map<int64_t, int64_t> free_;  // start -> length
};

}  // namespace rta
