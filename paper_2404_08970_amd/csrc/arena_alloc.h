// First-fit allocator over one caller-provided block of device memory, used
// by the request loop to admit requests by their HBM footprint.  Host-only
// bookkeeping (it never touches the memory): free ranges are kept sorted by
// offset and merged with their neighbours on release, so the largest free
// range is exact and fragmentation is limited to holes between live requests.
#pragma once
#include <stddef.h>

#include <iterator>
#include <map>

namespace gwr {

class RangeAllocator {
 public:
  static constexpr size_t kAlign = 256;
  static constexpr size_t kFail = ~(size_t)0;

  explicit RangeAllocator(size_t bytes = 0) { reset(bytes); }

  void reset(size_t bytes) {
    free_.clear();
    live_.clear();
    cap_ = bytes / kAlign * kAlign;
    used_ = 0;
    if (cap_) free_[0] = cap_;
  }

  static size_t round(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

  // Offset of a new range of at least n bytes (lowest address that fits), or
  // kFail.  n = 0 is served as kAlign bytes.
  size_t alloc(size_t n) {
    n = round(n ? n : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[off + n] = len - n;
      live_[off] = n;
      used_ += n;
      return off;
    }
    return kFail;
  }

  // Release the range that starts at `off`; returns false if no live range
  // starts there.
  bool release(size_t off) {
    auto lv = live_.find(off);
    if (lv == live_.end()) return false;
    size_t len = lv->second;
    live_.erase(lv);
    used_ -= len;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + len == next->first) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return true;
      }
    }
    free_[off] = len;
    return true;
  }

  size_t capacity() const { return cap_; }
  size_t used() const { return used_; }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& kv : free_)
      if (kv.second > m) m = kv.second;
    return m;
  }
  size_t free_ranges() const { return free_.size(); }
  size_t live_ranges() const { return live_.size(); }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
  std::map<size_t, size_t> live_;  // offset -> length
  size_t cap_ = 0, used_ = 0;
};

}  // namespace gwr
