// First-fit allocator over one contiguous device block (offsets only; host
// code, no device calls).  The request server carves each admitted request's
// workspace from it, so admission is decided by what the block can still hold
// and no per-request hipMalloc/hipFree is needed.  Not thread-safe: the
// server calls it under its lock.
#pragma once
#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace lr {

class Arena {
 public:
  static constexpr size_t ALIGN = 256;

  explicit Arena(size_t capacity = 0) { reset(capacity); }

  void reset(size_t capacity) {
    free_.clear();
    cap_ = capacity & ~(ALIGN - 1);
    used_ = 0;
    if (cap_) free_[0] = cap_;
  }

  static size_t round_up(size_t bytes) { return (bytes + ALIGN - 1) & ~(ALIGN - 1); }

  // Lowest-offset free range that holds `bytes` (rounded up to ALIGN).
  bool alloc(size_t bytes, size_t* off) {
    const size_t need = round_up(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const size_t o = it->first, sz = it->second;
      free_.erase(it);
      if (sz > need) free_[o + need] = sz - need;
      used_ += need;
      *off = o;
      return true;
    }
    return false;
  }

  // Return a range obtained from alloc(off, bytes) with the same `bytes`;
  // merges it with free neighbours.
  void release(size_t off, size_t bytes) {
    size_t sz = round_up(bytes ? bytes : 1);
    used_ -= sz;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + sz == next->first) {
      sz += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += sz;
        return;
      }
    }
    free_[off] = sz;
  }

  bool fits(size_t bytes) const {
    const size_t need = round_up(bytes ? bytes : 1);
    for (const auto& f : free_)
      if (f.second >= need) return true;
    return false;
  }

  size_t capacity() const { return cap_; }
  size_t used() const { return used_; }
  size_t free_ranges() const { return free_.size(); }

 private:
  std::map<size_t, size_t> free_;  // offset -> size of each maximal free range
  size_t cap_ = 0, used_ = 0;
};

}  // namespace lr
