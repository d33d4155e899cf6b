// Host bookkeeping of the served loop's device arena (plain C++: no device
// code, so a host-only test builds it as it is).
#pragma once

#include <cstdint>
#include <iterator>
#include <map>

namespace mpc {

// Allocator over [0, units) with coalescing (host bookkeeping of the device
// arena): state slots first-fit from the low end, workspace slots from the
// highest fit down, so the workspace of a batch stays contiguous, apart from
// the long-lived states, and coalesces back as the batch retires.
class Arena {
 public:
  void init(int64_t units) {
    free_.clear();
    if (units > 0) free_[0] = units;
    free_units_ = units;
  }
  int64_t alloc(int64_t units) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= units) {
        const int64_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > units) free_[off + units] = len - units;
        free_units_ -= units;
        return off;
      }
    }
    return -1;
  }
  int64_t alloc_high(int64_t units) {
    for (auto it = free_.rbegin(); it != free_.rend(); ++it) {
      if (it->second >= units) {
        const int64_t off = it->first + it->second - units;
        if (it->second == units) free_.erase(std::next(it).base());
        else it->second -= units;
        free_units_ -= units;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t units) {
    free_units_ += units;
    auto it = free_.emplace(off, units).first;
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
  int64_t free_units() const { return free_units_; }
  size_t fragments() const { return free_.size(); }  // free blocks

 private:
  std::map<int64_t, int64_t> free_;
  int64_t free_units_ = 0;
};

}  // namespace mpc
