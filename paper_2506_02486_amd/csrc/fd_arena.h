// fd_arena.h -- first-fit allocator over the offsets [0, size) of a device arena
// (host-only bookkeeping of the shot server; no HIP).
#pragma once

#include <stddef.h>

#include <iterator>
#include <map>

namespace fd {

// Holes are kept by offset; alloc takes the lowest hole that fits and release
// merges a freed block with the holes on either side, so freeing everything
// leaves one hole [0, size) again.
class Arena {
 public:
  explicit Arena(size_t size) {
    if (size) free_[0] = size;
  }
  // Lowest offset with n free bytes, n > 0; false (and *off untouched) if none.
  bool alloc(size_t n, size_t* off) {
    if (n == 0) return false;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t at = it->first + n;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  // Return a block that alloc handed out (same offset and size, not yet released).
  void release(size_t off, size_t n) {
    auto it = free_.emplace(off, n).first;
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
  // The holes, offset -> length, in offset order.
  const std::map<size_t, size_t>& holes() const { return free_; }

 private:
  std::map<size_t, size_t> free_;
};

}  // namespace fd
