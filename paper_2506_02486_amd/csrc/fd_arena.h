// fd_arena.h -- allocators over the offsets [0, size) of a device arena (host-only
// bookkeeping of the shot server; no HIP).
//
// The shot server carves every shot's buffers out of one caller-owned device
// arena, as the paper's runtime carves device allocations out of its one global
// segment with a linear-heap or a buddy allocator (Sec. 3.1).  Two policies:
//   Arena      : first fit over a list of holes (the default);
//   BuddyArena : binary buddy blocks of a power of two times a unit.
#pragma once

#include <stddef.h>

#include <iterator>
#include <map>
#include <set>
#include <vector>

namespace fd {

class ArenaAllocator {
 public:
  virtual ~ArenaAllocator() = default;
  // Offset of a block of at least n bytes, n > 0; false (and *off untouched) if none.
  virtual bool alloc(size_t n, size_t* off) = 0;
  // Return a block that alloc handed out (same offset and n, not yet released).
  virtual void release(size_t off, size_t n) = 0;
};

// First fit.  Holes are kept by offset; alloc takes the lowest hole that fits and
// release merges a freed block with the holes on either side, so freeing everything
// leaves one hole [0, size) again.
class Arena : public ArenaAllocator {
 public:
  explicit Arena(size_t size) {
    if (size) free_[0] = size;
  }
  bool alloc(size_t n, size_t* off) override {
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
  void release(size_t off, size_t n) override {
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

// Binary buddy allocator.  The arena is covered from offset 0 by "roots": the
// largest power-of-two number of units that fits, then the largest that fits in the
// rest, and so on (each root aligned to its own size).  A block of order o is
// unit << o bytes at an offset that is a multiple of its size; a request takes the
// lowest-offset free block of the smallest order that holds it, splitting it in
// halves down to the order of the request (the upper halves become free blocks),
// and a released block merges with its buddy (the other half of its parent) while
// that buddy is free and the parent lies within one root.  Free blocks are
// therefore always the maximal free aligned blocks.  The remainder of the arena
// below one unit is never handed out.
class BuddyArena : public ArenaAllocator {
 public:
  // unit: a power of two (bytes).
  BuddyArena(size_t size, size_t unit) : unit_(unit) {
    size_t units = size / unit;
    size_t at = 0;
    while (units) {
      int o = 0;
      while (((size_t)2 << o) <= units) ++o;
      roots_[at] = o;
      grow(o);
      free_[o].insert(at);
      at += unit << o;
      units -= (size_t)1 << o;
    }
  }
  bool alloc(size_t n, size_t* off) override {
    if (n == 0) return false;
    const int want = order_for(n);
    int o = want;
    while (o < (int)free_.size() && free_[o].empty()) ++o;
    if (o >= (int)free_.size()) return false;
    size_t at = *free_[o].begin();
    free_[o].erase(free_[o].begin());
    while (o > want) {  // keep the lower half, free the upper
      --o;
      free_[o].insert(at + (unit_ << o));
    }
    *off = at;
    return true;
  }
  void release(size_t off, size_t n) override {
    int o = order_for(n);
    const int top = root_order(off);
    while (o < top) {
      const size_t buddy = off ^ (unit_ << o);
      auto it = free_[o].find(buddy);
      if (it == free_[o].end()) break;
      free_[o].erase(it);
      if (buddy < off) off = buddy;
      ++o;
    }
    free_[o].insert(off);
  }
  // Smallest order whose blocks hold n bytes.
  int order_for(size_t n) const {
    int o = 0;
    while ((unit_ << o) < n) ++o;
    return o;
  }
  size_t unit() const { return unit_; }
  // Free blocks by order (offsets in increasing order).
  const std::vector<std::set<size_t>>& free_blocks() const { return free_; }
  // Root blocks: offset -> order.
  const std::map<size_t, int>& roots() const { return roots_; }

 private:
  void grow(int o) {
    if ((int)free_.size() <= o) free_.resize(o + 1);
  }
  int root_order(size_t off) const {
    auto it = roots_.upper_bound(off);
    --it;
    return it->second;
  }
  size_t unit_;
  std::map<size_t, int> roots_;
  std::vector<std::set<size_t>> free_;
};

}  // namespace fd
