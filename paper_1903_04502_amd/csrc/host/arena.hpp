// First-fit allocator over byte offsets of one caller-owned arena (the
// serving admission; host, plain C++, also built alone with sanitizers by the
// CPU tests). Free blocks are kept sorted by offset and merged with their
// neighbours when a block is released, so a fully released arena is one block.
#pragma once

#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>

namespace pr {

class ArenaFreeList {
 public:
  void reset(size_t bytes) {
    free_.clear();
    if (bytes) free_[0] = bytes;
  }
  // Lowest-offset free block of at least `bytes` (> 0); false if none.
  bool alloc(size_t bytes, size_t* off) {
    if (bytes == 0) return false;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t roff = it->first + bytes;
        free_.erase(it);
        if (rest) free_[roff] = rest;
        return true;
      }
    }
    return false;
  }
  // Return [off, off + bytes) (a block alloc handed out, not yet released).
  void release(size_t off, size_t bytes) {
    if (bytes == 0) return;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t free_bytes() const {
    size_t f = 0;
    for (const auto& kv : free_) f += kv.second;
    return f;
  }
  size_t largest() const {
    size_t l = 0;
    for (const auto& kv : free_) l = std::max(l, kv.second);
    return l;
  }
  const std::map<size_t, size_t>& blocks() const { return free_; }

 private:
  std::map<size_t, size_t> free_;   // offset -> length
};

}  // namespace pr
