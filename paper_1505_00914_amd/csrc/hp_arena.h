// hp_arena.h -- first-fit sub-allocator over one fixed range of bytes,
// used by the server to admit requests against a device-memory budget.  It
// only does offset bookkeeping on the host (no device calls), so it can be
// exercised on its own.
//
// Blocks are aligned to kAlign bytes.  Freed blocks are merged with free
// neighbours, so a drained arena is one free block again.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace hp {

class Arena {
 public:
  static constexpr size_t kAlign = 256;
  static constexpr size_t kFail = ~(size_t)0;

  explicit Arena(size_t bytes = 0) { reset(bytes); }

  void reset(size_t bytes) {
    free_.clear();
    used_.clear();
    size_ = bytes / kAlign * kAlign;
    in_use_ = 0;
    if (size_) free_[0] = size_;
  }

  static size_t round(size_t bytes) { return (bytes + kAlign - 1) / kAlign * kAlign; }

  // Offset of a new block of `bytes` (rounded up), or kFail when no free
  // block is large enough.  Zero-byte requests take one aligned unit.
  size_t alloc(size_t bytes) {
    const size_t need = round(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const size_t at = it->first, rest = it->second - need;
      free_.erase(it);
      if (rest) free_[at + need] = rest;
      used_[at] = need;
      in_use_ += need;
      return at;
    }
    return kFail;
  }

  // Release a block returned by alloc; false if `at` is not a live block.
  bool release(size_t at) {
    auto u = used_.find(at);
    if (u == used_.end()) return false;
    size_t start = at, len = u->second;
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
    return true;
  }

  size_t size() const { return size_; }
  size_t in_use() const { return in_use_; }
  size_t live_blocks() const { return used_.size(); }
  size_t free_blocks() const { return free_.size(); }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto &f : free_) m = f.second > m ? f.second : m;
    return m;
  }

 private:
  std::map<size_t, size_t> free_;  // offset -> length
  std::map<size_t, size_t> used_;  // offset -> length
  size_t size_ = 0, in_use_ = 0;
};

}  // namespace hp
