// Device memory arena of the render server: one allocation, made when the
// server starts, carved into blocks for requests.  First fit over an
// address-ordered free list; released ranges merge with free neighbours.  Any
// sub-range of a block can be released on its own, so a request can reserve an
// upper bound, give back what planning shows it does not need, and keep only
// its result after completion.  Not thread-safe: the server's mutex guards it.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace xl {

class Arena {
 public:
  static constexpr size_t kAlign = 256;
  static size_t round(size_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

  void reset(size_t bytes) {
    size_ = bytes & ~(kAlign - 1);
    used_ = 0;
    free_.clear();
    if (size_ > 0) free_[0] = size_;
  }
  size_t size() const { return size_; }
  size_t used() const { return used_; }

  // Offset of a block of `bytes` (rounded up to kAlign), or false if no free
  // range is large enough.
  bool alloc(size_t bytes, size_t* off) {
    bytes = round(bytes);
    if (bytes == 0) bytes = kAlign;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      free_.erase(it);
      if (rest > 0) free_[at] = rest;
      used_ += bytes;
      return true;
    }
    return false;
  }

  // Return [off, off + bytes) (kAlign multiples inside an allocated block).
  void release(size_t off, size_t bytes) {
    bytes = round(bytes);
    if (bytes == 0) return;
    used_ -= bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        off = prev->first;
        bytes += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      free_.erase(next);
    }
    free_[off] = bytes;
  }

 private:
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
};

}  // namespace xl
