// Offsets inside one device block of fixed size (host-side bookkeeping
// only; no device calls): the serving loop's budget.  Resident scenes are
// placed from the low end and the transient step blocks from the high end,
// so that steps coming and going do not split the space that scenes need.
// Free ranges are kept by offset and merged with their neighbours on
// release.  Sizes are rounded up to 256 bytes.
#pragma once
#include <stdint.h>

#include <iterator>
#include <map>

namespace bfc {

class Heap {
 public:
  explicit Heap(int64_t size = 0) { reset(size); }

  void reset(int64_t size) {
    free_.clear();
    size_ = size & ~(int64_t)255;
    used_ = peak_ = 0;
    if (size_ > 0) free_[0] = size_;
  }

  static int64_t round(int64_t bytes) { return (bytes + 255) & ~(int64_t)255; }

  // Offset of a new block of `bytes`, or -1 if no free range holds it.  low:
  // the lowest range that fits below `limit` (default: the end), block at
  // its start; else the highest range that fits, block at its end.
  int64_t alloc(int64_t bytes, bool low, int64_t limit = -1) {
    const int64_t n = round(bytes < 1 ? 1 : bytes);
    if (limit < 0) limit = size_;
    auto pick = free_.end();
    if (low) {
      for (auto it = free_.begin(); it != free_.end() && it->first + n <= limit; ++it)
        if (it->second >= n) { pick = it; break; }
    } else {
      for (auto it = free_.rbegin(); it != free_.rend(); ++it)
        if (it->second >= n) { pick = std::prev(it.base()); break; }
    }
    if (pick == free_.end()) return -1;
    const int64_t off = pick->first, len = pick->second;
    int64_t at;
    if (low) {
      at = off;
      free_.erase(pick);
      if (len > n) free_[off + n] = len - n;
    } else {
      at = off + len - n;
      if (len > n) pick->second = len - n;
      else free_.erase(pick);
    }
    used_ += n;
    if (used_ > peak_) peak_ = used_;
    return at;
  }

  // Return a block from alloc (same size argument).
  void release(int64_t off, int64_t bytes) {
    const int64_t n = round(bytes < 1 ? 1 : bytes);
    used_ -= n;
    auto next = free_.lower_bound(off);
    int64_t start = off, len = n;
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    if (next != free_.end() && next->first == off + n) {
      len += next->second;
      free_.erase(next);
    }
    free_[start] = len;
  }

  int64_t size() const { return size_; }
  int64_t used() const { return used_; }
  int64_t peak() const { return peak_; }
  int64_t largest_free() const {
    int64_t m = 0;
    for (const auto& kv : free_) m = kv.second > m ? kv.second : m;
    return m;
  }
  int ranges() const { return (int)free_.size(); }

 private:
  std::map<int64_t, int64_t> free_;  // offset -> length
  int64_t size_ = 0, used_ = 0, peak_ = 0;
};

}  // namespace bfc
