// ccl_pool.h -- first-fit sub-allocator over one caller-owned byte range.
//
// Host-only bookkeeping of the serving loop (no HIP calls): offsets into a
// device buffer, every block rounded up to 256 bytes, free neighbours merged
// on release.  Not thread-safe; the server that owns it is used by one host
// thread at a time.
#ifndef CCL_POOL_H
#define CCL_POOL_H

#include <stddef.h>
#include <stdint.h>

#include <iterator>
#include <map>

namespace ccl {

class Pool {
 public:
  static constexpr size_t ALIGN = 256;
  static constexpr size_t NONE = ~(size_t)0;

  explicit Pool(size_t bytes = 0) { reset(bytes); }

  void reset(size_t bytes) {
    size_ = bytes / ALIGN * ALIGN;
    used_ = 0;
    free_.clear();
    if (size_) free_[0] = size_;
  }

  static size_t round(size_t n) { return (n + ALIGN - 1) / ALIGN * ALIGN; }

  // offset of a block of at least n bytes (n = 0 takes one unit), or NONE
  size_t alloc(size_t n) {
    n = round(n ? n : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      size_t off = it->first, rest = it->second - n;
      free_.erase(it);
      if (rest) free_[off + n] = rest;
      used_ += n;
      return off;
    }
    return NONE;
  }

  // give back a block returned by alloc(n) with the same n
  void release(size_t off, size_t n) {
    n = round(n ? n : 1);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && off + it->second == nx->first) {
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

  size_t size() const { return size_; }
  size_t used() const { return used_; }
  size_t free_blocks() const { return free_.size(); }
  size_t largest_free() const {
    size_t m = 0;
    for (auto& f : free_) m = f.second > m ? f.second : m;
    return m;
  }

 private:
  size_t size_ = 0, used_ = 0;
  std::map<size_t, size_t> free_;  // offset -> bytes, disjoint, never adjacent
};

}  // namespace ccl

#endif  // CCL_POOL_H
