// Best-fit allocator of offsets in [0, size) for the server's device arena
// (host-only bookkeeping: no device calls).  Blocks are 256-byte aligned;
// freed neighbours coalesce.  Not thread-safe except used()/peak(), which
// may be read from any thread.
#pragma once

#include <algorithm>
#include <atomic>
#include <cstddef>
#include <map>

namespace fdwt {

constexpr size_t kNone = ~(size_t)0;

inline size_t arena_round(size_t b) { return (std::max<size_t>(b, 1) + 255) & ~(size_t)255; }

class Arena {
 public:
  void reset(size_t size) {
    free_by_off_.clear();
    free_by_size_.clear();
    size_ = size;
    used_ = 0;
    peak_ = 0;
    if (size) insert_free(0, size);
  }
  // Offset of a free block of at least `bytes`, or kNone.
  size_t alloc(size_t bytes) {
    bytes = arena_round(bytes);
    auto it = free_by_size_.lower_bound(bytes);
    if (it == free_by_size_.end()) return kNone;
    const size_t off = it->second, sz = it->first;
    erase_free(off, sz);
    if (sz > bytes) insert_free(off + bytes, sz - bytes);
    used_ += bytes;
    if (used_.load() > peak_.load()) peak_ = used_.load();
    return off;
  }
  // Returns a block obtained from alloc(bytes).
  void release(size_t off, size_t bytes) {
    bytes = arena_round(bytes);
    used_ -= bytes;
    size_t o = off, sz = bytes;
    auto nx = free_by_off_.lower_bound(o);
    if (nx != free_by_off_.end() && nx->first == o + sz) {
      sz += nx->second;
      erase_free(nx->first, nx->second);
    }
    auto pv = free_by_off_.lower_bound(o);
    if (pv != free_by_off_.begin()) {
      --pv;
      if (pv->first + pv->second == o) {
        o = pv->first;
        sz += pv->second;
        erase_free(pv->first, pv->second);
      }
    }
    insert_free(o, sz);
  }
  size_t used() const { return used_.load(); }
  size_t peak() const { return peak_.load(); }
  size_t size() const { return size_; }
  size_t free_blocks() const { return free_by_off_.size(); }
  size_t largest_free() const { return free_by_size_.empty() ? 0 : free_by_size_.rbegin()->first; }

 private:
  void insert_free(size_t off, size_t sz) {
    free_by_off_[off] = sz;
    free_by_size_.emplace(sz, off);
  }
  void erase_free(size_t off, size_t sz) {
    free_by_off_.erase(off);
    auto r = free_by_size_.equal_range(sz);
    for (auto i = r.first; i != r.second; ++i)
      if (i->second == off) {
        free_by_size_.erase(i);
        break;
      }
  }
  std::map<size_t, size_t> free_by_off_;
  std::multimap<size_t, size_t> free_by_size_;
  size_t size_ = 0;
  std::atomic<size_t> used_{0}, peak_{0};
};

}  // namespace fdwt
