// arena.h -- best-fit allocator over a byte range (host-side bookkeeping of
// the serving loop's output arena).  Pure C++; no device code.
#pragma once
#include <cstdint>
#include <map>
#include <set>
#include <utility>

namespace gx {

// Best-fit allocator over the caller's output arena (256-byte granules):
// free blocks indexed by size for allocation and by offset for merging.
class Arena {
 public:
  explicit Arena(uint64_t bytes) { insert(0, bytes & ~255ull); }
  bool alloc(uint64_t bytes, uint64_t* off) {
    bytes = (bytes + 255) & ~255ull;
    auto it = by_size_.lower_bound({bytes, 0});
    if (it == by_size_.end()) return false;
    const uint64_t size = it->first, at = it->second;
    erase(at, size);
    if (size > bytes) insert(at + bytes, size - bytes);
    *off = at;
    return true;
  }
  void release(uint64_t off, uint64_t bytes) {
    bytes = (bytes + 255) & ~255ull;
    auto next = by_off_.lower_bound(off);
    if (next != by_off_.end() && off + bytes == next->first) {
      const uint64_t n_at = next->first, n_size = next->second;
      erase(n_at, n_size);
      bytes += n_size;
    }
    auto prev = by_off_.lower_bound(off);
    if (prev != by_off_.begin()) {
      --prev;
      if (prev->first + prev->second == off) {
        const uint64_t p_at = prev->first, p_size = prev->second;
        erase(p_at, p_size);
        off = p_at;
        bytes += p_size;
      }
    }
    insert(off, bytes);
  }

 private:
  void insert(uint64_t at, uint64_t size) {
    if (!size) return;
    by_off_[at] = size;
    by_size_.insert({size, at});
  }
  void erase(uint64_t at, uint64_t size) {
    by_off_.erase(at);
    by_size_.erase({size, at});
  }
  std::map<uint64_t, uint64_t> by_off_;
  std::set<std::pair<uint64_t, uint64_t>> by_size_;
};

}  // namespace gx
