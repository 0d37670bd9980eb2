// First-fit allocator over the byte range [0, size) with coalescing on free:
// the server's device arena (the request admission of the serving path hands
// out ranges of one allocation of exactly the memory budget).  Plain C++, no
// device code, so that host tests can build it on its own.
#pragma once

#include <cstddef>
#include <iterator>
#include <list>
#include <utility>

namespace tsqbx {

class Arena {
 public:
  void init(size_t size) {
    free_.clear();
    if (size) free_.push_back({0, size});
  }
  // The first free range of at least n bytes: *off receives its start and
  // the range shrinks from the front.  False (and *off untouched) if none.
  bool alloc(size_t n, size_t *off) {
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= n) {
        *off = it->first;
        it->first += n;
        it->second -= n;
        if (it->second == 0) free_.erase(it);
        return true;
      }
    return false;
  }
  // Return [off, off + n), merging it with free neighbours.  The range must
  // have come from alloc and not been returned since.
  void release(size_t off, size_t n) {
    if (n == 0) return;
    auto it = free_.begin();
    while (it != free_.end() && it->first < off) ++it;
    it = free_.insert(it, {off, n});
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
        it = pv;
      }
    }
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
  }
  size_t free_bytes() const {
    size_t b = 0;
    for (auto &r : free_) b += r.second;
    return b;
  }
  size_t free_ranges() const { return free_.size(); }

 private:
  std::list<std::pair<size_t, size_t>> free_;  // (offset, length), sorted by offset
};

}  // namespace tsqbx
