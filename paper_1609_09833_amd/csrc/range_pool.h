// Free-range bookkeeping of the serving loop's walker pool (host code, no
// device calls): a pool of `size` atom slots handed out as contiguous ranges.
// Best fit in O(log n): the shortest free range that holds the request
// (lowest offset among equals); freed ranges merge with free neighbours, so
// no two free ranges ever touch.
#pragma once

#include <cstdint>
#include <iterator>
#include <limits>
#include <map>
#include <set>
#include <utility>

namespace abp {

class RangePool {
 public:
  // Everything free again.
  void reset(int64_t size) {
    by_off_.clear();
    by_len_.clear();
    if (size > 0) insert(0, size);
  }

  // A range of n > 0 slots; false when no free range is long enough.
  bool alloc(int64_t n, int64_t* off) {
    auto b = by_len_.lower_bound({n, std::numeric_limits<int64_t>::min()});
    if (b == by_len_.end()) return false;
    const int64_t len = b->first, at = b->second;
    erase(by_off_.find(at));
    if (len > n) insert(at + n, len - n);
    *off = at;
    return true;
  }

  // Returns [off, off + n), which alloc handed out.
  void free(int64_t off, int64_t n) {
    auto nx = by_off_.lower_bound(off);
    if (nx != by_off_.end() && off + n == nx->first) {     // merge with the next range
      n += nx->second;
      auto after = std::next(nx);
      erase(nx);
      nx = after;
    }
    if (nx != by_off_.begin()) {                            // merge with the previous range
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        off = pv->first;
        n += pv->second;
        erase(pv);
      }
    }
    insert(off, n);
  }

  const std::map<int64_t, int64_t>& ranges() const { return by_off_; }   // offset -> length

 private:
  void insert(int64_t off, int64_t n) {
    by_off_.emplace(off, n);
    by_len_.emplace(n, off);
  }
  void erase(std::map<int64_t, int64_t>::iterator it) {
    by_len_.erase({it->second, it->first});
    by_off_.erase(it);
  }

  std::map<int64_t, int64_t> by_off_;              // offset -> length
  std::set<std::pair<int64_t, int64_t>> by_len_;   // (length, offset)
};

}  // namespace abp
