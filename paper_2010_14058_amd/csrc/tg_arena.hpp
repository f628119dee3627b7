// First-fit sub-allocator over a byte range [0, size) (host-side
// bookkeeping only; the range is a caller-owned device buffer).  Blocks are
// 256-byte aligned; a freed block merges with free neighbours.  Not thread
// safe: the serving loop holds its lock around every call.
#pragma once

#include <cstddef>
#include <cstdint>
#include <map>

namespace tg {

class Arena {
  public:
    static constexpr size_t ALIGN = 256;

    explicit Arena(size_t size = 0) { reset(size); }

    void reset(size_t size) {
        size_ = size & ~(ALIGN - 1);
        free_.clear();
        used_.clear();
        in_use_ = 0;
        if (size_) free_[0] = size_;
    }

    static size_t round(size_t bytes) { return (bytes + ALIGN - 1) & ~(ALIGN - 1); }

    // Offset of a new block of `bytes` (rounded up), or -1 if no free range
    // is large enough.
    int64_t alloc(size_t bytes) {
        const size_t need = round(bytes > 0 ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > need) free_[off + need] = len - need;
            used_[off] = need;
            in_use_ += need;
            return (int64_t)off;
        }
        return -1;
    }

    // Returns false if off is not the start of a live block.
    bool release(int64_t off) {
        auto it = used_.find((size_t)off);
        if (it == used_.end()) return false;
        size_t start = it->first, len = it->second;
        used_.erase(it);
        in_use_ -= len;
        auto next = free_.lower_bound(start);
        if (next != free_.end() && next->first == start + len) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                prev->second += len;
                return true;
            }
        }
        free_[start] = len;
        return true;
    }

    size_t size() const { return size_; }
    size_t in_use() const { return in_use_; }
    size_t largest_free() const {
        size_t b = 0;
        for (const auto &f : free_) b = f.second > b ? f.second : b;
        return b;
    }
    size_t free_ranges() const { return free_.size(); }
    size_t blocks() const { return used_.size(); }

  private:
    size_t size_ = 0, in_use_ = 0;
    std::map<size_t, size_t> free_;  // offset -> length, disjoint, never adjacent
    std::map<size_t, size_t> used_;  // offset -> length
};

}  // namespace tg
