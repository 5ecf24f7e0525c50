// First-fit sub-allocator over one contiguous device region (host bookkeeping only).
//
// The serving loop reserves its whole HBM budget once and carves request buffers
// out of it, so admission never calls hipMalloc and the budget is enforced by
// construction.  Offsets are aligned to `align` bytes; freed ranges coalesce with
// their neighbours.  Not thread-safe: the caller serialises access.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <limits>
#include <map>

namespace slsht {

class Arena {
public:
    static constexpr size_t kFail = std::numeric_limits<size_t>::max();

    explicit Arena(size_t capacity = 0, size_t align = 256) { reset(capacity, align); }

    void reset(size_t capacity, size_t align = 256) {
        align_ = align ? align : 1;
        cap_ = capacity / align_ * align_;
        used_ = 0;
        free_.clear();
        live_.clear();
        if (cap_) free_[0] = cap_;
    }

    size_t round(size_t n) const {
        if (n == 0) n = 1;
        if (n > std::numeric_limits<size_t>::max() - (align_ - 1)) return kFail;
        return (n + align_ - 1) / align_ * align_;
    }

    // Offset of a new block of n bytes, or kFail if no free range is large enough.
    size_t alloc(size_t n) {
        const size_t need = round(n);
        if (need == kFail) return kFail;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            const size_t off = it->first, rest = it->second - need;
            free_.erase(it);
            if (rest) free_[off + need] = rest;
            live_[off] = need;
            used_ += need;
            return off;
        }
        return kFail;
    }

    // Returns false for an offset that is not a live block.
    bool release(size_t off) {
        auto it = live_.find(off);
        if (it == live_.end()) return false;
        size_t start = off, len = it->second;
        used_ -= len;
        live_.erase(it);
        auto nx = free_.lower_bound(start);
        if (nx != free_.end() && start + len == nx->first) {
            len += nx->second;
            nx = free_.erase(nx);
        }
        if (nx != free_.begin()) {
            auto pv = std::prev(nx);
            if (pv->first + pv->second == start) {
                start = pv->first;
                len += pv->second;
                free_.erase(pv);
            }
        }
        free_[start] = len;
        return true;
    }

    size_t capacity() const { return cap_; }
    size_t used() const { return used_; }
    size_t live_blocks() const { return live_.size(); }
    size_t free_ranges() const { return free_.size(); }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto& kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }

private:
    size_t align_ = 256, cap_ = 0, used_ = 0;
    std::map<size_t, size_t> free_;   // offset -> length of free ranges
    std::map<size_t, size_t> live_;   // offset -> length of allocated blocks
};

}  // namespace slsht
