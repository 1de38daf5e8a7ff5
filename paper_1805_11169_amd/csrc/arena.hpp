// First-fit allocator over one caller-owned device range (the serving arena).
// Host-only bookkeeping: offsets into the range, never dereferenced here.
// Blocks are 256-byte aligned (the workspace alignment icwf_create needs);
// freeing coalesces with both neighbours, so a stream of uneven simulations
// does not fragment the range beyond what their live footprints require.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>

namespace icwf {

class Arena {
public:
    static constexpr size_t kAlign = 256;
    static constexpr size_t kFail = ~size_t(0);

    explicit Arena(size_t bytes) : size_(bytes / kAlign * kAlign) {
        if (size_) free_[0] = size_;
    }

    static size_t round_up(size_t n) { return (n + kAlign - 1) / kAlign * kAlign; }

    // Offset of a block of at least n bytes, or kFail.
    size_t alloc(size_t n) {
        if (n == 0) return kFail;
        n = round_up(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t off = it->first, len = it->second;
            free_.erase(it);
            if (len > n) free_[off + n] = len - n;
            used_[off] = n;
            in_use_ += n;
            if (in_use_ > peak_) peak_ = in_use_;
            return off;
        }
        return kFail;
    }

    // Release a block returned by alloc; false if off is not a live block.
    bool release(size_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return false;
        size_t len = u->second;
        used_.erase(u);
        in_use_ -= len;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + len == next->first) {
            len += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += len;
                return true;
            }
        }
        free_[off] = len;
        return true;
    }

    size_t size() const { return size_; }
    size_t in_use() const { return in_use_; }
    size_t peak() const { return peak_; }
    size_t largest_free() const {
        size_t m = 0;
        for (const auto &kv : free_)
            if (kv.second > m) m = kv.second;
        return m;
    }
    size_t free_blocks() const { return free_.size(); }
    size_t live_blocks() const { return used_.size(); }

private:
    size_t size_;
    size_t in_use_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;   // offset -> length, disjoint, never adjacent
    std::map<size_t, size_t> used_;   // offset -> length
};

}  // namespace icwf
