// Offset sub-allocator for one contiguous memory region (the device pool or
// the pinned host spill area).  Pure host bookkeeping: it hands out byte
// offsets, never touches the memory, and is unit-tested on the CPU.
//
// The paper reserves a large part of device memory at start up and lets a
// cache manage it (section 4.1, Figure 2).  Here that region is carved up
// first-fit with 256-byte granularity; freed blocks coalesce with their
// neighbours.  A movable upper limit (<= capacity) lets a caller shrink the
// usable part of the region at run time.
#pragma once

#include <cstddef>
#include <cstdint>
#include <map>

namespace qdpmi {

class OffsetPool {
public:
    static constexpr size_t kAlign = 256;

    void reset(size_t capacity) {
        capacity_ = capacity & ~(kAlign - 1);
        limit_ = capacity_;
        free_.clear();
        used_.clear();
        used_bytes_ = 0;
        high_water_ = 0;
        if (capacity_) free_[0] = capacity_;
    }

    size_t capacity() const { return capacity_; }
    size_t limit() const { return limit_; }
    size_t used_bytes() const { return used_bytes_; }
    size_t high_water() const { return high_water_; }
    size_t n_blocks() const { return used_.size(); }

    static size_t round_up(size_t n) { return (n + kAlign - 1) & ~(kAlign - 1); }

    // First fit below the limit.  Returns false if no free block fits.
    bool alloc(size_t bytes, size_t* off) {
        const size_t need = round_up(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            const size_t start = it->first, size = it->second;
            if (start + need > limit_) break;  // blocks are ordered by offset
            if (size < need) continue;
            free_.erase(it);
            if (size > need) free_[start + need] = size - need;
            used_[start] = need;
            used_bytes_ += need;
            if (start + need > high_water_) high_water_ = start + need;
            *off = start;
            return true;
        }
        return false;
    }

    // Release a block previously returned by alloc.  Returns false for an
    // unknown offset (double free).
    bool release(size_t off) {
        auto it = used_.find(off);
        if (it == used_.end()) return false;
        size_t start = off, size = it->second;
        used_.erase(it);
        used_bytes_ -= size;
        auto next = free_.lower_bound(start);
        if (next != free_.end() && next->first == start + size) {
            size += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                size += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = size;
        return true;
    }

    // Size of a live block (0 if unknown).
    size_t block_size(size_t off) const {
        auto it = used_.find(off);
        return it == used_.end() ? 0 : it->second;
    }

    void set_limit(size_t limit) { limit_ = limit > capacity_ ? capacity_ : (limit & ~(kAlign - 1)); }

    // Largest free block that lies wholly below the limit.
    size_t largest_free() const {
        size_t best = 0;
        for (const auto& kv : free_) {
            if (kv.first >= limit_) break;
            size_t end = kv.first + kv.second;
            if (end > limit_) end = limit_;
            if (end - kv.first > best) best = end - kv.first;
        }
        return best;
    }

    // Consistency check used by the tests: blocks tile the region exactly.
    bool check() const {
        size_t pos = 0, used = 0;
        auto f = free_.begin();
        auto u = used_.begin();
        while (f != free_.end() || u != used_.end()) {
            if (f != free_.end() && f->first == pos) {
                pos += f->second;
                ++f;
                if (f != free_.end() && f->first == pos) return false;  // not coalesced
            } else if (u != used_.end() && u->first == pos) {
                pos += u->second;
                used += u->second;
                ++u;
            } else {
                return false;
            }
        }
        return pos == capacity_ && used == used_bytes_;
    }

private:
    size_t capacity_ = 0, limit_ = 0, used_bytes_ = 0, high_water_ = 0;
    std::map<size_t, size_t> free_;  // offset -> size
    std::map<size_t, size_t> used_;  // offset -> size
};

}  // namespace qdpmi
