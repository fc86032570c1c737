// arena.h -- host bookkeeping of the serving runtime's device memory budget
// (plain C++: no device code, so it can be checked on the CPU alone).
#pragma once

#include <algorithm>
#include <cstdint>
#include <iterator>
#include <map>

namespace obg {

// Budgeted device arena: one allocation carved best-fit into blocks of 256-B
// multiples; freed blocks coalesce with their free neighbours, so any request
// that fits the free total of a quiet arena is served.
struct Arena {
    uint8_t *base = nullptr;
    uint64_t size = 0, in_use = 0, peak = 0;
    std::map<uint64_t, uint64_t> free_;   // offset -> bytes; no two adjacent

    static uint64_t round(uint64_t b) { return (b + 255) & ~uint64_t(255); }
    void init(uint8_t *p, uint64_t bytes) {
        base = p;
        size = bytes & ~uint64_t(255);
        free_.clear();
        free_[0] = size;
    }
    uint8_t *get(uint64_t bytes) {
        bytes = round(bytes);
        auto best = free_.end();
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes && (best == free_.end() || it->second < best->second)) best = it;
        if (best == free_.end()) return nullptr;
        const uint64_t off = best->first, len = best->second;
        free_.erase(best);
        if (len > bytes) free_[off + bytes] = len - bytes;
        in_use += bytes;
        peak = std::max(peak, in_use);
        return base + off;
    }
    void put(uint8_t *p, uint64_t bytes) {
        bytes = round(bytes);
        in_use -= bytes;
        uint64_t off = (uint64_t)(p - base);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    uint64_t largest() const {
        uint64_t m = 0;
        for (auto &f : free_) m = std::max(m, f.second);
        return m;
    }
};

}  // namespace obg
