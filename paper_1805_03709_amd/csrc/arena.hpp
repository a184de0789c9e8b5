// First-fit allocator of the serving arena's byte ranges (host code, plain C++): ranges
// are rounded up to 256 bytes, taken from the lowest-offset free range that fits, and
// freed ranges merge with free neighbours, so releasing everything leaves one range.
#pragma once
#include <cstdint>
#include <iterator>
#include <map>

namespace vbh {

struct Arena {
    std::map<int64_t, int64_t> free_;  // offset -> size
    void init(int64_t bytes) { free_ = {{0, bytes}}; }
    int64_t alloc(int64_t n) {
        n = (n + 255) & ~int64_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                const int64_t off = it->first, rest = it->second - n;
                free_.erase(it);
                if (rest) free_[off + n] = rest;
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t n) {
        n = (n + 255) & ~int64_t(255);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
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
};

}  // namespace vbh
