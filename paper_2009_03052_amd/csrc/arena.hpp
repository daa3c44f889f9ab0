// First-fit allocator of byte ranges inside one pre-allocated device arena
// (the server's output budget). Host code only: it hands out offsets, never
// touches the memory, and keeps free ranges coalesced.
#pragma once

#include <algorithm>
#include <cstdint>
#include <iterator>
#include <map>

// byte offsets in 256-byte granules
class Arena {
    std::map<int64_t, int64_t> free_;   // offset -> size
    int64_t used_ = 0, peak_ = 0;

  public:
    static int64_t round(int64_t b) { return (b + 255) & ~(int64_t)255; }
    void reset(int64_t cap)
    {
        free_.clear();
        if (cap > 0) free_[0] = cap;
        used_ = peak_ = 0;
    }
    int64_t alloc(int64_t bytes)
    {
        bytes = round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            const int64_t off = it->first, rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return off;
        }
        return -1;
    }
    void release(int64_t off, int64_t bytes)
    {
        bytes = round(bytes);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
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
    int64_t used() const { return used_; }
    int64_t peak() const { return peak_; }
};

