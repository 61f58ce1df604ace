// First-fit allocator of byte ranges within one device allocation, used by
// the server's arena (host only: it hands out offsets, the server adds the
// base address).  Ranges are rounded to ARENA_ALIGN; freed ranges merge with
// their free neighbours.
#pragma once
#include <algorithm>
#include <cstddef>
#include <iterator>
#include <map>

namespace ehs {

constexpr size_t ARENA_ALIGN = 1 << 16;

struct Arena {
    size_t cap = 0, used = 0, peak = 0;
    std::map<size_t, size_t> free_;  // offset -> bytes

    void init(size_t c)
    {
        cap = c / ARENA_ALIGN * ARENA_ALIGN;
        free_.clear();
        if (cap) free_[0] = cap;
        used = peak = 0;
    }
    static size_t round(size_t n) { return (n + ARENA_ALIGN - 1) / ARENA_ALIGN * ARENA_ALIGN; }
    bool alloc(size_t n, size_t* off)
    {
        n = round(std::max<size_t>(n, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            size_t rest = it->second - n, o2 = it->first + n;
            free_.erase(it);
            if (rest) free_[o2] = rest;
            used += n;
            peak = std::max(peak, used);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n)
    {
        n = round(std::max<size_t>(n, 1));
        used -= n;
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


}  // namespace ehs
