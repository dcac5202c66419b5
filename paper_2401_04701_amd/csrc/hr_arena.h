// First-fit allocator of granules inside one arena (host code, no device
// calls): the serving loop places each admitted job's shadow words with it.
#pragma once
#include <stdint.h>

#include <iterator>
#include <map>

// Free ranges are kept as offset -> length (in granules), merged with their
// neighbours when released, so a free range is never adjacent to another.
struct arena_alloc {
    std::map<uint64_t, uint64_t> free_;   // offset -> length, in granules
    explicit arena_alloc(uint64_t granules) { free_[0] = granules; }
    bool alloc(uint64_t n, uint64_t* off)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            *off = it->first;
            const uint64_t rest = it->second - n;
            const uint64_t at = it->first + n;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t n)
    {
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
