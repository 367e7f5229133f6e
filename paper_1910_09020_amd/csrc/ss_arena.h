// First-fit allocator of byte ranges (the device-resident serving loop's
// arena).  Pure host code; not thread-safe (the server guards it).
#pragma once
#include <cstddef>
#include <iterator>
#include <map>

// Offsets into an arena of `bytes` bytes; released ranges merge with free neighbours.
struct Arena {
    std::map<size_t, size_t> free_ranges;      // offset -> bytes
    void reset(size_t bytes)
    {
        free_ranges.clear();
        if (bytes) free_ranges[0] = bytes;
    }
    bool alloc(size_t bytes, size_t* off)
    {
        for (auto it = free_ranges.begin(); it != free_ranges.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t left = it->second - bytes, at = it->first + bytes;
            free_ranges.erase(it);
            if (left) free_ranges[at] = left;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        auto it = free_ranges.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_ranges.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_ranges.erase(nx);
        }
        if (it != free_ranges.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_ranges.erase(it);
            }
        }
    }
};

