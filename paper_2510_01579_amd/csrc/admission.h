// Admission bookkeeping of the serving loop, free of any device call so that it
// can be tested on its own: a first-fit allocator of byte ranges in the
// server's HBM arena, and the FIFO rule that decides how many queued jobs the
// next launch takes.
#pragma once

#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>
#include <vector>

namespace mmgap {
namespace serve {

constexpr size_t kArenaAlign = 256;

// Bytes a request of v bytes occupies in the arena (at least one 256-byte unit).
inline size_t arena_round(size_t v)
{
    if (v == 0) v = 1;
    return (v + kArenaAlign - 1) / kArenaAlign * kArenaAlign;
}

// First-fit allocator over [0, capacity): free ranges keyed by offset,
// coalesced with their neighbours on release.  Sizes are rounded up to 256
// bytes.  Not thread-safe (the server holds its lock).
class Arena {
public:
    explicit Arena(size_t capacity = 0) { reset(capacity); }

    void reset(size_t capacity)
    {
        cap_ = capacity / kArenaAlign * kArenaAlign;
        free_.clear();
        if (cap_) free_[0] = cap_;
        free_total_ = cap_;
    }

    // Takes `bytes` (rounded up); false if no free range is large enough.
    bool alloc(size_t bytes, size_t *off)
    {
        const size_t need = arena_round(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            *off = it->first;
            const size_t rest = it->second - need;
            const size_t at = it->first + need;
            free_.erase(it);
            if (rest) free_[at] = rest;
            free_total_ -= need;
            return true;
        }
        return false;
    }

    // Returns a range obtained from alloc() with the same `bytes`.
    void release(size_t off, size_t bytes)
    {
        const size_t size = arena_round(bytes);
        auto next = free_.lower_bound(off);
        size_t start = off, len = size;
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                start = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && off + size == next->first) {
            len += next->second;
            free_.erase(next);
        }
        free_[start] = len;
        free_total_ += size;
    }

    size_t capacity() const { return cap_; }
    size_t free_bytes() const { return free_total_; }
    size_t largest_free() const
    {
        size_t m = 0;
        for (const auto &r : free_) m = r.second > m ? r.second : m;
        return m;
    }
    size_t ranges() const { return free_.size(); }

private:
    std::map<size_t, size_t> free_;
    size_t cap_ = 0, free_total_ = 0;
};

// How many jobs at the head of the queue the next launch admits: the longest
// prefix (at most max_jobs) whose summed footprints fit in `room` bytes.  A
// head job that does not fit blocks everything behind it, so that jobs are
// started in arrival order and none starves.
inline int admit_prefix(const std::vector<size_t> &footprints, size_t room, int max_jobs)
{
    size_t used = 0;
    int k = 0;
    while (k < (int)footprints.size() && k < max_jobs) {
        const size_t f = arena_round(footprints[k]);
        if (used + f > room) break;
        used += f;
        ++k;
    }
    return k;
}

}  // namespace serve
}  // namespace mmgap
