// Admission bookkeeping of the serving loop, free of any device call so that it
// can be tested on its own (against a simulated device on the host): a
// first-fit allocator of byte ranges in the server's HBM arena, the FIFO rule
// that decides how many queued jobs the next launch takes, one admission round
// over the in-flight slots, and the latency accounting against a deadline.
#pragma once

#include <algorithm>
#include <cmath>
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

// One admission round of the serving loop.  busy: the in-flight slots;
// queue: the footprints of the waiting jobs in arrival order.  Each free slot,
// in index order, takes the longest prefix of what is still queued (at most
// max_batch_jobs jobs) that fits the arena's largest free range, as one range
// taken first-fit; the round ends at the first free slot whose head job does
// not fit (the head waits for memory, and nothing behind it passes it).
struct Admitted {
    int slot;           // in-flight slot that launches the batch
    int jobs;           // the next `jobs` queued jobs, in order
    size_t off, bytes;  // the batch's arena range
};
inline std::vector<Admitted> admit_round(const std::vector<bool> &busy,
                                         const std::vector<size_t> &queue, int max_batch_jobs,
                                         Arena &arena)
{
    std::vector<Admitted> out;
    size_t head = 0;
    for (int si = 0; si < (int)busy.size() && head < queue.size(); ++si) {
        if (busy[si]) continue;
        const int look = (int)std::min<size_t>(queue.size() - head, (size_t)max_batch_jobs);
        const std::vector<size_t> fp(queue.begin() + head, queue.begin() + head + look);
        const int k = admit_prefix(fp, arena.largest_free(), look);
        if (k == 0) break;
        size_t bytes = 0;
        for (int i = 0; i < k; ++i) bytes += arena_round(fp[i]);
        size_t off = 0;
        if (!arena.alloc(bytes, &off)) break;
        out.push_back(Admitted{si, k, off, bytes});
        head += k;
    }
    return out;
}

// Completed jobs' latencies against a deadline: how many, how many strictly
// above the deadline, and the nearest-rank 50th and 99th percentiles (the
// smallest latency with at least that share of the jobs at or below it).
struct LatencyStats {
    size_t count = 0, missed = 0;
    double p50 = 0.0, p99 = 0.0, max = 0.0;
};
inline LatencyStats latency_stats(std::vector<double> lat, double deadline)
{
    LatencyStats s;
    s.count = lat.size();
    if (lat.empty()) return s;
    std::sort(lat.begin(), lat.end());
    for (double v : lat) s.missed += v > deadline ? 1 : 0;
    auto rank = [&](double pct) {
        size_t r = (size_t)std::ceil(pct / 100.0 * (double)lat.size());
        if (r < 1) r = 1;
        return lat[r - 1];
    };
    s.p50 = rank(50.0);
    s.p99 = rank(99.0);
    s.max = lat.back();
    return s;
}

}  // namespace serve
}  // namespace mmgap
