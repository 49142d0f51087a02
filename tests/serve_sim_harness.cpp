// The serving loop's admission round and latency accounting (admission.h)
// driven by a simulated device, for tests/test_serve_sim_cpu.py: batches
// complete after a modelled duration (the sum of their jobs' durations) on a
// simulated clock.  Input on stdin:
//   slots S cap C maxjobs M deadline D
//   job ARRIVAL FOOTPRINT DURATION      (one line per job, times in us)
//   end
// Output: one line per job in input order, "refused" (it could never fit the
// arena, as submission refuses it) or "START END SLOT", then
// "stats COUNT MISSED P50 P99 MAX".
#include <cstdint>
#include <iostream>
#include <sstream>
#include <string>
#include <vector>

#include "admission.h"

struct SimJob {
    int64_t arrival, footprint, duration;
    int64_t start = -1, end = -1;
    int slot = -1;
    bool refused = false;
};

int main()
{
    std::string word;
    int slots = 0, maxjobs = 0;
    size_t cap = 0;
    double deadline = 0;
    std::cin >> word >> slots >> word >> cap >> word >> maxjobs >> word >> deadline;
    std::vector<SimJob> jobs;
    while (std::cin >> word && word == "job") {
        SimJob j{};
        std::cin >> j.arrival >> j.footprint >> j.duration;
        jobs.push_back(j);
    }
    mmgap::serve::Arena arena(cap);
    struct Batch {
        bool busy = false;
        int64_t end = 0;
        size_t off = 0, bytes = 0;
        std::vector<int> ids;
    };
    std::vector<Batch> sl(slots);
    std::vector<int> queue;                 // waiting job indices, arrival order
    std::vector<double> lat;
    size_t next = 0;
    int64_t now = 0;
    for (;;) {
        // 1. completions observed at `now`, slot order
        for (Batch &b : sl) {
            if (!b.busy || b.end > now) continue;
            for (int id : b.ids) lat.push_back((double)(b.end - jobs[id].arrival));
            arena.release(b.off, b.bytes);
            b.busy = false;
            b.ids.clear();
        }
        // 2. arrivals up to `now`; a job that could never fit is refused
        while (next < jobs.size() && jobs[next].arrival <= now) {
            SimJob &j = jobs[next];
            if (mmgap::serve::arena_round((size_t)j.footprint) > arena.capacity()) j.refused = true;
            else queue.push_back((int)next);
            ++next;
        }
        // 3. one admission round
        std::vector<bool> busy;
        for (const Batch &b : sl) busy.push_back(b.busy);
        std::vector<size_t> fp;
        for (int id : queue) fp.push_back((size_t)jobs[id].footprint);
        size_t taken = 0;
        for (const mmgap::serve::Admitted &ad : mmgap::serve::admit_round(busy, fp, maxjobs, arena)) {
            Batch &b = sl[ad.slot];
            b.busy = true;
            b.off = ad.off;
            b.bytes = ad.bytes;
            int64_t dur = 0;
            for (int i = 0; i < ad.jobs; ++i) {
                const int id = queue[taken + i];
                b.ids.push_back(id);
                jobs[id].start = now;
                jobs[id].slot = ad.slot;
                dur += jobs[id].duration;
            }
            b.end = now + dur;
            for (int id : b.ids) jobs[id].end = b.end;
            taken += ad.jobs;
        }
        queue.erase(queue.begin(), queue.begin() + taken);
        // 4. the next event: an arrival or a completion
        int64_t t = INT64_MAX;
        if (next < jobs.size()) t = jobs[next].arrival;
        for (const Batch &b : sl)
            if (b.busy && b.end < t) t = b.end;
        if (t == INT64_MAX) break;          // nothing running, nothing to come
        now = t > now ? t : now;
    }
    for (const SimJob &j : jobs) {
        if (j.refused) std::cout << "refused\n";
        else std::cout << j.start << " " << j.end << " " << j.slot << "\n";
    }
    const mmgap::serve::LatencyStats s = mmgap::serve::latency_stats(lat, deadline);
    std::cout << "stats " << s.count << " " << s.missed << " " << (int64_t)s.p50 << " "
              << (int64_t)s.p99 << " " << (int64_t)s.max << "\n";
    return 0;
}
