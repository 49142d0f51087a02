// Internal to the library: the context object and the host-side helpers shared
// by the C ABI entry points (capi.hip) and the serving loop (server.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "kernels.h"
#include "mmgap.h"

struct mmgap_server;

namespace mmgap {
namespace host {

constexpr int kRing = 8;                        // schedule upload slots
constexpr size_t kDefaultBudget = size_t(16) << 30;
constexpr size_t kAlign = 256;
constexpr int kProfRing = 256;                  // profiled calls kept
constexpr int kMaxFusedChains = 256;            // four wavefronts of a workgroup

}  // namespace host
}  // namespace mmgap

struct mmgap_ctx {
    int device = 0;
    size_t budget = mmgap::host::kDefaultBudget;
    std::string err;
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    char *noalloc_scratch = nullptr;            // this device's fixed array (capi.hip)
    size_t plan_bytes = 0;                      // device memory held by live plans and the server
    float *beta_dev = nullptr;                  // [kRing][kMaxSweeps]
    float *beta_host = nullptr;                 // pinned, same shape
    hipEvent_t ring_ev[mmgap::host::kRing] = {};
    int ring_pos = 0;
    hipEvent_t done = nullptr;                  // end of the last call's work
    hipStream_t aux = nullptr;                  // second stream (MMGaP-E's MMSE-SIC chain)
    hipEvent_t aux_ev[3] = {};                  // forks and the join of that stream
    bool done_valid = false;
    uint32_t *accept_dev = nullptr;             // Metropolis threshold table
    bool stage_launches = false;                // MMGAP_OPT_STAGE_LAUNCHES
    bool profiling = false;
    long prof_count = 0;                        // profiled calls since enabling
    bool prof_open = false;                     // the current record has its start event
    hipEvent_t prof_ev[mmgap::host::kProfRing][4] = {};   // start, before/after anneal, end
    int cus = 0;                                // compute units of the device
    int fused_per_cu[mmgap::kFusedClasses] = {};   // resident workgroups per CU, per class
    mmgap_server *server = nullptr;
};

namespace mmgap {
namespace host {

// Records a message for the context (or for mmgap_create when ctx is NULL)
// and returns `code`.
int fail(mmgap_ctx *ctx, int code, const char *fmt, ...);
int hip_fail(mmgap_ctx *ctx, hipError_t e, const char *what);

// Switches to a device for the lifetime of the guard.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Bump allocator of byte offsets, 256-byte aligned.
struct Bump {
    size_t off = 0;
    size_t take(size_t bytes)
    {
        const size_t o = off;
        off += align_up(bytes);
        return o;
    }
};

struct ProblemShape {
    int K = 0, q = 0, KT = 0, n_inst = 0;
};

int check_problem(mmgap_ctx *ctx, const mmgap_problem *p, int kind, ProblemShape *sh);
int check_schedule(mmgap_ctx *ctx, const mmgap_schedule *s);

// How a batch job runs: through the persistent kernels' work items; or, with
// launches of its own inside the batch, by CIM-CAC anneals (build, anneal,
// selection), by the one-launch search (build, the MMSE-SIC guess where
// asked, search), or by the plain path's Metropolis anneals for problems wider
// than the persistent kernels' 32 dimensions (build, anneal, selection).
enum BatchRoute { kRoutePersistent = 0, kRouteCim = 1, kRouteSearch = 2, kRoutePlain = 3 };

// A batch of jobs for the persistent fused kernels, laid out on the host:
// descriptors, work items grouped by register class (each group by decreasing
// cost), and byte offsets of one device block holding
//   [ descriptors | items | class counters | schedules ]   (the header, uploaded)
//   [ per job: fields | move fields (detection around a guess) | fallbacks ]
//   (scratch; the couplings, H and the VPP inverse of a work item live in LDS only)
struct BatchLayout {
    std::vector<FusedJob> jobs;
    std::vector<FusedItem> items;
    std::vector<std::vector<float>> betas;
    std::vector<size_t> of, ofp, ox, oxs, ob;
    std::vector<int> route;             // BatchRoute per job
    std::vector<CimParams> cim;         // CIM-CAC constants of kRouteCim jobs
    std::vector<int> search_lanes;      // kRouteSearch: lanes per instance
    std::vector<size_t> oG, oE, oS, oA; // own-launch routes: couplings [n_sc][KT][KT], chain
                                        // energies and spin words (CIM), VPP inverse
    size_t o_jobs = 0, o_items = 0, o_counters = 0;
    size_t header_bytes = 0;
    size_t bytes = 0;
    int cls_first[kFusedClasses] = {};
    int cls_items[kFusedClasses] = {};
};

// Validates the jobs and lays them out (no device work).  flags: mmgap_plan
// flags (MMGAP_PLAN_PERSISTENT keeps Metropolis jobs on the persistent kernels).
int batch_layout(mmgap_ctx *ctx, int n_jobs, const mmgap_job *jobs, int flags,
                 BatchLayout *out);
// Points the descriptors at a device block of out->bytes bytes and writes the
// header image (header_bytes) that must be copied to its start.
void batch_bind(BatchLayout &lay, char *dev_base, std::vector<unsigned char> &image);

// One launch of a bound batch: counter reset, then one persistent kernel per
// class present, largest class first.
struct SepLaunch {                  // the launches of one own-launch job
    int route = 0, kind = 0, KT = 0, q = 0;
    DetBuildArgs det{};
    VppBuildArgs vpp{};
    AnnealArgs ann{};
    SelectArgs sel{};
    SearchArgs srch{};
};
struct BatchLaunch {
    std::vector<SicArgs> sic;       // MMSE-SIC launches of jobs with that guess
    std::vector<SepLaunch> sep;     // jobs with launches of their own, after the MMSE-SIC ones
    FusedJob *jobs = nullptr;
    FusedItem *items = nullptr;
    unsigned int *counters = nullptr;
    int first[kFusedClasses] = {};
    int count[kFusedClasses] = {};
    int blocks[kFusedClasses] = {};
};
int batch_launch_config(mmgap_ctx *ctx, const BatchLayout &lay, char *dev_base, int blocks,
                        BatchLaunch *out);
hipError_t batch_enqueue(const BatchLaunch &b, const uint32_t *accept_table, hipStream_t st);

// Server teardown, called by mmgap_destroy (server.hip).
void server_shutdown(mmgap_ctx *ctx);

}  // namespace host
}  // namespace mmgap
