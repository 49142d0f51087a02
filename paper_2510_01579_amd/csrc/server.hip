// Serving loop: a native thread that admits submitted jobs into an HBM arena
// in arrival order, launches each admitted group as one batch of the
// persistent fused kernels on one of several streams (batches overlap on the
// device) -- each batch's launches recorded as a HIP graph and replayed -- and
// observes their completion.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "admission.h"
#include "context.h"

using namespace mmgap::host;
using Clock = std::chrono::steady_clock;

namespace {

constexpr size_t kMaxPending = 4096;
constexpr int kMaxInflight = 8;
constexpr size_t kDefaultArena = size_t(1) << 30;

enum JobState { kPending = 0, kRunning = 1, kDone = 2 };

struct ServerJob {
    mmgap_job job{};
    std::vector<float> beta;        // the job's own copy of its schedule
    mmgap_cim_params cim{};         // and of its CIM-CAC constants
    size_t footprint = 0;           // device bytes of the job as a batch of its own
    hipEvent_t ready = nullptr;     // caller's stream at submission
    Clock::time_point t_submit, t_done;
    int state = kPending;
    int status = MMGAP_OK;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipStream_t capture = nullptr;  // records the batch's launches (never executes them)
    hipGraphExec_t exec = nullptr;  // the slot's executable graph, updated per batch
    uint64_t exec_mask = ~0ull;     // the launch sequence the executable graph records
    hipEvent_t done = nullptr;
    bool busy = false;
    size_t off = 0, bytes = 0;      // arena range of the running batch
    std::vector<unsigned long long> ids;
    void *staging = nullptr;        // pinned header image of the running batch
    size_t staging_bytes = 0;
};

}  // namespace

struct mmgap_server {
    mmgap_ctx *ctx = nullptr;
    mmgap_ctx sink;                 // error messages and device facts of the server thread
    int max_inflight = 1;
    int max_batch_jobs = 64;
    char *arena = nullptr;
    mmgap::serve::Arena alloc;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable wake;   // new work or stop, for the server thread
    std::condition_variable idle;   // a job completed, for drain
    std::deque<unsigned long long> pending;
    std::unordered_map<unsigned long long, ServerJob> jobs;
    unsigned long long next_id = 1;
    size_t unfinished = 0;          // submitted and not yet complete
    std::vector<double> latencies_us;   // completed jobs since start or the last reset
    bool stopping = false;
    std::thread thread;
};

namespace {

// Completion of the slot's batch (the slot must be busy).
void reap(mmgap_server *sv, Slot &sl, hipError_t result, Clock::time_point now)
{
    for (unsigned long long id : sl.ids) {
        auto it = sv->jobs.find(id);
        if (it == sv->jobs.end()) continue;
        ServerJob &j = it->second;
        j.state = kDone;
        j.t_done = now;
        j.status = result == hipSuccess ? MMGAP_OK : MMGAP_EDEVICE;
        sv->latencies_us.push_back(
            std::chrono::duration<double, std::micro>(j.t_done - j.t_submit).count());
        if (j.ready) {
            (void)hipEventDestroy(j.ready);
            j.ready = nullptr;
        }
        --sv->unfinished;
    }
    sl.ids.clear();
    sv->alloc.release(sl.off, sl.bytes);
    sl.busy = false;
}

// Records a batch's launches (the counter reset, the MMSE-SIC launches, the
// jobs with launches of their own, then one persistent kernel per class
// present) as a HIP graph and replays it on the slot's stream.  The slot keeps
// its executable graph and updates it in place from the new recording while
// the batch launches the same sequence of kernels (kernel arguments and grid
// sizes change from batch to batch, the topology does not), so a batch costs
// one update and one graph launch; otherwise it is instantiated anew.
hipError_t enqueue_graph(mmgap_server *sv, Slot &sl, const BatchLaunch &bl)
{
    // the launch sequence: classes present, MMSE-SIC launches, and each
    // own-launch job's kernels (route, kind, KT, q), hashed
    uint64_t mask = 0;
    for (int c = 0; c < mmgap::kFusedClasses; ++c)
        if (bl.count[c] > 0 && bl.blocks[c] > 0) mask |= 1ull << c;
    mask = mask * 1000003ull + bl.sic.size();
    for (const SepLaunch &x : bl.sep)
        mask = mask * 1000003ull + (uint64_t)((x.route * 2 + x.kind) * 256 + x.KT * 8 + x.q);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(sl.capture, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    const hipError_t el = batch_enqueue(bl, sv->ctx->accept_dev, sl.capture);
    e = hipStreamEndCapture(sl.capture, &graph);
    if (e == hipSuccess) e = el;
    if (e == hipSuccess && sl.exec && sl.exec_mask == mask) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        if (hipGraphExecUpdate(sl.exec, graph, &bad, &res) != hipSuccess ||
            res != hipGraphExecUpdateSuccess) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(sl.exec);
            sl.exec = nullptr;
        }
    } else if (sl.exec) {
        (void)hipGraphExecDestroy(sl.exec);
        sl.exec = nullptr;
    }
    if (e == hipSuccess && !sl.exec) {
        e = hipGraphInstantiate(&sl.exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) sl.exec = nullptr;
        sl.exec_mask = e == hipSuccess ? mask : ~0ull;
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (e == hipSuccess) e = hipGraphLaunch(sl.exec, sl.stream);
    return e;
}

// Launches the first k pending jobs as one batch on slot `si`.  Returns false
// (after completing the jobs with an error) if the batch could not be started.
bool launch(mmgap_server *sv, int si, int k, size_t bytes, size_t off)
{
    Slot &sl = sv->slots[si];
    std::vector<unsigned long long> ids(sv->pending.begin(), sv->pending.begin() + k);
    sv->pending.erase(sv->pending.begin(), sv->pending.begin() + k);
    std::vector<mmgap_job> batch;
    batch.reserve(k);
    for (unsigned long long id : ids) batch.push_back(sv->jobs[id].job);

    sl.busy = true;
    sl.off = off;
    sl.bytes = bytes;
    sl.ids = ids;
    for (unsigned long long id : ids) sv->jobs[id].state = kRunning;

    BatchLayout lay;
    hipError_t e = hipSuccess;
    int rc = batch_layout(&sv->sink, k, batch.data(), 0, &lay);
    if (rc == MMGAP_OK && lay.bytes > bytes) rc = MMGAP_ENOMEM;   // footprints bound it
    char *base = sv->arena + off;
    BatchLaunch bl;
    std::vector<unsigned char> image;
    if (rc == MMGAP_OK) rc = batch_launch_config(&sv->sink, lay, base, 0, &bl);
    if (rc == MMGAP_OK) {
        batch_bind(lay, base, image);
        if (image.size() > sl.staging_bytes) {
            if (sl.staging) (void)hipHostFree(sl.staging);
            sl.staging = nullptr;
            sl.staging_bytes = 0;
            e = hipHostMalloc(&sl.staging, image.size() * 2, hipHostMallocDefault);
            if (e == hipSuccess) sl.staging_bytes = image.size() * 2;
            else sl.staging = nullptr;
        }
    }
    if (rc == MMGAP_OK && e == hipSuccess) {
        std::memcpy(sl.staging, image.data(), image.size());
        for (unsigned long long id : ids) {
            const ServerJob &j = sv->jobs[id];
            if (j.ready && e == hipSuccess) e = hipStreamWaitEvent(sl.stream, j.ready, 0);
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(base, sl.staging, image.size(), hipMemcpyHostToDevice, sl.stream);
        if (e == hipSuccess) e = enqueue_graph(sv, sl, bl);
        if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
    }
    if (rc != MMGAP_OK || e != hipSuccess) {
        // nothing (or only part) was enqueued: wait for what was, then fail the jobs
        (void)hipStreamSynchronize(sl.stream);
        reap(sv, sl, hipErrorLaunchFailure, Clock::now());
        sv->idle.notify_all();
        return false;
    }
    return true;
}

void server_loop(mmgap_server *sv)
{
    (void)hipSetDevice(sv->ctx->device);
    std::unique_lock<std::mutex> lk(sv->mu);
    for (;;) {
        bool progressed = false;
        const Clock::time_point now = Clock::now();
        for (Slot &sl : sv->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            reap(sv, sl, q, now);
            progressed = true;
        }
        if (progressed) sv->idle.notify_all();
        // admit: per free slot the longest FIFO prefix that fits the largest
        // free range (admission.h)
        if (!sv->pending.empty()) {
            std::vector<bool> busy;
            for (const Slot &sl : sv->slots) busy.push_back(sl.busy);
            const size_t look = std::min(sv->pending.size(),
                                         (size_t)sv->max_batch_jobs * sv->slots.size());
            std::vector<size_t> queue;
            queue.reserve(look);
            for (size_t i = 0; i < look; ++i) queue.push_back(sv->jobs[sv->pending[i]].footprint);
            for (const mmgap::serve::Admitted &ad :
                 mmgap::serve::admit_round(busy, queue, sv->max_batch_jobs, sv->alloc)) {
                launch(sv, ad.slot, ad.jobs, ad.bytes, ad.off);   // takes the queue's head
                progressed = true;
            }
        }
        bool any_busy = false;
        for (const Slot &sl : sv->slots) any_busy = any_busy || sl.busy;
        if (sv->stopping && sv->pending.empty() && !any_busy) break;
        if (progressed) continue;
        if (!any_busy && sv->pending.empty()) {
            sv->wake.wait(lk);                      // idle: sleep until submit or stop
        } else {
            // batches in flight (or the head waits for memory): poll again at
            // once, letting submitters take the lock in between
            lk.unlock();
            std::this_thread::yield();
            lk.lock();
        }
    }
}

void server_free(mmgap_server *sv)
{
    for (Slot &sl : sv->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.exec) (void)hipGraphExecDestroy(sl.exec);
        if (sl.capture) (void)hipStreamDestroy(sl.capture);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.staging) (void)hipHostFree(sl.staging);
    }
    for (auto &kv : sv->jobs)
        if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
    if (sv->arena) {
        (void)hipFree(sv->arena);
        sv->ctx->plan_bytes -= sv->alloc.capacity();
    }
    delete sv;
}

}  // namespace

namespace mmgap {
namespace host {

void server_shutdown(mmgap_ctx *ctx)
{
    mmgap_server *sv = ctx->server;
    if (!sv) return;
    {
        std::lock_guard<std::mutex> g(sv->mu);
        sv->stopping = true;
    }
    sv->wake.notify_all();
    if (sv->thread.joinable()) sv->thread.join();
    ctx->server = nullptr;
    server_free(sv);
}

}  // namespace host
}  // namespace mmgap

extern "C" {

int mmgap_server_start(mmgap_ctx *ctx, int max_inflight, size_t arena_bytes, int max_batch_jobs)
{
    if (!ctx) return MMGAP_EINVAL;
    if (ctx->server) return fail(ctx, MMGAP_EBUSY, "a server is already running");
    if (max_inflight < 1 || max_inflight > kMaxInflight)
        return fail(ctx, MMGAP_EINVAL, "max_inflight=%d outside 1..%d", max_inflight, kMaxInflight);
    if (max_batch_jobs < 0) return fail(ctx, MMGAP_EINVAL, "max_batch_jobs=%d < 0", max_batch_jobs);
    size_t bytes = arena_bytes ? arena_bytes : kDefaultArena;
    bytes = mmgap::serve::arena_round(bytes);
    if (bytes + ctx->plan_bytes + ctx->scratch_bytes > ctx->budget)
        return fail(ctx, MMGAP_ENOMEM, "server arena of %zu bytes exceeds the HBM budget (%zu of %zu in use)",
                    bytes, ctx->plan_bytes + ctx->scratch_bytes, ctx->budget);
    DeviceGuard g(ctx->device);
    mmgap_server *sv = new (std::nothrow) mmgap_server();
    if (!sv) return fail(ctx, MMGAP_ENOMEM, "out of host memory");
    sv->ctx = ctx;
    sv->max_inflight = max_inflight;
    sv->max_batch_jobs = max_batch_jobs ? max_batch_jobs : 64;
    sv->sink.device = ctx->device;
    // device facts the batch helpers read, settled here so that the server
    // thread never writes the caller's context
    hipError_t e = hipDeviceGetAttribute(&sv->sink.cus, hipDeviceAttributeMultiprocessorCount,
                                         ctx->device);
    for (int c = 0; c < mmgap::kFusedClasses && e == hipSuccess; ++c)
        e = mmgap::fused_blocks_per_cu(c, &sv->sink.fused_per_cu[c]);
    if (e == hipSuccess) e = hipMalloc(&sv->arena, bytes);
    if (e != hipSuccess) {
        sv->arena = nullptr;
        server_free(sv);
        return hip_fail(ctx, e, "server setup");
    }
    sv->alloc.reset(bytes);
    ctx->plan_bytes += bytes;
    sv->slots.resize(max_inflight);
    for (Slot &sl : sv->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.capture, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        server_free(sv);
        return hip_fail(ctx, e, "server streams");
    }
    try {
        sv->thread = std::thread(server_loop, sv);
    } catch (...) {
        server_free(sv);
        return fail(ctx, MMGAP_ENOMEM, "cannot start the server thread");
    }
    ctx->server = sv;
    return MMGAP_OK;
}

int mmgap_server_submit(mmgap_ctx *ctx, const mmgap_job *job, void *stream,
                        unsigned long long *job_id)
{
    if (!ctx) return MMGAP_EINVAL;
    mmgap_server *sv = ctx->server;
    if (!sv) return fail(ctx, MMGAP_EINVAL, "no server is running");
    if (!job || !job_id) return fail(ctx, MMGAP_EINVAL, "job and job_id are required");
    BatchLayout lay;
    int rc = batch_layout(ctx, 1, job, 0, &lay);
    if (rc) return rc;
    if (mmgap::serve::arena_round(lay.bytes) > sv->alloc.capacity())
        return fail(ctx, MMGAP_ENOMEM, "job needs %zu bytes, the server arena holds %zu", lay.bytes,
                    sv->alloc.capacity());
    ServerJob j;
    j.job = *job;
    const bool cim = job->sched.dynamics == MMGAP_DYN_CIM;
    if (cim) j.cim = *job->sched.cim;
    else j.beta.assign(job->sched.beta2, job->sched.beta2 + job->sched.sweeps);
    j.job.sched.beta2 = nullptr;            // pointed at the copies once stored
    j.job.sched.cim = nullptr;
    j.footprint = lay.bytes;
    DeviceGuard g(ctx->device);
    hipError_t e = hipEventCreateWithFlags(&j.ready, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(j.ready, (hipStream_t)stream);
    if (e != hipSuccess) {
        if (j.ready) (void)hipEventDestroy(j.ready);
        return hip_fail(ctx, e, "submit event");
    }
    unsigned long long id;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->pending.size() >= kMaxPending) {
            (void)hipEventDestroy(j.ready);
            return fail(ctx, MMGAP_EBUSY, "%zu jobs are waiting", sv->pending.size());
        }
        id = sv->next_id++;
        j.t_submit = Clock::now();
        ServerJob &stored = sv->jobs[id];
        stored = std::move(j);
        stored.job.sched.beta2 = cim ? nullptr : stored.beta.data();
        stored.job.sched.cim = cim ? &stored.cim : nullptr;
        sv->pending.push_back(id);
        ++sv->unfinished;
    }
    sv->wake.notify_all();
    *job_id = id;
    return MMGAP_OK;
}

int mmgap_server_poll(mmgap_ctx *ctx, unsigned long long job_id, int *done, double *latency_us)
{
    if (!ctx) return MMGAP_EINVAL;
    mmgap_server *sv = ctx->server;
    if (!sv) return fail(ctx, MMGAP_EINVAL, "no server is running");
    if (!done) return fail(ctx, MMGAP_EINVAL, "done is NULL");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(job_id);
    if (it == sv->jobs.end()) return fail(ctx, MMGAP_EINVAL, "unknown job id %llu", job_id);
    const ServerJob &j = it->second;
    *done = j.state == kDone ? 1 : 0;
    if (!*done) return MMGAP_OK;
    if (latency_us)
        *latency_us = std::chrono::duration<double, std::micro>(j.t_done - j.t_submit).count();
    const int status = j.status;
    sv->jobs.erase(it);
    if (status != MMGAP_OK) return fail(ctx, status, "job %llu: its batch failed on the device", job_id);
    return MMGAP_OK;
}

int mmgap_server_stats(mmgap_ctx *ctx, double deadline_us, int reset, mmgap_server_stats_t *out)
{
    if (!ctx) return MMGAP_EINVAL;
    mmgap_server *sv = ctx->server;
    if (!sv) return fail(ctx, MMGAP_EINVAL, "no server is running");
    if (!out) return fail(ctx, MMGAP_EINVAL, "out is NULL");
    if (!(deadline_us >= 0.0)) return fail(ctx, MMGAP_EINVAL, "deadline_us must be >= 0");
    std::lock_guard<std::mutex> lk(sv->mu);
    const mmgap::serve::LatencyStats s = mmgap::serve::latency_stats(sv->latencies_us, deadline_us);
    out->completed = (unsigned long long)s.count;
    out->missed = (unsigned long long)s.missed;
    out->p50_us = s.p50;
    out->p99_us = s.p99;
    out->max_us = s.max;
    if (reset) sv->latencies_us.clear();
    return MMGAP_OK;
}

int mmgap_server_drain(mmgap_ctx *ctx)
{
    if (!ctx) return MMGAP_EINVAL;
    mmgap_server *sv = ctx->server;
    if (!sv) return fail(ctx, MMGAP_EINVAL, "no server is running");
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->idle.wait(lk, [sv] { return sv->unfinished == 0; });
    return MMGAP_OK;
}

int mmgap_server_stop(mmgap_ctx *ctx)
{
    if (!ctx) return MMGAP_EINVAL;
    if (!ctx->server) return MMGAP_OK;
    DeviceGuard g(ctx->device);
    server_shutdown(ctx);
    return MMGAP_OK;
}

}  // extern "C"
