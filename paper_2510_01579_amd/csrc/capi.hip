// C ABI of the Ising hot path: contexts, argument checks, scratch management
// and the launch sequences (build -> anneal -> select) of include/mmgap.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "context.h"

using namespace mmgap::host;

namespace {
thread_local std::string g_create_error;

// Scratch of mmgap_detect_noalloc: one fixed array per device, held until the
// process ends.  In host code the array's name is only a stand-in; the device
// address of each device's copy comes from hipGetSymbolAddress, taken once per
// device (with that device current) when a context is created there.
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mutex;
char *g_noalloc_ptr[kNoAllocDevices] = {};

// The current device's address of `scratch` (the device is `device`).
hipError_t noalloc_scratch_address(int device, char **out)
{
    *out = nullptr;
    if (device < 0 || device >= kNoAllocDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mutex);
    if (!g_noalloc_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_noalloc_ptr[device] = static_cast<char *>(p);
    }
    *out = g_noalloc_ptr[device];
    return hipSuccess;
}
}  // namespace

namespace mmgap {
namespace host {

int fail(mmgap_ctx *ctx, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    else g_create_error = buf;
    return code;
}

int hip_fail(mmgap_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, MMGAP_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace host
}  // namespace mmgap

namespace {

int ensure_scratch(mmgap_ctx *ctx, size_t bytes)
{
    if (bytes + ctx->plan_bytes > ctx->budget)
        return fail(ctx, MMGAP_ENOMEM,
                    "scratch of %zu bytes (+%zu held by plans) exceeds the HBM budget of %zu bytes",
                    bytes, ctx->plan_bytes, ctx->budget);
    if (bytes <= ctx->scratch_bytes) return MMGAP_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(ctx, e, "hipDeviceSynchronize");
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    ctx->scratch = nullptr;
    ctx->scratch_bytes = 0;
    size_t want = bytes + bytes / 4;
    if (want + ctx->plan_bytes > ctx->budget) want = bytes;
    e = hipMalloc(&ctx->scratch, want);
    if (e != hipSuccess) {
        ctx->scratch = nullptr;
        return fail(ctx, MMGAP_ENOMEM, "hipMalloc(%zu): %s", want, hipGetErrorString(e));
    }
    ctx->scratch_bytes = want;
    return MMGAP_OK;
}

template <typename T>
T *at(mmgap_ctx *ctx, size_t off)
{
    return reinterpret_cast<T *>(static_cast<char *>(ctx->scratch) + off);
}

bool pow2_weight(int w) { return w >= 1 && w <= 64 && (w & (w - 1)) == 0; }

int pow2_ceil(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Lanes per instance when several instances share a wavefront: chains rounded
// up to a power of two, at least 64 / max_per_wave; 0 (one instance per
// wavefront) when chains > 32 or when the instances of a wavefront would not
// share one G (64 / lanes must divide inst_per_G; 0 = no such constraint).
int packed_lanes(int chains, int inst_per_G, int max_per_wave)
{
    if (chains > 32) return 0;
    int per_wave = 64 / pow2_ceil(chains);
    if (per_wave > max_per_wave) per_wave = max_per_wave;
    while (inst_per_G > 0 && per_wave > 1 && inst_per_G % per_wave) per_wave >>= 1;
    return per_wave > 1 ? 64 / per_wave : 0;
}

// Lanes per instance of the one-launch search (k_search), or 0 when it cannot
// run the problem: Metropolis anneals, KT <= 32, chains <= 64, 64 / lanes
// instances of a subcarrier per wavefront (at most 16, so at least 4 lanes),
// n_rx <= 2 lanes.
int search_lanes_of(int chains, int n_sym, int n_rx, int KT, bool cim)
{
    if (cim || KT > 32 || chains > 64) return 0;
    int gl = 64;
    if (chains <= 32) {
        const int p = packed_lanes(chains, n_sym, 16);
        if (p) gl = p;
    }
    return n_rx <= 2 * gl ? gl : 0;
}

int qam_bits(int qam)
{
    switch (qam) {
    case 4: return 1;
    case 16: return 2;
    case 64: return 3;
    default: return 0;
    }
}


}  // namespace

namespace mmgap {
namespace host {

int check_schedule(mmgap_ctx *ctx, const mmgap_schedule *s)
{
    if (!s) return fail(ctx, MMGAP_EINVAL, "schedule is NULL");
    if (s->chains < 1 || s->chains > mmgap::kMaxChains)
        return fail(ctx, MMGAP_EUNSUPPORTED, "chains=%d outside 1..%d", s->chains, mmgap::kMaxChains);
    if (s->sweeps < 1 || s->sweeps > mmgap::kMaxSweeps)
        return fail(ctx, MMGAP_EUNSUPPORTED, "sweeps=%d outside 1..%d", s->sweeps, mmgap::kMaxSweeps);
    if (s->init != 0 && s->init != 1) return fail(ctx, MMGAP_EINVAL, "schedule.init must be 0 or 1");
    if (s->dynamics == MMGAP_DYN_CIM) {
        const mmgap_cim_params *c = s->cim;
        if (!c) return fail(ctx, MMGAP_EINVAL, "schedule.cim is NULL");
        const float v[6] = {c->dt, c->p, c->a, c->zeta, c->eps, c->amp0};
        for (float x : v)
            if (!std::isfinite(x)) return fail(ctx, MMGAP_EINVAL, "schedule.cim has a non-finite constant");
        if (!(c->dt > 0.0f)) return fail(ctx, MMGAP_EINVAL, "schedule.cim.dt must be > 0");
        if (c->f_mvm < 1) return fail(ctx, MMGAP_EINVAL, "schedule.cim.f_mvm must be >= 1");
        return MMGAP_OK;
    }
    if (s->dynamics != MMGAP_DYN_METROPOLIS)
        return fail(ctx, MMGAP_EINVAL, "schedule.dynamics=%d is not METROPOLIS or CIM", s->dynamics);
    if (!s->beta2) return fail(ctx, MMGAP_EINVAL, "schedule.beta2 is NULL");
    for (int t = 0; t < s->sweeps; ++t) {
        const float b = s->beta2[t];
        if (!(b >= 0.0f) || !std::isfinite(b))
            return fail(ctx, MMGAP_EINVAL, "schedule.beta2[%d]=%g is not finite and >= 0", t, (double)b);
    }
    return MMGAP_OK;
}

int check_problem(mmgap_ctx *ctx, const mmgap_problem *p, int kind, ProblemShape *sh)
{
    if (!p) return fail(ctx, MMGAP_EINVAL, "problem is NULL");
    if (p->kind != MMGAP_KIND_DET && p->kind != MMGAP_KIND_VPP)
        return fail(ctx, MMGAP_EINVAL, "problem.kind=%d is not DET or VPP", p->kind);
    if (kind >= 0 && p->kind != kind)
        return fail(ctx, MMGAP_EINVAL, "problem.kind=%d does not match this entry point", p->kind);
    if (p->n_rx < 1 || p->n_tx < 1 || p->n_sc < 0 || p->n_sym < 1)
        return fail(ctx, MMGAP_EINVAL, "bad sizes n_rx=%d n_tx=%d n_sc=%d n_sym=%d", p->n_rx,
                    p->n_tx, p->n_sc, p->n_sym);
    if (p->n_sym > 64) return fail(ctx, MMGAP_EUNSUPPORTED, "n_sym=%d > 64", p->n_sym);
    const int q = qam_bits(p->qam);
    if (!q) return fail(ctx, MMGAP_EUNSUPPORTED, "qam=%d not in {4,16,64}", p->qam);
    if (p->kind == MMGAP_KIND_DET) {
        if (p->n_tx > 32 || p->n_rx > 64)
            return fail(ctx, MMGAP_EUNSUPPORTED, "DET needs n_tx <= 32 and n_rx <= 64 (got %d x %d)",
                        p->n_rx, p->n_tx);
        if (p->n_tx > 16 && q > 2)
            return fail(ctx, MMGAP_EUNSUPPORTED,
                        "DET with more than 16 users supports QPSK and 16-QAM (got %d-QAM)",
                        p->qam);
        if (!(p->noise_var >= 0.0f) || !std::isfinite(p->noise_var))
            return fail(ctx, MMGAP_EINVAL, "noise_var must be finite and >= 0");
        sh->K = 2 * p->n_tx;
        sh->q = q;
    } else {
        if (p->n_rx > 16 || p->n_tx > 64)
            return fail(ctx, MMGAP_EUNSUPPORTED, "VPP needs n_rx <= 16 and n_tx <= 64 (got %d x %d)",
                        p->n_rx, p->n_tx);
        if (!std::isfinite(p->tau)) return fail(ctx, MMGAP_EINVAL, "tau must be finite");
        sh->K = 2 * p->n_rx;
        sh->q = 2;
    }
    sh->KT = mmgap::padded_k(sh->K);
    const long long ni = (long long)p->n_sc * p->n_sym;
    if (ni > 0x7FFFFFFFll) return fail(ctx, MMGAP_EUNSUPPORTED, "too many instances");
    sh->n_inst = (int)ni;
    return MMGAP_OK;
}

}  // namespace host
}  // namespace mmgap

namespace {

// Orders this call after the context's previous call (which may have used
// another stream) so that the shared scratch is never used concurrently.
int begin_call(mmgap_ctx *ctx, hipStream_t s)
{
    if (ctx->done_valid) {
        hipError_t e = hipStreamWaitEvent(s, ctx->done, 0);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamWaitEvent");
    }
    return MMGAP_OK;
}

int end_call(mmgap_ctx *ctx, hipStream_t s)
{
    hipError_t e = hipEventRecord(ctx->done, s);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventRecord");
    ctx->done_valid = true;
    return MMGAP_OK;
}

void prof_mark(mmgap_ctx *ctx, int i, hipStream_t s)
{
    if (!ctx->profiling) return;
    // a solver launch after the first of one call (stages, two guesses) opens
    // its own record: its start is its schedule upload
    if (i == 0) ctx->prof_open = true;
    else if (i == 1 && !ctx->prof_open) (void)hipEventRecord(ctx->prof_ev[ctx->prof_count % kProfRing][0], s);
    (void)hipEventRecord(ctx->prof_ev[ctx->prof_count % kProfRing][i], s);
}

// Copies the host schedule into a device ring slot; returns the device table.
int upload_beta(mmgap_ctx *ctx, const mmgap_schedule *s, hipStream_t st, const float **out)
{
    const int slot = ctx->ring_pos;
    ctx->ring_pos = (ctx->ring_pos + 1) % kRing;
    hipError_t e = hipEventSynchronize(ctx->ring_ev[slot]);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventSynchronize");
    float *h = ctx->beta_host + (size_t)slot * mmgap::kMaxSweeps;
    float *d = ctx->beta_dev + (size_t)slot * mmgap::kMaxSweeps;
    std::memcpy(h, s->beta2, sizeof(float) * (size_t)s->sweeps);
    e = hipMemcpyAsync(d, h, sizeof(float) * (size_t)s->sweeps, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMemcpyAsync(schedule)");
    e = hipEventRecord(ctx->ring_ev[slot], st);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventRecord(schedule)");
    *out = d;
    return MMGAP_OK;
}

double qam_c(int qam) { return 1.0 / std::sqrt(2.0 * (qam - 1) / 3.0); }
double qam_c2(int qam) { return 1.0 / (2.0 * (qam - 1) / 3.0); }
double vpp_tau(const mmgap_problem *p)
{
    if (p->tau > 0.0f) return (double)p->tau;
    return 2.0 * std::sqrt((double)p->qam) * qam_c(p->qam);
}

void det_weights(int q, int *w)
{
    for (int b = 0; b < mmgap::kMaxQ; ++b) w[b] = b < q ? 1 << (q - 1 - b) : 1;
}

void vpp_weights(int *w)
{
    w[0] = 1;
    w[1] = 1;
    w[2] = 1;
    w[3] = 1;
}

// Anneal + select over padded structures already on the device.
int run_solver(mmgap_ctx *ctx, hipStream_t st, int n_inst, int K, int q, int KT, const int *w,
               const float *Gp, int inst_per_G, const float *fp, const signed char *xp,
               const mmgap_schedule *sched, float *chainE, uint32_t *chainS,
               mmgap::SelectArgs sel)
{
    const bool cim = sched->dynamics == MMGAP_DYN_CIM;
    if (cim && (KT > 32 || KT * q > 64))
        return fail(ctx, MMGAP_EUNSUPPORTED,
                    "CIM dynamics needs K <= 32 and K q <= 64 spins (padded %d x %d)", KT, q);
    const float *beta = nullptr;
    if (!cim) {
        int rc = upload_beta(ctx, sched, st, &beta);
        if (rc) return rc;
    }
    mmgap::AnnealArgs a{};
    a.G = Gp;
    a.inst_per_G = inst_per_G;
    a.f = fp;
    a.x_fb = xp;
    a.beta2 = beta;
    a.accept_table = ctx->accept_dev;
    a.sweeps = sched->sweeps;
    a.chains = sched->chains;
    a.n_inst = n_inst;
    for (int b = 0; b < mmgap::kMaxQ; ++b) a.w[b] = w[b];
    a.key0 = (uint32_t)sched->seed;
    a.key1 = (uint32_t)(sched->seed >> 32);
    a.inst_base = sched->inst_base;
    a.init_mode = sched->init;
    a.glanes = packed_lanes(sched->chains, inst_per_G, 64);
    a.chain_E = chainE;
    a.chain_S = chainS;
    if (cim) {
        a.cim.dt = sched->cim->dt;
        a.cim.pm1 = sched->cim->p - 1.0f;        // rounded once in float32
        a.cim.a = sched->cim->a;
        a.cim.nzeta = -sched->cim->zeta;
        a.cim.eps = sched->cim->eps;
        a.cim.amp0 = sched->cim->amp0;
        a.cim.f_mvm = sched->cim->f_mvm;
    }
    prof_mark(ctx, 1, st);
    hipError_t e = cim ? mmgap::launch_cim(KT, q, a, st) : mmgap::launch_anneal(KT, q, a, st);
    if (e != hipSuccess) return hip_fail(ctx, e, cim ? "CIM anneal launch" : "anneal launch");
    prof_mark(ctx, 2, st);
    sel.n_inst = n_inst;
    sel.K = K;
    sel.KT = KT;
    sel.q = q;
    sel.chains = sched->chains;
    for (int b = 0; b < mmgap::kMaxQ; ++b) sel.w[b] = w[b];
    sel.G = Gp;
    sel.inst_per_G = inst_per_G;
    sel.f = fp;
    sel.x_fb = xp;
    sel.chain_E = chainE;
    sel.chain_S = chainS;
    e = mmgap::launch_select(sel, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "select launch");
    prof_mark(ctx, 3, st);
    if (ctx->profiling) {
        ++ctx->prof_count;
        ctx->prof_open = false;
    }
    return MMGAP_OK;
}

// Relative cost of one work item: the workgroup is held for `sweeps` sweeps of
// KT Q flip attempts, each about 20 operations plus the K-term field row shared
// by the Q attempts of a dimension, once per stage.
double item_cost(const mmgap::FusedJob &j)
{
    return (double)j.sweeps * j.KT * (20.0 * j.Q + j.KT) * (j.stages > 0 ? j.stages : 1) *
           (j.guesses == 3 ? 2 : 1);
}

}  // namespace

namespace mmgap {
namespace host {

int batch_layout(mmgap_ctx *ctx, int n_jobs, const mmgap_job *jobs, int flags,
                 BatchLayout *out)
{
    BatchLayout &L = *out;
    L = BatchLayout();
    L.jobs.resize((size_t)n_jobs);
    L.betas.resize((size_t)n_jobs);
    L.route.assign((size_t)n_jobs, kRoutePersistent);
    L.cim.resize((size_t)n_jobs);
    L.search_lanes.assign((size_t)n_jobs, 0);
    for (int j = 0; j < n_jobs; ++j) {
        const mmgap_job &jb = jobs[j];
        ProblemShape sh;
        int rc = check_problem(ctx, &jb.prob, -1, &sh);
        if (!rc) rc = check_schedule(ctx, &jb.sched);
        if (rc) return fail(ctx, rc, "job %d: %s", j, ctx->err.c_str());
        const bool cim = jb.sched.dynamics == MMGAP_DYN_CIM;
        if (sh.n_inst > 0 && (!jb.H || !jb.y_or_u || !jb.out0))
            return fail(ctx, MMGAP_EINVAL, "job %d: H, y_or_u and out0 are required", j);
        if (jb.stages < 0 || jb.stages > mmgap::kMaxStages)
            return fail(ctx, MMGAP_EUNSUPPORTED, "job %d: stages=%d outside 0..%d", j, jb.stages,
                        mmgap::kMaxStages);
        if (jb.stages > 0 && jb.prob.kind != MMGAP_KIND_DET)
            return fail(ctx, MMGAP_EUNSUPPORTED, "job %d: stages apply to detection only", j);
        if (jb.guesses < 0 || jb.guesses > (MMGAP_GUESS_MMSE | MMGAP_GUESS_SIC))
            return fail(ctx, MMGAP_EINVAL, "job %d: guesses=%d is not 0 or a set of MMGAP_GUESS_*",
                        j, jb.guesses);
        if (jb.guesses > 0 && jb.stages < 1)
            return fail(ctx, MMGAP_EINVAL, "job %d: guesses need stages >= 1", j);
        // moves around a guess: two unit-weight spins per real dimension
        const int aq = jb.stages > 0 ? 2 : sh.q;
        // no persistent variant above 32 dimensions: such a job runs the plain
        // path's launches inside the batch (binary encoding only)
        const int variant = mmgap::fused_variant(sh.KT, aq);
        if (variant < 0 && jb.stages > 0)
            return fail(ctx, MMGAP_EUNSUPPORTED,
                        "job %d: moves around a guess are batched up to 32 dimensions (K=%d)", j,
                        sh.K);
        if ((jb.guesses & MMGAP_GUESS_SIC) && jb.prob.n_tx > 16)
            return fail(ctx, MMGAP_EUNSUPPORTED, "job %d: MMSE-SIC supports n_tx <= 16 (got %d)",
                        j, jb.prob.n_tx);
        if (cim) {
            // CIM-CAC anneals: the build, anneal and selection launches of the
            // plain entry points, inside the batch
            if (jb.stages > 0)
                return fail(ctx, MMGAP_EUNSUPPORTED,
                            "job %d: CIM dynamics in a batch with the binary encoding only "
                            "(stages = 0)", j);
            if (sh.KT > 32 || sh.KT * sh.q > 64)
                return fail(ctx, MMGAP_EUNSUPPORTED,
                            "job %d: CIM dynamics needs K <= 32 and K q <= 64 spins", j);
            L.route[j] = kRouteCim;
            const mmgap_cim_params *c = jb.sched.cim;
            L.cim[j] = mmgap::CimParams{c->dt, c->p - 1.0f, c->a, -c->zeta, c->eps, c->amp0,
                                        c->f_mvm};
        } else if (variant < 0) {
            L.route[j] = kRoutePlain;
        } else if (jb.stages > 0 && !(flags & MMGAP_PLAN_PERSISTENT)) {
            const int gl = search_lanes_of(jb.sched.chains, jb.prob.n_sym, jb.prob.n_rx, sh.KT,
                                           false);
            if (gl) {
                L.route[j] = kRouteSearch;
                L.search_lanes[j] = gl;
            }
        }
        if (L.route[j] == kRoutePersistent && jb.sched.chains > kMaxFusedChains)
            return fail(ctx, MMGAP_EUNSUPPORTED, "job %d: chains=%d > %d in a batch", j,
                        jb.sched.chains, kMaxFusedChains);
        const mmgap_problem &p = jb.prob;
        mmgap::FusedJob &f = L.jobs[j];
        f = mmgap::FusedJob{};
        f.kind = p.kind;
        f.variant = variant;
        f.KT = sh.KT;
        f.Q = aq;
        f.dq = sh.q;
        f.stages = jb.stages;
        f.guesses = jb.guesses;
        f.K = sh.K;
        f.n_rows = p.n_rx;
        f.n_cols = p.n_tx;
        f.n_sym = p.n_sym;
        f.n_sc = p.n_sc;
        f.chains = jb.sched.chains;
        f.sweeps = jb.sched.sweeps;
        f.init = jb.sched.init;
        f.wpi = jb.sched.chains <= 64 ? 1 : (jb.sched.chains <= 128 ? 2 : 4);
        f.glanes = packed_lanes(jb.sched.chains, 0, 16);   // an item lies in one subcarrier
        f.ldf = (sh.KT + 31) / 32 * 32;   // 128-byte field rows: no scalar-cache line is shared
        if (jb.stages > 0) vpp_weights(f.w);      // {1, 1}: a move of -2, 0 or 2 levels
        else if (p.kind == MMGAP_KIND_DET) det_weights(sh.q, f.w);
        else vpp_weights(f.w);
        f.key0 = (uint32_t)jb.sched.seed;
        f.key1 = (uint32_t)(jb.sched.seed >> 32);
        f.inst_base = jb.sched.inst_base;
        f.c = qam_c(p.qam);
        f.c2 = qam_c2(p.qam);
        f.noise_var = (double)p.noise_var;
        f.tau = p.kind == MMGAP_KIND_VPP ? vpp_tau(&p) : 0.0;
        f.H = (const float2 *)jb.H;
        f.y = (const float2 *)jb.y_or_u;
        f.out0 = jb.out0;
        f.out1 = jb.out1;
        f.out2 = jb.out2;
        if (!cim) L.betas[j].assign(jb.sched.beta2, jb.sched.beta2 + jb.sched.sweeps);
        const int per = f.glanes ? 4 * (64 / f.glanes) : 4 / f.wpi;
        if (L.route[j] == kRoutePersistent)
            for (int sc = 0; sc < p.n_sc; ++sc)
                for (int s0 = 0; s0 < p.n_sym; s0 += per)
                    L.items.push_back({j, sc, s0, std::min(per, p.n_sym - s0)});
    }
    if (L.items.size() > 0x7FFFFFFFu) return fail(ctx, MMGAP_EUNSUPPORTED, "too many work items");
    // grouped by register class, each group ordered by decreasing cost
    auto cls_of = [&](const mmgap::FusedItem &a) {
        return mmgap::fused_kernel_class(L.jobs[a.job].variant);
    };
    std::stable_sort(L.items.begin(), L.items.end(),
                     [&](const mmgap::FusedItem &a, const mmgap::FusedItem &b) {
                         const int ca = cls_of(a), cb = cls_of(b);
                         if (ca != cb) return ca < cb;
                         return item_cost(L.jobs[a.job]) > item_cost(L.jobs[b.job]);
                     });
    for (size_t i = 0; i < L.items.size(); ++i) {
        const int c = cls_of(L.items[i]);
        if (L.cls_items[c] == 0) L.cls_first[c] = (int)i;
        ++L.cls_items[c];
    }
    Bump lay;
    L.o_jobs = lay.take(sizeof(mmgap::FusedJob) * std::max<size_t>(L.jobs.size(), 1));
    L.o_items = lay.take(sizeof(mmgap::FusedItem) * std::max<size_t>(L.items.size(), 1));
    L.o_counters = lay.take(sizeof(unsigned int) * mmgap::kFusedClasses);
    L.ob.resize(n_jobs);
    L.of.resize(n_jobs);
    L.ofp.resize(n_jobs);
    L.ox.resize(n_jobs);
    L.oxs.resize(n_jobs);
    L.oG.assign(n_jobs, 0);
    L.oE.assign(n_jobs, 0);
    L.oS.assign(n_jobs, 0);
    L.oA.assign(n_jobs, 0);
    for (int j = 0; j < n_jobs; ++j) L.ob[j] = lay.take(sizeof(float) * L.betas[j].size());
    L.header_bytes = lay.off;
    for (int j = 0; j < n_jobs; ++j) {
        const mmgap::FusedJob &f = L.jobs[j];
        const size_t ni = (size_t)f.n_sc * f.n_sym;
        if (L.route[j] != kRoutePersistent) {
            // the plain entry points' layout: rows of KT
            L.oG[j] = lay.take(sizeof(float) * (size_t)f.n_sc * f.KT * f.KT);
            L.of[j] = lay.take(sizeof(float) * ni * f.KT);
            L.ofp[j] = 0;
            L.ox[j] = lay.take(ni * (size_t)f.KT);
            L.oxs[j] = (f.guesses & MMGAP_GUESS_SIC) ? lay.take(ni * (size_t)f.KT) : 0;
            if (L.route[j] == kRouteCim || L.route[j] == kRoutePlain) {
                const size_t nw = (size_t)mmgap::spin_words(f.KT, f.Q);
                L.oE[j] = lay.take(sizeof(float) * ni * f.chains);
                L.oS[j] = lay.take(sizeof(uint32_t) * ni * f.chains * nw);
                if (f.kind == MMGAP_KIND_VPP)
                    L.oA[j] = lay.take(sizeof(double2) * (size_t)f.n_sc * f.n_rows * f.n_rows);
            }
            continue;
        }
        L.of[j] = lay.take(sizeof(float) * ni * f.ldf);
        L.ofp[j] = f.stages > 0 ? lay.take(sizeof(float) * ni * f.ldf) : 0;
        L.ox[j] = lay.take(ni * (size_t)f.KT);
        L.oxs[j] = (f.guesses & MMGAP_GUESS_SIC) ? lay.take(ni * (size_t)f.KT) : 0;
    }
    L.bytes = lay.off;
    return MMGAP_OK;
}

void batch_bind(BatchLayout &L, char *base, std::vector<unsigned char> &image)
{
    for (size_t j = 0; j < L.jobs.size(); ++j) {
        mmgap::FusedJob &f = L.jobs[j];
        f.beta2 = reinterpret_cast<const float *>(base + L.ob[j]);
        f.f = reinterpret_cast<float *>(base + L.of[j]);
        f.fp = f.stages > 0 ? reinterpret_cast<float *>(base + L.ofp[j]) : nullptr;
        f.x_fb = reinterpret_cast<signed char *>(base + L.ox[j]);
        f.x_sic = (f.guesses & MMGAP_GUESS_SIC) ? reinterpret_cast<signed char *>(base + L.oxs[j])
                                                : nullptr;
    }
    image.assign(L.header_bytes, 0);
    if (!L.jobs.empty())
        std::memcpy(image.data() + L.o_jobs, L.jobs.data(), sizeof(mmgap::FusedJob) * L.jobs.size());
    if (!L.items.empty())
        std::memcpy(image.data() + L.o_items, L.items.data(),
                    sizeof(mmgap::FusedItem) * L.items.size());
    for (size_t j = 0; j < L.jobs.size(); ++j)
        std::memcpy(image.data() + L.ob[j], L.betas[j].data(), sizeof(float) * L.betas[j].size());
}

int batch_launch_config(mmgap_ctx *ctx, const BatchLayout &L, char *base, int blocks,
                        BatchLaunch *out)
{
    BatchLaunch &b = *out;
    b = BatchLaunch();
    b.jobs = reinterpret_cast<mmgap::FusedJob *>(base + L.o_jobs);
    b.items = reinterpret_cast<mmgap::FusedItem *>(base + L.o_items);
    b.counters = reinterpret_cast<unsigned int *>(base + L.o_counters);
    hipError_t e = hipSuccess;
    if (ctx->cus == 0)
        e = hipDeviceGetAttribute(&ctx->cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    for (int c = 0; c < mmgap::kFusedClasses && e == hipSuccess; ++c) {
        b.first[c] = L.cls_first[c];
        b.count[c] = L.cls_items[c];
        if (!b.count[c]) continue;
        if (ctx->fused_per_cu[c] == 0) e = mmgap::fused_blocks_per_cu(c, &ctx->fused_per_cu[c]);
        if (e == hipSuccess && ctx->fused_per_cu[c] < 1) e = hipErrorInvalidConfiguration;
        b.blocks[c] = std::min(blocks > 0 ? blocks : ctx->fused_per_cu[c] * ctx->cus, b.count[c]);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "occupancy query");
    for (size_t j = 0; j < L.jobs.size(); ++j) {
        const mmgap::FusedJob &f = L.jobs[j];
        if (L.route[j] == kRoutePersistent || f.n_sc * f.n_sym == 0) continue;
        SepLaunch sl;
        sl.route = L.route[j];
        sl.kind = f.kind;
        sl.KT = f.KT;
        sl.q = f.Q;
        float *G = reinterpret_cast<float *>(base + L.oG[j]);
        float *fr = reinterpret_cast<float *>(base + L.of[j]);
        signed char *xr = reinterpret_cast<signed char *>(base + L.ox[j]);
        const int ni = f.n_sc * f.n_sym;
        if (f.kind == MMGAP_KIND_DET) {
            mmgap::DetBuildArgs &d = sl.det;
            d.H = f.H;
            d.y = f.y;
            d.n_sc = f.n_sc;
            d.n_r = f.n_rows;
            d.n_t = f.n_cols;
            d.n_sym = f.n_sym;
            d.ld = f.KT;
            d.qtop = (1 << f.dq) - 1;
            d.c = f.c;
            d.c2 = f.c2;
            d.noise_var = f.noise_var;
            d.G = G;
            d.f = fr;
            d.x_fb = xr;
            d.ynorm = nullptr;
        } else {
            mmgap::VppBuildArgs &v = sl.vpp;
            v.H = f.H;
            v.u = f.y;
            v.n_sc = f.n_sc;
            v.n_u = f.n_rows;
            v.n_t = f.n_cols;
            v.n_sym = f.n_sym;
            v.ld = f.KT;
            v.tau = f.tau;
            v.G = G;
            v.f = fr;
            v.x_fb = xr;
            v.Ainv = reinterpret_cast<double2 *>(base + L.oA[j]);
            v.unorm = nullptr;
        }
        if (sl.route == kRouteCim || sl.route == kRoutePlain) {
            mmgap::AnnealArgs &a = sl.ann;
            a.G = G;
            a.inst_per_G = f.n_sym;
            a.f = fr;
            a.x_fb = xr;
            a.sweeps = f.sweeps;
            a.chains = f.chains;
            a.n_inst = ni;
            for (int b = 0; b < mmgap::kMaxQ; ++b) a.w[b] = f.w[b];
            a.key0 = f.key0;
            a.key1 = f.key1;
            a.inst_base = f.inst_base;
            a.init_mode = f.init;
            a.glanes = packed_lanes(f.chains, f.n_sym, 64);
            a.chain_E = reinterpret_cast<float *>(base + L.oE[j]);
            a.chain_S = reinterpret_cast<uint32_t *>(base + L.oS[j]);
            if (sl.route == kRouteCim) a.cim = L.cim[j];
            else a.beta2 = reinterpret_cast<const float *>(base + L.ob[j]);
            mmgap::SelectArgs &se = sl.sel;
            se.mode = f.kind == MMGAP_KIND_DET ? mmgap::kSelectDet : mmgap::kSelectVpp;
            se.n_inst = ni;
            se.K = f.K;
            se.KT = f.KT;
            se.q = f.Q;
            se.chains = f.chains;
            for (int b = 0; b < mmgap::kMaxQ; ++b) se.w[b] = f.w[b];
            se.G = G;
            se.inst_per_G = f.n_sym;
            se.f = fr;
            se.x_fb = xr;
            se.chain_E = a.chain_E;
            se.chain_S = a.chain_S;
            se.H = f.H;
            se.y = f.y;
            se.n_rows = f.n_rows;
            se.n_cols = f.n_cols;
            se.n_sym = f.n_sym;
            se.c = f.c;
            if (f.kind == MMGAP_KIND_DET) {
                se.sym_out = static_cast<unsigned char *>(f.out0);
                se.metric_out = static_cast<float *>(f.out1);
            } else {
                se.Ainv = sl.vpp.Ainv;
                se.tau = f.tau;
                se.v_out = static_cast<signed char *>(f.out0);
                se.x_out = static_cast<float2 *>(f.out1);
                se.gamma_out = static_cast<float *>(f.out2);
            }
        } else {
            mmgap::SearchArgs &r = sl.srch;
            const int g = f.guesses ? f.guesses : MMGAP_GUESS_MMSE;
            r.G = G;
            r.inst_per_G = f.n_sym;
            r.f = fr;
            r.guess_a = (g & MMGAP_GUESS_MMSE) ? xr : nullptr;
            r.guess_b = (g & MMGAP_GUESS_SIC) ? reinterpret_cast<signed char *>(base + L.oxs[j])
                                              : nullptr;
            r.beta2 = reinterpret_cast<const float *>(base + L.ob[j]);
            r.n_inst = ni;
            r.K = f.K;
            r.sweeps = f.sweeps;
            r.chains = f.chains;
            r.stages = f.stages;
            r.init_mode = f.init;
            r.glanes = L.search_lanes[j];
            r.key0 = f.key0;
            r.key1 = f.key1;
            r.inst_base = f.inst_base;
            r.dq = f.dq;
            r.H = f.H;
            r.y = f.y;
            r.n_rows = f.n_rows;
            r.n_cols = f.n_cols;
            r.n_sym = f.n_sym;
            r.c = f.c;
            r.sym_out = static_cast<unsigned char *>(f.out0);
            r.metric_out = static_cast<float *>(f.out1);
            r.from_b = f.guesses ? static_cast<unsigned char *>(f.out2) : nullptr;
        }
        b.sep.push_back(sl);
    }
    for (size_t j = 0; j < L.jobs.size(); ++j) {
        const mmgap::FusedJob &f = L.jobs[j];
        if (!(f.guesses & MMGAP_GUESS_SIC) || f.n_sc * f.n_sym == 0) continue;
        mmgap::SicArgs sa{};
        sa.H = f.H;
        sa.y = f.y;
        sa.n_sc = f.n_sc;
        sa.n_r = f.n_rows;
        sa.n_t = f.n_cols;
        sa.n_sym = f.n_sym;
        sa.q = f.dq;
        sa.c = f.c;
        sa.noise_var = f.noise_var;
        sa.levels = reinterpret_cast<signed char *>(base + L.oxs[j]);
        sa.ldl = f.KT;
        b.sic.push_back(sa);
    }
    return MMGAP_OK;
}

hipError_t batch_enqueue(const BatchLaunch &b, const uint32_t *accept_table, hipStream_t st)
{
    hipError_t e = mmgap::launch_fused_reset(b.counters, st);
    // the MMSE-SIC guesses of the jobs that search from it, before the
    // searches and persistent kernels that read them
    for (size_t k = 0; k < b.sic.size() && e == hipSuccess; ++k) e = mmgap::launch_sic(b.sic[k], st);
    // jobs with launches of their own: build, then CIM-CAC or Metropolis
    // anneal and selection, or the search
    for (size_t k = 0; k < b.sep.size() && e == hipSuccess; ++k) {
        const SepLaunch &sl = b.sep[k];
        e = sl.kind == MMGAP_KIND_DET ? mmgap::launch_det_build(sl.det, st)
                                      : mmgap::launch_vpp_build(sl.vpp, st);
        if (e != hipSuccess) break;
        if (sl.route == kRouteCim) {
            e = mmgap::launch_cim(sl.KT, sl.q, sl.ann, st);
            if (e == hipSuccess) e = mmgap::launch_select(sl.sel, st);
        } else if (sl.route == kRoutePlain) {
            mmgap::AnnealArgs a = sl.ann;
            a.accept_table = accept_table;
            e = mmgap::launch_anneal(sl.KT, sl.q, a, st);
            if (e == hipSuccess) e = mmgap::launch_select(sl.sel, st);
        } else {
            mmgap::SearchArgs r = sl.srch;
            r.accept_table = accept_table;
            e = mmgap::launch_search(sl.KT, r, st);
        }
    }
    for (int c = mmgap::kFusedClasses - 1; c >= 0 && e == hipSuccess; --c)
        e = mmgap::launch_fused(c, b.jobs, b.items + b.first[c], b.count[c], b.counters + c,
                                accept_table, b.blocks[c], st);
    return e;
}

}  // namespace host
}  // namespace mmgap

struct mmgap_plan {
    mmgap_ctx *ctx = nullptr;
    int n_items = 0;
    BatchLaunch launch;
    void *mem = nullptr;
    size_t bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    bool done_valid = false;
};

namespace {

void plan_free(mmgap_plan *p)
{
    if (!p) return;
    if (p->done) {
        if (p->done_valid) (void)hipEventSynchronize(p->done);
        (void)hipEventDestroy(p->done);
    }
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->mem) {
        (void)hipFree(p->mem);
        p->ctx->plan_bytes -= p->bytes;
    }
    delete p;
}

}  // namespace

extern "C" {

int mmgap_create(mmgap_ctx **out, int device, size_t hbm_budget_bytes)
{
    if (!out) return fail(nullptr, MMGAP_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || ndev <= 0)
        return fail(nullptr, MMGAP_EDEVICE, "no HIP device available (%s)", hipGetErrorString(e));
    if (device < 0 || device >= ndev)
        return fail(nullptr, MMGAP_EINVAL, "device %d outside 0..%d", device, ndev - 1);
    mmgap_ctx *ctx = new (std::nothrow) mmgap_ctx();
    if (!ctx) return fail(nullptr, MMGAP_ENOMEM, "out of host memory");
    ctx->device = device;
    if (hbm_budget_bytes) ctx->budget = hbm_budget_bytes;
    DeviceGuard g(device);
    if (!g.ok) {
        delete ctx;
        return fail(nullptr, MMGAP_EDEVICE, "hipSetDevice(%d) failed", device);
    }
    const size_t ring = sizeof(float) * (size_t)kRing * mmgap::kMaxSweeps;
    e = hipMalloc(&ctx->beta_dev, ring);
    if (e == hipSuccess) e = hipHostMalloc(&ctx->beta_host, ring, hipHostMallocDefault);
    for (int i = 0; i < kRing && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&ctx->ring_ev[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->done, hipEventDisableTiming);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking);
    for (int i = 0; i < 3 && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&ctx->aux_ev[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipMalloc(&ctx->accept_dev, sizeof(uint32_t) * mmgap::kAcceptTable);
    if (e == hipSuccess) {
        // T[j] = round(2^16 * 2^(-j/64)): no entry is within 1e-3 of a rounding tie
        uint32_t table[mmgap::kAcceptTable];
        for (int j = 0; j + 1 < mmgap::kAcceptTable; ++j)
            table[j] = (uint32_t)std::llround(65536.0 * std::exp2(-(double)j / 64.0));
        table[mmgap::kAcceptTable - 1] = 0u;
        e = hipMemcpy(ctx->accept_dev, table, sizeof table, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess && device < kNoAllocDevices)
        e = noalloc_scratch_address(device, &ctx->noalloc_scratch);
    if (e != hipSuccess) {
        mmgap_destroy(ctx);
        return fail(nullptr, MMGAP_EDEVICE, "context setup: %s", hipGetErrorString(e));
    }
    *out = ctx;
    return MMGAP_OK;
}

int mmgap_destroy(mmgap_ctx *ctx)
{
    if (!ctx) return MMGAP_OK;
    DeviceGuard g(ctx->device);
    server_shutdown(ctx);
    (void)hipDeviceSynchronize();
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->beta_dev) (void)hipFree(ctx->beta_dev);
    if (ctx->beta_host) (void)hipHostFree(ctx->beta_host);
    for (int i = 0; i < kRing; ++i)
        if (ctx->ring_ev[i]) (void)hipEventDestroy(ctx->ring_ev[i]);
    for (int r = 0; r < kProfRing; ++r)
        for (int i = 0; i < 4; ++i)
            if (ctx->prof_ev[r][i]) (void)hipEventDestroy(ctx->prof_ev[r][i]);
    if (ctx->done) (void)hipEventDestroy(ctx->done);
    for (int i = 0; i < 3; ++i)
        if (ctx->aux_ev[i]) (void)hipEventDestroy(ctx->aux_ev[i]);
    if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
    if (ctx->accept_dev) (void)hipFree(ctx->accept_dev);
    delete ctx;
    return MMGAP_OK;
}

const char *mmgap_last_error(const mmgap_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

int mmgap_build_ising(mmgap_ctx *ctx, const mmgap_problem *prob, const void *H,
                      const void *y_or_u, float *G, float *f, signed char *x_fallback,
                      float *J_dense, float *h_dense, float *e_const, void *stream)
{
    if (!ctx) return MMGAP_EINVAL;
    ProblemShape sh;
    int rc = check_problem(ctx, prob, -1, &sh);
    if (rc) return rc;
    if (sh.n_inst == 0) return MMGAP_OK;
    if (!H || !y_or_u || !G || !f) return fail(ctx, MMGAP_EINVAL, "H, y_or_u, G and f are required");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    Bump plan;
    const size_t o_norm = e_const ? plan.take(sizeof(double) * (size_t)sh.n_inst) : 0;
    if ((rc = ensure_scratch(ctx, plan.off))) return rc;
    if ((rc = begin_call(ctx, st))) return rc;
    hipError_t e;
    int w[mmgap::kMaxQ];
    double *norm = e_const ? at<double>(ctx, o_norm) : nullptr;
    if (prob->kind == MMGAP_KIND_DET) {
        mmgap::DetBuildArgs a{};
        a.H = (const float2 *)H;
        a.y = (const float2 *)y_or_u;
        a.n_sc = prob->n_sc;
        a.n_r = prob->n_rx;
        a.n_t = prob->n_tx;
        a.n_sym = prob->n_sym;
        a.ld = sh.K;
        a.qtop = (1 << sh.q) - 1;
        a.c = qam_c(prob->qam);
        a.c2 = qam_c2(prob->qam);
        a.noise_var = (double)prob->noise_var;
        a.G = G;
        a.f = f;
        a.x_fb = x_fallback;
        a.ynorm = norm;
        e = mmgap::launch_det_build(a, st);
        det_weights(sh.q, w);
    } else {
        mmgap::VppBuildArgs a{};
        a.H = (const float2 *)H;
        a.u = (const float2 *)y_or_u;
        a.n_sc = prob->n_sc;
        a.n_u = prob->n_rx;
        a.n_t = prob->n_tx;
        a.n_sym = prob->n_sym;
        a.ld = sh.K;
        a.tau = vpp_tau(prob);
        a.G = G;
        a.f = f;
        a.x_fb = x_fallback;
        a.Ainv = nullptr;
        a.unorm = norm;
        e = mmgap::launch_vpp_build(a, st);
        vpp_weights(w);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "build launch");
    if (J_dense || h_dense || e_const) {
        mmgap::ExpandArgs x{};
        x.G = G;
        x.f = f;
        x.norm = norm;
        x.n_sc = prob->n_sc;
        x.n_sym = prob->n_sym;
        x.K = sh.K;
        x.q = sh.q;
        for (int b = 0; b < mmgap::kMaxQ; ++b) x.w[b] = w[b];
        x.J = J_dense;
        x.h = h_dense;
        x.e_const = e_const;
        e = mmgap::launch_expand(x, st);
        if (e != hipSuccess) return hip_fail(ctx, e, "expand launch");
    }
    return end_call(ctx, st);
}

int mmgap_solve(mmgap_ctx *ctx, int n_inst, int K, int q, const signed char *w,
                const float *G, int inst_per_G, const float *f, const signed char *x_fallback,
                const mmgap_schedule *sched, signed char *spins_out, float *e_out,
                int *win_out, void *stream)
{
    if (!ctx) return MMGAP_EINVAL;
    if (n_inst < 0) return fail(ctx, MMGAP_EINVAL, "n_inst=%d < 0", n_inst);
    if (K < 1 || K > mmgap::kMaxK) return fail(ctx, MMGAP_EUNSUPPORTED, "K=%d outside 1..64", K);
    if (q < 1 || q > mmgap::kMaxQ) return fail(ctx, MMGAP_EUNSUPPORTED, "q=%d outside 1..4", q);
    if (K > 32 && q > 2)
        return fail(ctx, MMGAP_EUNSUPPORTED, "K=%d > 32 supports q <= 2 (got %d)", K, q);
    if (!w) return fail(ctx, MMGAP_EINVAL, "w is NULL");
    int wv[mmgap::kMaxQ] = {1, 1, 1, 1};
    for (int b = 0; b < q; ++b) {
        if (!pow2_weight(w[b]))
            return fail(ctx, MMGAP_EUNSUPPORTED, "w[%d]=%d is not a power of two in 1..64", b, w[b]);
        wv[b] = w[b];
    }
    if (inst_per_G < 1) return fail(ctx, MMGAP_EINVAL, "inst_per_G=%d < 1", inst_per_G);
    int rc = check_schedule(ctx, sched);
    if (rc) return rc;
    if (n_inst == 0) return MMGAP_OK;
    if (!G || !f || !spins_out || !e_out)
        return fail(ctx, MMGAP_EINVAL, "G, f, spins_out and e_out are required");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const int KT = mmgap::padded_k(K);
    const int NW = mmgap::spin_words(KT, q);
    const int n_G = (n_inst + inst_per_G - 1) / inst_per_G;
    const bool pad = KT != K;
    Bump plan;
    const size_t oG = pad ? plan.take(sizeof(float) * (size_t)n_G * KT * KT) : 0;
    const size_t of = pad ? plan.take(sizeof(float) * (size_t)n_inst * KT) : 0;
    const size_t ox = (pad && x_fallback) ? plan.take((size_t)n_inst * KT) : 0;
    const size_t oE = plan.take(sizeof(float) * (size_t)n_inst * sched->chains);
    const size_t oS = plan.take(sizeof(uint32_t) * (size_t)n_inst * sched->chains * NW);
    if ((rc = ensure_scratch(ctx, plan.off))) return rc;
    if ((rc = begin_call(ctx, st))) return rc;
    prof_mark(ctx, 0, st);
    const float *Gp = G;
    const float *fp = f;
    const signed char *xp = x_fallback;
    hipError_t e = hipSuccess;
    if (pad) {
        e = mmgap::launch_pad_matrix(G, at<float>(ctx, oG), n_G, K, KT, st);
        if (e == hipSuccess) e = mmgap::launch_pad_rows_f32(f, at<float>(ctx, of), n_inst, K, KT, st);
        if (e == hipSuccess && x_fallback)
            e = mmgap::launch_pad_rows_i8(x_fallback, at<signed char>(ctx, ox), n_inst, K, KT, st);
        if (e != hipSuccess) return hip_fail(ctx, e, "pad launch");
        Gp = at<float>(ctx, oG);
        fp = at<float>(ctx, of);
        xp = x_fallback ? at<signed char>(ctx, ox) : nullptr;
    }
    mmgap::SelectArgs sel{};
    sel.mode = mmgap::kSelectSolve;
    sel.spins_out = spins_out;
    sel.e_out = e_out;
    sel.win_out = win_out;
    rc = run_solver(ctx, st, n_inst, K, q, KT, wv, Gp, inst_per_G, fp, xp, sched,
                    at<float>(ctx, oE), at<uint32_t>(ctx, oS), sel);
    if (rc) return rc;
    return end_call(ctx, st);
}

int mmgap_cim_chains(mmgap_ctx *ctx, int n_inst, int K, int q, const signed char *w,
                     const float *G, int inst_per_G, const float *f,
                     const signed char *x_fallback, const mmgap_schedule *sched,
                     signed char *spins_out, float *e_out, unsigned char *diverged_out,
                     void *stream)
{
    if (!ctx) return MMGAP_EINVAL;
    if (n_inst < 0) return fail(ctx, MMGAP_EINVAL, "n_inst=%d < 0", n_inst);
    if (K < 1 || K > mmgap::kMaxK) return fail(ctx, MMGAP_EUNSUPPORTED, "K=%d outside 1..64", K);
    if (q < 1 || q > mmgap::kMaxQ) return fail(ctx, MMGAP_EUNSUPPORTED, "q=%d outside 1..4", q);
    if (K > 32 && q > 2)
        return fail(ctx, MMGAP_EUNSUPPORTED, "K=%d > 32 supports q <= 2 (got %d)", K, q);
    if (!w) return fail(ctx, MMGAP_EINVAL, "w is NULL");
    int wv[mmgap::kMaxQ] = {1, 1, 1, 1};
    for (int b = 0; b < q; ++b) {
        if (!pow2_weight(w[b]))
            return fail(ctx, MMGAP_EUNSUPPORTED, "w[%d]=%d is not a power of two in 1..64", b, w[b]);
        wv[b] = w[b];
    }
    if (inst_per_G < 1) return fail(ctx, MMGAP_EINVAL, "inst_per_G=%d < 1", inst_per_G);
    int rc = check_schedule(ctx, sched);
    if (rc) return rc;
    if (sched->dynamics != MMGAP_DYN_CIM)
        return fail(ctx, MMGAP_EINVAL, "mmgap_cim_chains needs a CIM-CAC schedule");
    const int KT = mmgap::padded_k(K);
    if (KT > 32 || KT * q > 64)
        return fail(ctx, MMGAP_EUNSUPPORTED,
                    "CIM dynamics needs K <= 32 and K q <= 64 spins (padded %d x %d)", KT, q);
    if (n_inst == 0) return MMGAP_OK;
    if (!G || !f || !spins_out)
        return fail(ctx, MMGAP_EINVAL, "G, f and spins_out are required");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const int NW = mmgap::spin_words(KT, q);
    const int n_G = (n_inst + inst_per_G - 1) / inst_per_G;
    const bool pad = KT != K;
    Bump plan;
    const size_t oG = pad ? plan.take(sizeof(float) * (size_t)n_G * KT * KT) : 0;
    const size_t of = pad ? plan.take(sizeof(float) * (size_t)n_inst * KT) : 0;
    const size_t ox = (pad && x_fallback) ? plan.take((size_t)n_inst * KT) : 0;
    const size_t oE = plan.take(sizeof(float) * (size_t)n_inst * sched->chains);
    const size_t oS = plan.take(sizeof(uint32_t) * (size_t)n_inst * sched->chains * NW);
    if ((rc = ensure_scratch(ctx, plan.off))) return rc;
    if ((rc = begin_call(ctx, st))) return rc;
    const float *Gp = G;
    const float *fp = f;
    const signed char *xp = x_fallback;
    hipError_t e = hipSuccess;
    if (pad) {
        e = mmgap::launch_pad_matrix(G, at<float>(ctx, oG), n_G, K, KT, st);
        if (e == hipSuccess) e = mmgap::launch_pad_rows_f32(f, at<float>(ctx, of), n_inst, K, KT, st);
        if (e == hipSuccess && x_fallback)
            e = mmgap::launch_pad_rows_i8(x_fallback, at<signed char>(ctx, ox), n_inst, K, KT, st);
        if (e != hipSuccess) return hip_fail(ctx, e, "pad launch");
        Gp = at<float>(ctx, oG);
        fp = at<float>(ctx, of);
        xp = x_fallback ? at<signed char>(ctx, ox) : nullptr;
    }
    mmgap::AnnealArgs a{};
    a.G = Gp;
    a.inst_per_G = inst_per_G;
    a.f = fp;
    a.x_fb = xp;
    a.sweeps = sched->sweeps;
    a.chains = sched->chains;
    a.n_inst = n_inst;
    for (int b = 0; b < mmgap::kMaxQ; ++b) a.w[b] = wv[b];
    a.key0 = (uint32_t)sched->seed;
    a.key1 = (uint32_t)(sched->seed >> 32);
    a.inst_base = sched->inst_base;
    a.init_mode = sched->init;
    a.glanes = packed_lanes(sched->chains, inst_per_G, 64);
    a.chain_E = e_out ? e_out : at<float>(ctx, oE);
    a.chain_S = at<uint32_t>(ctx, oS);
    a.cim.dt = sched->cim->dt;
    a.cim.pm1 = sched->cim->p - 1.0f;
    a.cim.a = sched->cim->a;
    a.cim.nzeta = -sched->cim->zeta;
    a.cim.eps = sched->cim->eps;
    a.cim.amp0 = sched->cim->amp0;
    a.cim.f_mvm = sched->cim->f_mvm;
    a.chain_div = diverged_out;
    a.n_real = K * q;
    e = mmgap::launch_cim(KT, q, a, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "CIM anneal launch");
    // spins of every chain, padding dropped (real spins come first in each word row)
    e = mmgap::launch_chain_spins(a.chain_S, NW, K * q, (size_t)n_inst * sched->chains,
                                  spins_out, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "spin expansion launch");
    return end_call(ctx, st);
}

}  // extern "C"

namespace {

// Scratch layout of one detection call (byte offsets from the scratch base).
struct DetectScratch {
    size_t oG, of, ox, oE, oS, bytes;
};

DetectScratch detect_scratch(const mmgap_problem *prob, const ProblemShape &sh,
                             const mmgap_schedule *sched)
{
    const int KT = sh.KT, NW = mmgap::spin_words(KT, sh.q), ni = sh.n_inst;
    Bump plan;
    DetectScratch d;
    d.oG = plan.take(sizeof(float) * (size_t)prob->n_sc * KT * KT);
    d.of = plan.take(sizeof(float) * (size_t)ni * KT);
    d.ox = plan.take((size_t)ni * KT);
    d.oE = plan.take(sizeof(float) * (size_t)ni * sched->chains);
    d.oS = plan.take(sizeof(uint32_t) * (size_t)ni * sched->chains * NW);
    d.bytes = plan.off;
    return d;
}

// The detection launches (build, anneal, select/decode) with every scratch
// buffer at `base` (device memory of at least L.bytes bytes).
int detect_launches(mmgap_ctx *ctx, hipStream_t st, const mmgap_problem *prob,
                    const ProblemShape &sh, const DetectScratch &L, char *base, const void *H,
                    const void *y, const mmgap_schedule *sched, unsigned char *sym_out,
                    float *metric_out)
{
    const int KT = sh.KT, ni = sh.n_inst;
    int rc = begin_call(ctx, st);
    if (rc) return rc;
    prof_mark(ctx, 0, st);
    mmgap::DetBuildArgs b{};
    b.H = (const float2 *)H;
    b.y = (const float2 *)y;
    b.n_sc = prob->n_sc;
    b.n_r = prob->n_rx;
    b.n_t = prob->n_tx;
    b.n_sym = prob->n_sym;
    b.ld = KT;
    b.qtop = (1 << sh.q) - 1;
    b.c = qam_c(prob->qam);
    b.c2 = qam_c2(prob->qam);
    b.noise_var = (double)prob->noise_var;
    b.G = reinterpret_cast<float *>(base + L.oG);
    b.f = reinterpret_cast<float *>(base + L.of);
    b.x_fb = reinterpret_cast<signed char *>(base + L.ox);
    b.ynorm = nullptr;
    hipError_t e = mmgap::launch_det_build(b, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "build launch");
    int w[mmgap::kMaxQ];
    det_weights(sh.q, w);
    mmgap::SelectArgs sel{};
    sel.mode = mmgap::kSelectDet;
    sel.H = (const float2 *)H;
    sel.y = (const float2 *)y;
    sel.n_rows = prob->n_rx;
    sel.n_cols = prob->n_tx;
    sel.n_sym = prob->n_sym;
    sel.c = b.c;
    sel.sym_out = sym_out;
    sel.metric_out = metric_out;
    rc = run_solver(ctx, st, ni, sh.K, sh.q, KT, w, b.G, prob->n_sym, b.f, b.x_fb, sched,
                    reinterpret_cast<float *>(base + L.oE),
                    reinterpret_cast<uint32_t *>(base + L.oS), sel);
    if (rc) return rc;
    return end_call(ctx, st);
}

}  // namespace

extern "C" {

int mmgap_detect(mmgap_ctx *ctx, const mmgap_problem *prob, const void *H, const void *y,
                 const mmgap_schedule *sched, unsigned char *sym_out, float *metric_out,
                 void *stream)
{
    if (!ctx) return MMGAP_EINVAL;
    ProblemShape sh;
    int rc = check_problem(ctx, prob, MMGAP_KIND_DET, &sh);
    if (rc) return rc;
    if ((rc = check_schedule(ctx, sched))) return rc;
    if (sh.n_inst == 0) return MMGAP_OK;
    if (!H || !y || !sym_out) return fail(ctx, MMGAP_EINVAL, "H, y and sym_out are required");
    DeviceGuard g(ctx->device);
    const DetectScratch L = detect_scratch(prob, sh, sched);
    if ((rc = ensure_scratch(ctx, L.bytes))) return rc;
    return detect_launches(ctx, (hipStream_t)stream, prob, sh, L, static_cast<char *>(ctx->scratch),
                           H, y, sched, sym_out, metric_out);
}

int mmgap_detect_noalloc(mmgap_ctx *ctx, const mmgap_problem *prob, const void *H,
                         const void *y, const mmgap_schedule *sched, unsigned char *sym_out,
                         float *metric_out, void *stream)
{
    if (!ctx) return MMGAP_EINVAL;
    ProblemShape sh;
    int rc = check_problem(ctx, prob, MMGAP_KIND_DET, &sh);
    if (rc) return rc;
    if ((rc = check_schedule(ctx, sched))) return rc;
    if (sh.n_inst == 0) return MMGAP_OK;
    if (!H || !y || !sym_out) return fail(ctx, MMGAP_EINVAL, "H, y and sym_out are required");
    const DetectScratch L = detect_scratch(prob, sh, sched);
    if (L.bytes > kNoAllocScratchBytes)
        return fail(ctx, MMGAP_EUNSUPPORTED,
                    "the call needs %zu bytes of scratch, above the fixed %zu of "
                    "mmgap_detect_noalloc (fewer subcarriers or chains per call)",
                    L.bytes, kNoAllocScratchBytes);
    if (!ctx->noalloc_scratch)
        return fail(ctx, MMGAP_EUNSUPPORTED, "no fixed scratch on device %d", ctx->device);
    DeviceGuard g(ctx->device);
    return detect_launches(ctx, (hipStream_t)stream, prob, sh, L, ctx->noalloc_scratch, H, y,
                           sched, sym_out, metric_out);
}

namespace {

// Stages of moves around the guess xg (device, [ni][KT], updated in place):
// per stage the move fields f - G x_g, an anneal of the {-2, 0, 2}-move
// problem with the zero move zmov as the fallback and Philox key
// seed_base + s, and the selection that applies the winning move; the last
// stage decodes into sym_out / metric_out when `decode`.
int run_delta_stages(mmgap_ctx *ctx, hipStream_t st, const mmgap_problem *prob,
                     const ProblemShape &sh, const void *H, const void *y,
                     const mmgap_schedule *sched, int stages, uint64_t seed_base, float *G,
                     float *f, float *fp, signed char *xg, signed char *zmov, float *chainE,
                     uint32_t *chainS, bool decode, unsigned char *sym_out, float *metric_out)
{
    const int q = 2, KT = sh.KT, ni = sh.n_inst;
    const int w[mmgap::kMaxQ] = {1, 1, 0, 0};
    for (int s = 0; s < stages; ++s) {
        mmgap::DeltaPrepArgs d{};
        d.G = G;
        d.inst_per_G = prob->n_sym;
        d.f = f;
        d.guess = xg;
        d.f_out = fp;
        d.n_inst = ni;
        d.KT = KT;
        hipError_t e = mmgap::launch_delta_prep(d, st);
        if (e != hipSuccess) return hip_fail(ctx, e, "move-field launch");
        mmgap_schedule ss = *sched;
        ss.seed = seed_base + (uint64_t)s;        // one Philox key per stage
        mmgap::SelectArgs sel{};
        sel.mode = mmgap::kSelectDelta;
        sel.H = (const float2 *)H;
        sel.y = (const float2 *)y;
        sel.n_rows = prob->n_rx;
        sel.n_cols = prob->n_tx;
        sel.n_sym = prob->n_sym;
        sel.c = qam_c(prob->qam);
        sel.sym_out = sym_out;
        sel.metric_out = metric_out;
        sel.guess = xg;
        sel.f_full = f;
        sel.qtop = (1 << sh.q) - 1;
        sel.dq = sh.q;
        sel.decode = decode && s == stages - 1;
        int rc = run_solver(ctx, st, ni, sh.K, q, KT, w, G, prob->n_sym, fp, zmov, &ss, chainE,
                            chainS, sel);
        if (rc) return rc;
    }
    return MMGAP_OK;
}

// Lanes per instance of the one-launch search (k_search), or 0 when the stage
// launches must run it: chains <= 64, 64 / lanes instances of a subcarrier
// per wavefront (at most 16, so at least 4 lanes), n_rx <= 2 lanes.
int search_lanes(const mmgap_ctx *ctx, const mmgap_problem *prob, const ProblemShape &sh,
                 const mmgap_schedule *sched)
{
    if (ctx->stage_launches) return 0;
    return search_lanes_of(sched->chains, prob->n_sym, prob->n_rx, sh.KT,
                           sched->dynamics == MMGAP_DYN_CIM);
}

// Every stage of the chains from guess A and/or guess B (device rows
// [n][KT], read only), the choice and the decode, in one launch.
int run_search(mmgap_ctx *ctx, hipStream_t st, const mmgap_problem *prob,
               const ProblemShape &sh, const void *H, const void *y,
               const mmgap_schedule *sched, int stages, int lanes, const float *G,
               const float *f, const signed char *xa, const signed char *xb,
               unsigned char *sym_out, float *metric_out, unsigned char *from_b)
{
    const float *beta = nullptr;
    int rc = upload_beta(ctx, sched, st, &beta);
    if (rc) return rc;
    mmgap::SearchArgs a{};
    a.G = G;
    a.inst_per_G = prob->n_sym;
    a.f = f;
    a.guess_a = xa;
    a.guess_b = xb;
    a.beta2 = beta;
    a.accept_table = ctx->accept_dev;
    a.n_inst = sh.n_inst;
    a.K = sh.K;
    a.sweeps = sched->sweeps;
    a.chains = sched->chains;
    a.stages = stages;
    a.init_mode = sched->init;
    a.glanes = lanes;
    a.key0 = (uint32_t)sched->seed;
    a.key1 = (uint32_t)(sched->seed >> 32);
    a.inst_base = sched->inst_base;
    a.dq = sh.q;
    a.H = (const float2 *)H;
    a.y = (const float2 *)y;
    a.n_rows = prob->n_rx;
    a.n_cols = prob->n_tx;
    a.n_sym = prob->n_sym;
    a.c = qam_c(prob->qam);
    a.sym_out = sym_out;
    a.metric_out = metric_out;
    a.from_b = from_b;
    prof_mark(ctx, 1, st);
    hipError_t e = mmgap::launch_search(sh.KT, a, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "search launch");
    prof_mark(ctx, 2, st);
    prof_mark(ctx, 3, st);
    if (ctx->profiling) {
        ++ctx->prof_count;
        ctx->prof_open = false;
    }
    return MMGAP_OK;
}

// The detection build into G, f and the sliced MMSE estimate xg.
int det_build_into(mmgap_ctx *ctx, hipStream_t st, const mmgap_problem *prob,
                   const ProblemShape &sh, const void *H, const void *y, float *G, float *f,
                   signed char *xg)
{
    mmgap::DetBuildArgs b{};
    b.H = (const float2 *)H;
    b.y = (const float2 *)y;
    b.n_sc = prob->n_sc;
    b.n_r = prob->n_rx;
    b.n_t = prob->n_tx;
    b.n_sym = prob->n_sym;
    b.ld = sh.KT;
    b.qtop = (1 << sh.q) - 1;
    b.c = qam_c(prob->qam);
    b.c2 = qam_c2(prob->qam);
    b.noise_var = (double)prob->noise_var;
    b.G = G;
    b.f = f;
    b.x_fb = xg;
    b.ynorm = nullptr;
    hipError_t e = mmgap::launch_det_build(b, st);
    return e == hipSuccess ? MMGAP_OK : hip_fail(ctx, e, "build launch");
}

mmgap::SicArgs sic_args(const mmgap_problem *prob, const ProblemShape &sh, const void *H,
                        const void *y)
{
    mmgap::SicArgs a{};
    a.H = (const float2 *)H;
    a.y = (const float2 *)y;
    a.n_sc = prob->n_sc;
    a.n_r = prob->n_rx;
    a.n_t = prob->n_tx;
    a.n_sym = prob->n_sym;
    a.q = sh.q;
    a.c = qam_c(prob->qam);
    a.noise_var = (double)prob->noise_var;
    return a;
}

}  // namespace

int mmgap_detect_delta(mmgap_ctx *ctx, const mmgap_problem *prob, const void *H, const void *y,
                       const mmgap_schedule *sched, int stages, const signed char *guess,
                       unsigned char *sym_out, float *metric_out, void *stream)
{
    if (!ctx) return MMGAP_EINVAL;
    ProblemShape sh;
    int rc = check_problem(ctx, prob, MMGAP_KIND_DET, &sh);
    if (rc) return rc;
    if ((rc = check_schedule(ctx, sched))) return rc;
    if (stages < 1 || stages > mmgap::kMaxStages)
        return fail(ctx, MMGAP_EUNSUPPORTED, "stages=%d outside 1..%d", stages, mmgap::kMaxStages);
    if (sh.n_inst == 0) return MMGAP_OK;
    if (!H || !y || !sym_out) return fail(ctx, MMGAP_EINVAL, "H, y and sym_out are required");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    // the move problem: two unit-weight spins per real dimension
    const int KT = sh.KT, NW = mmgap::spin_words(KT, 2), ni = sh.n_inst;
    Bump plan;
    const size_t oG = plan.take(sizeof(float) * (size_t)prob->n_sc * KT * KT);
    const size_t of = plan.take(sizeof(float) * (size_t)ni * KT);
    const size_t ofp = plan.take(sizeof(float) * (size_t)ni * KT);
    const size_t oxg = plan.take((size_t)ni * KT);
    const int lanes = search_lanes(ctx, prob, sh, sched);
    // the stage launches' zero move and chain states (not used by the one-launch search)
    const size_t oz = lanes ? 0 : plan.take((size_t)ni * KT);
    const size_t oE = lanes ? 0 : plan.take(sizeof(float) * (size_t)ni * sched->chains);
    const size_t oS = lanes ? 0 : plan.take(sizeof(uint32_t) * (size_t)ni * sched->chains * NW);
    if ((rc = ensure_scratch(ctx, plan.off))) return rc;
    if ((rc = begin_call(ctx, st))) return rc;
    prof_mark(ctx, 0, st);
    // the sliced MMSE estimate is the first guess
    rc = det_build_into(ctx, st, prob, sh, H, y, at<float>(ctx, oG), at<float>(ctx, of),
                        at<signed char>(ctx, oxg));
    if (rc) return rc;
    hipError_t e;
    if (guess) {
        e = mmgap::launch_pad_rows_i8(guess, at<signed char>(ctx, oxg), ni, sh.K, KT, st);
        if (e != hipSuccess) return hip_fail(ctx, e, "guess copy");
    }
    if (lanes) {
        rc = run_search(ctx, st, prob, sh, H, y, sched, stages, lanes, at<float>(ctx, oG),
                        at<float>(ctx, of), at<signed char>(ctx, oxg), nullptr, sym_out,
                        metric_out, nullptr);
        if (rc) return rc;
        return end_call(ctx, st);
    }
    e = mmgap::launch_fill_u8(at<signed char>(ctx, oz), 0, (size_t)ni * KT, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "zero-move fill");
    rc = run_delta_stages(ctx, st, prob, sh, H, y, sched, stages, sched->seed, at<float>(ctx, oG),
                          at<float>(ctx, of), at<float>(ctx, ofp), at<signed char>(ctx, oxg),
                          at<signed char>(ctx, oz), at<float>(ctx, oE), at<uint32_t>(ctx, oS),
                          true, sym_out, metric_out);
    if (rc) return rc;
    return end_call(ctx, st);
}

int mmgap_detect_sic(mmgap_ctx *ctx, const mmgap_problem *prob, const void *H, const void *y,
                     unsigned char *sym_out, float *metric_out, signed char *levels_out,
                     int *order_out, void *stream)
{
    if (!ctx) return MMGAP_EINVAL;
    ProblemShape sh;
    int rc = check_problem(ctx, prob, MMGAP_KIND_DET, &sh);
    if (rc) return rc;
    if (prob->n_tx > 16)
        return fail(ctx, MMGAP_EUNSUPPORTED, "MMSE-SIC supports n_tx <= 16 (got %d)", prob->n_tx);
    if (sh.n_inst == 0) return MMGAP_OK;
    if (!H || !y) return fail(ctx, MMGAP_EINVAL, "H and y are required");
    if (metric_out && !sym_out) return fail(ctx, MMGAP_EINVAL, "metric_out needs sym_out");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    if ((rc = begin_call(ctx, st))) return rc;
    mmgap::SicArgs a = sic_args(prob, sh, H, y);
    a.levels = levels_out;
    a.ldl = 2 * prob->n_tx;
    a.sym_out = sym_out;
    a.metric_out = metric_out;
    a.order_out = order_out;
    hipError_t e = mmgap::launch_sic(a, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "MMSE-SIC launch");
    return end_call(ctx, st);
}

int mmgap_detect_e(mmgap_ctx *ctx, const mmgap_problem *prob, const void *H, const void *y,
                   const mmgap_schedule *sched, int stages, int guesses, unsigned char *sym_out,
                   float *metric_out, unsigned char *from_sic_out, void *stream)
{
    if (!ctx) return MMGAP_EINVAL;
    ProblemShape sh;
    int rc = check_problem(ctx, prob, MMGAP_KIND_DET, &sh);
    if (rc) return rc;
    if ((rc = check_schedule(ctx, sched))) return rc;
    if (stages < 1 || stages > mmgap::kMaxStages)
        return fail(ctx, MMGAP_EUNSUPPORTED, "stages=%d outside 1..%d", stages, mmgap::kMaxStages);
    if (guesses < 1 || guesses > (MMGAP_GUESS_MMSE | MMGAP_GUESS_SIC))
        return fail(ctx, MMGAP_EINVAL, "guesses=%d is not a non-empty set of MMGAP_GUESS_*",
                    guesses);
    if (prob->n_tx > 16)
        return fail(ctx, MMGAP_EUNSUPPORTED, "MMSE-SIC supports n_tx <= 16 (got %d)", prob->n_tx);
    if (sh.n_inst == 0) return MMGAP_OK;
    if (!H || !y || !sym_out) return fail(ctx, MMGAP_EINVAL, "H, y and sym_out are required");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const bool use_a = guesses & MMGAP_GUESS_MMSE, use_b = guesses & MMGAP_GUESS_SIC;
    const int KT = sh.KT, NW = mmgap::spin_words(KT, 2), ni = sh.n_inst;
    // Through the stage launches each chain has its own move fields and chain
    // state, and with both guesses the MMSE-SIC guess and its chain run on the
    // context's second stream, beside the build and the chain from the MMSE
    // guess (paper section 5.3: the two guesses of MMGaP-E are independent).
    const bool both = use_a && use_b;
    Bump plan;
    const size_t oG = plan.take(sizeof(float) * (size_t)prob->n_sc * KT * KT);
    const size_t of = plan.take(sizeof(float) * (size_t)ni * KT);
    const size_t oxa = plan.take((size_t)ni * KT);
    const size_t oxb = plan.take((size_t)ni * KT);
    const size_t oz = plan.take((size_t)ni * KT);
    // the stage launches' per-chain move fields and chain states (not used by
    // the one-launch search)
    const int lanes = search_lanes(ctx, prob, sh, sched);
    size_t ofp[2] = {}, oE[2] = {}, oS[2] = {};
    for (int c = 0; c < (lanes ? 0 : both ? 2 : 1); ++c) {
        ofp[c] = plan.take(sizeof(float) * (size_t)ni * KT);
        oE[c] = plan.take(sizeof(float) * (size_t)ni * sched->chains);
        oS[c] = plan.take(sizeof(uint32_t) * (size_t)ni * sched->chains * NW);
    }
    if (!both) {
        ofp[1] = ofp[0];
        oE[1] = oE[0];
        oS[1] = oS[0];
    }
    if ((rc = ensure_scratch(ctx, plan.off))) return rc;
    if ((rc = begin_call(ctx, st))) return rc;
    prof_mark(ctx, 0, st);
    float *G = at<float>(ctx, oG), *f = at<float>(ctx, of);
    signed char *xa = at<signed char>(ctx, oxa), *xb = at<signed char>(ctx, oxb);
    signed char *zm = at<signed char>(ctx, oz);
    hipError_t e = hipSuccess;
    // with both chains through the stage launches the MMSE-SIC estimate goes to
    // the second stream, beside the build; otherwise the two latency-bound
    // kernels run faster one after the other on one stream (measured 0.39
    // against 0.44 ms for one chain on a 16x16 slot)
    const bool fork = both && !lanes;
    hipStream_t sb = fork ? ctx->aux : st;
    if (fork) {
        e = hipEventRecord(ctx->aux_ev[0], st);
        if (e == hipSuccess) e = hipStreamWaitEvent(sb, ctx->aux_ev[0], 0);
        if (e != hipSuccess) return hip_fail(ctx, e, "second stream");
    }
    if (use_b) {
        mmgap::SicArgs sa = sic_args(prob, sh, H, y);
        sa.levels = xb;
        sa.ldl = KT;
        e = mmgap::launch_sic(sa, sb);
        if (e != hipSuccess) return hip_fail(ctx, e, "MMSE-SIC launch");
    }
    // the MMSE estimate (the build's factorisation and solves) only for its chain
    if ((rc = det_build_into(ctx, st, prob, sh, H, y, G, f, use_a ? xa : nullptr))) return rc;
    if (lanes) {
        // both chains, the choice and the decode in one launch after the build
        // and the MMSE-SIC estimate
        rc = run_search(ctx, st, prob, sh, H, y, sched, stages, lanes, G, f,
                        use_a ? xa : nullptr, use_b ? xb : nullptr, sym_out, metric_out,
                        from_sic_out);
        if (rc) return rc;
        return end_call(ctx, st);
    }
    e = mmgap::launch_fill_u8(zm, 0, (size_t)ni * KT, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "zero-move fill");
    if (fork) {                   // the MMSE-SIC chain stays on the second stream
        e = hipEventRecord(ctx->aux_ev[1], st);
        if (e == hipSuccess) e = hipStreamWaitEvent(sb, ctx->aux_ev[1], 0);
        if (e != hipSuccess) return hip_fail(ctx, e, "second stream");
    }
    // the chain from the MMSE guess (keys seed + s) and the one from the
    // MMSE-SIC guess (keys seed + 64 + s); a single chain decodes its own answer
    if (use_a) {
        rc = run_delta_stages(ctx, st, prob, sh, H, y, sched, stages, sched->seed, G, f,
                              at<float>(ctx, ofp[0]), xa, zm, at<float>(ctx, oE[0]),
                              at<uint32_t>(ctx, oS[0]), !both, sym_out, metric_out);
        if (rc) return rc;
    }
    if (use_b) {
        rc = run_delta_stages(ctx, sb, prob, sh, H, y, sched, stages,
                              sched->seed + (uint64_t)mmgap::kMaxStages, G, f,
                              at<float>(ctx, ofp[1]), xb, zm, at<float>(ctx, oE[1]),
                              at<uint32_t>(ctx, oS[1]), !both, sym_out, metric_out);
        if (rc) return rc;
    }
    if (!both) {
        if (from_sic_out) {
            e = mmgap::launch_fill_u8(from_sic_out, use_b ? 1 : 0, (size_t)ni, st);
            if (e != hipSuccess) return hip_fail(ctx, e, "from_sic fill");
        }
        return end_call(ctx, st);
    }
    e = hipEventRecord(ctx->aux_ev[2], sb);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, ctx->aux_ev[2], 0);
    if (e != hipSuccess) return hip_fail(ctx, e, "second stream");
    mmgap::PickArgs pk{};
    pk.G = G;
    pk.inst_per_G = prob->n_sym;
    pk.f = f;
    pk.xa = xa;
    pk.xb = xb;
    pk.n_inst = ni;
    pk.K = sh.K;
    pk.KT = KT;
    pk.q = sh.q;
    pk.H = (const float2 *)H;
    pk.y = (const float2 *)y;
    pk.n_rows = prob->n_rx;
    pk.n_cols = prob->n_tx;
    pk.n_sym = prob->n_sym;
    pk.c = qam_c(prob->qam);
    pk.sym_out = sym_out;
    pk.metric_out = metric_out;
    pk.from_b = from_sic_out;
    e = mmgap::launch_pick(pk, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "pick launch");
    return end_call(ctx, st);
}

int mmgap_vpp_precode(mmgap_ctx *ctx, const mmgap_problem *prob, const void *H, const void *u,
                      const mmgap_schedule *sched, signed char *v_out, void *x_out,
                      float *gamma_out, void *stream)
{
    if (!ctx) return MMGAP_EINVAL;
    ProblemShape sh;
    int rc = check_problem(ctx, prob, MMGAP_KIND_VPP, &sh);
    if (rc) return rc;
    if ((rc = check_schedule(ctx, sched))) return rc;
    if (sh.n_inst == 0) return MMGAP_OK;
    if (!H || !u || !v_out) return fail(ctx, MMGAP_EINVAL, "H, u and v_out are required");
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    const int KT = sh.KT, NW = mmgap::spin_words(KT, sh.q), ni = sh.n_inst;
    const int nu = prob->n_rx;
    Bump plan;
    const size_t oG = plan.take(sizeof(float) * (size_t)prob->n_sc * KT * KT);
    const size_t of = plan.take(sizeof(float) * (size_t)ni * KT);
    const size_t ox = plan.take((size_t)ni * KT);
    const size_t oA = plan.take(sizeof(double2) * (size_t)prob->n_sc * nu * nu);
    const size_t oE = plan.take(sizeof(float) * (size_t)ni * sched->chains);
    const size_t oS = plan.take(sizeof(uint32_t) * (size_t)ni * sched->chains * NW);
    if ((rc = ensure_scratch(ctx, plan.off))) return rc;
    if ((rc = begin_call(ctx, st))) return rc;
    prof_mark(ctx, 0, st);
    mmgap::VppBuildArgs b{};
    b.H = (const float2 *)H;
    b.u = (const float2 *)u;
    b.n_sc = prob->n_sc;
    b.n_u = nu;
    b.n_t = prob->n_tx;
    b.n_sym = prob->n_sym;
    b.ld = KT;
    b.tau = vpp_tau(prob);
    b.G = at<float>(ctx, oG);
    b.f = at<float>(ctx, of);
    b.x_fb = at<signed char>(ctx, ox);
    b.Ainv = at<double2>(ctx, oA);
    b.unorm = nullptr;
    hipError_t e = mmgap::launch_vpp_build(b, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "build launch");
    int w[mmgap::kMaxQ];
    vpp_weights(w);
    mmgap::SelectArgs sel{};
    sel.mode = mmgap::kSelectVpp;
    sel.H = (const float2 *)H;
    sel.y = (const float2 *)u;
    sel.n_rows = nu;
    sel.n_cols = prob->n_tx;
    sel.n_sym = prob->n_sym;
    sel.Ainv = b.Ainv;
    sel.tau = b.tau;
    sel.v_out = v_out;
    sel.x_out = (float2 *)x_out;
    sel.gamma_out = gamma_out;
    rc = run_solver(ctx, st, ni, sh.K, sh.q, KT, w, b.G, prob->n_sym, b.f, b.x_fb, sched,
                    at<float>(ctx, oE), at<uint32_t>(ctx, oS), sel);
    if (rc) return rc;
    return end_call(ctx, st);
}

int mmgap_set_option(mmgap_ctx *ctx, int option, int value)
{
    if (!ctx) return MMGAP_EINVAL;
    if (option == MMGAP_OPT_STAGE_LAUNCHES && (value == 0 || value == 1)) {
        ctx->stage_launches = value != 0;
        return MMGAP_OK;
    }
    return fail(ctx, MMGAP_EINVAL, "unknown option %d or value %d", option, value);
}

int mmgap_set_profiling(mmgap_ctx *ctx, int enable)
{
    if (!ctx) return MMGAP_EINVAL;
    DeviceGuard g(ctx->device);
    if (enable && !ctx->prof_ev[0][0]) {
        for (int r = 0; r < kProfRing; ++r)
            for (int i = 0; i < 4; ++i) {
                hipError_t e = hipEventCreate(&ctx->prof_ev[r][i]);
                if (e != hipSuccess) return hip_fail(ctx, e, "hipEventCreate(profile)");
            }
    }
    ctx->profiling = enable != 0;
    ctx->prof_count = 0;
    ctx->prof_open = false;
    return MMGAP_OK;
}

int mmgap_last_profile(mmgap_ctx *ctx, float *ms, int capacity)
{
    if (!ctx) return MMGAP_EINVAL;
    if (!ms || capacity < 3) return fail(ctx, MMGAP_EINVAL, "ms needs room for 3 entries");
    if (!ctx->profiling || ctx->prof_count == 0)
        return fail(ctx, MMGAP_EINVAL, "no profiled call (enable with mmgap_set_profiling)");
    DeviceGuard g(ctx->device);
    long avail = ctx->prof_count < kProfRing ? ctx->prof_count : kProfRing;
    long n = capacity / 3 < avail ? capacity / 3 : avail;
    const long first = ctx->prof_count - n;
    for (long c = 0; c < n; ++c) {
        hipEvent_t *ev = ctx->prof_ev[(first + c) % kProfRing];
        hipError_t e = hipEventSynchronize(ev[3]);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipEventSynchronize(profile)");
        for (int i = 0; i < 3; ++i) {
            float v = 0.0f;
            e = hipEventElapsedTime(&v, ev[i], ev[i + 1]);
            if (e != hipSuccess) return hip_fail(ctx, e, "hipEventElapsedTime");
            ms[3 * c + i] = v;
        }
    }
    return (int)(3 * n);
}

int mmgap_plan_create(mmgap_ctx *ctx, int n_jobs, const mmgap_job *jobs, int flags, int blocks,
                      mmgap_plan **out)
{
    if (!ctx) return MMGAP_EINVAL;
    if (!out) return fail(ctx, MMGAP_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_jobs < 0 || (n_jobs > 0 && !jobs))
        return fail(ctx, MMGAP_EINVAL, "n_jobs=%d with jobs=%p", n_jobs, (const void *)jobs);
    if (flags & ~(MMGAP_PLAN_GRAPH | MMGAP_PLAN_PERSISTENT))
        return fail(ctx, MMGAP_EINVAL, "unknown flags 0x%x", flags);
    if (blocks < 0) return fail(ctx, MMGAP_EINVAL, "blocks=%d < 0", blocks);

    BatchLayout lay;
    int rc = batch_layout(ctx, n_jobs, jobs, flags, &lay);
    if (rc) return rc;
    if (lay.bytes + ctx->plan_bytes + ctx->scratch_bytes > ctx->budget)
        return fail(ctx, MMGAP_ENOMEM,
                    "plan of %zu bytes exceeds the HBM budget of %zu bytes (%zu in use)", lay.bytes,
                    ctx->budget, ctx->plan_bytes + ctx->scratch_bytes);

    DeviceGuard g(ctx->device);
    mmgap_plan *plan = new (std::nothrow) mmgap_plan();
    if (!plan) return fail(ctx, MMGAP_ENOMEM, "out of host memory");
    plan->ctx = ctx;
    plan->n_items = (int)lay.items.size();
    hipError_t e = hipMalloc(&plan->mem, lay.bytes);
    if (e != hipSuccess) {
        plan->mem = nullptr;
        plan_free(plan);
        return fail(ctx, MMGAP_ENOMEM, "hipMalloc(%zu): %s", lay.bytes, hipGetErrorString(e));
    }
    plan->bytes = lay.bytes;
    ctx->plan_bytes += lay.bytes;
    char *base = static_cast<char *>(plan->mem);
    if ((rc = batch_launch_config(ctx, lay, base, blocks, &plan->launch))) {
        plan_free(plan);
        return rc;
    }
    std::vector<unsigned char> image;
    batch_bind(lay, base, image);
    e = hipMemcpy(base, image.data(), image.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&plan->done, hipEventDisableTiming);
    if (e == hipSuccess && (flags & MMGAP_PLAN_GRAPH)) {
        hipStream_t cs = nullptr;
        e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e == hipSuccess) {
            e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                const hipError_t el = batch_enqueue(plan->launch, ctx->accept_dev, cs);
                e = hipStreamEndCapture(cs, &plan->graph);
                if (e == hipSuccess) e = el;
            }
            (void)hipStreamDestroy(cs);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
    }
    if (e != hipSuccess) {
        plan_free(plan);
        return hip_fail(ctx, e, "plan setup");
    }
    *out = plan;
    return MMGAP_OK;
}

int mmgap_plan_launch(mmgap_plan *plan, void *stream)
{
    if (!plan) return MMGAP_EINVAL;
    mmgap_ctx *ctx = plan->ctx;
    DeviceGuard g(ctx->device);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (plan->done_valid) e = hipStreamWaitEvent(st, plan->done, 0);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamWaitEvent");
    if (plan->exec) e = hipGraphLaunch(plan->exec, st);
    else e = batch_enqueue(plan->launch, ctx->accept_dev, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "fused launch");
    e = hipEventRecord(plan->done, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipEventRecord");
    plan->done_valid = true;
    return MMGAP_OK;
}

int mmgap_plan_info(const mmgap_plan *plan, int *n_items, int *blocks)
{
    if (!plan) return MMGAP_EINVAL;
    if (n_items) *n_items = plan->n_items;
    if (blocks)
        *blocks = std::max(plan->launch.blocks[0],
                           std::max(plan->launch.blocks[1], plan->launch.blocks[2]));
    return MMGAP_OK;
}

int mmgap_plan_destroy(mmgap_plan *plan)
{
    if (!plan) return MMGAP_OK;
    DeviceGuard g(plan->ctx->device);
    plan_free(plan);
    return MMGAP_OK;
}

}  // extern "C"
