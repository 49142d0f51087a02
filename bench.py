#!/usr/bin/env python3
"""Benchmark of the Ising hot path (ML-MIMO detection / VPP precoding) on one MI355X.

A step is one pass of the whole hot path -- Gram/field build, annealing,
selection and decode -- over every slot of the workload, on synthetic i.i.d.
Rayleigh channels (inputs resident in HBM before the timed region).  The
default workload is the uplink 16x16 64-QAM slot (3276 subcarriers x 12
symbols) at SNR 15, 20, 25 and 30 dB (common random numbers: the four slots
share channels, symbols and noise draw); each slot is launched and timed on
its own, so slot latencies are per slot.  Legs on the same inputs:
  * plain: the per-size entry points (one build, anneal and select launch per
    slot) at the workload's reference schedule -- the baseline;
  * fused: one persistent launch per slot (a batch plan replayed as a HIP
    graph) at the same schedule -- outputs must be identical to plain;
  * tuned: the fused launch at the schedules the offline tuner picked for each
    job's class and SNR bucket -- the binary encoding or moves around the MMSE
    guess in stages inside the persistent kernel;
  * delta_separate: the tuned moves-around-the-guess schedules through the
    multi-launch entry point (move fields, anneal, select per stage) -- must
    give the tuned leg's bytes;
  * beside them for detection: MMGaP-E (both guesses), MMSE-SIC alone, the
    search from the MMSE-SIC guess, the critical path of one subcarrier alone
    on the GPU, the build over 64 slots, and a bounded serving mix.
The reported value is the fastest leg whose quality on every slot -- symbol
error rate (detection) or mean transmit energy (VPP) -- is within 5% of the
plain leg's ("at matched SER").  The JSON line also carries slot latency
percentiles, the roofline position of the dominant kernel (VALU-bound) and
the CPU oracle timed on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Ising solves/sec + p99 slot latency vs plain launch, at matched SER"
# 32-bit VALU lane-operations per second: 256 CUs x 128 lane-ops per clock x 2.4 GHz,
# the rate the published FP32 vector peak (157.3 TFLOP/s = 78.6 T FMA/s) implies
PEAK_ALU_OPS = 256 * 128 * 2.4e9
PEAK_HBM = 8.0e12

N_SC, N_SYM = 3276, 12
QUALITY_TOL = 0.05           # matched SER: within 5% of the plain leg's


def _det(n_r, n_t, qam, chains, sweeps, snr, seed, init, n_sc=N_SC, n_sym=N_SYM,
         delta=(16, 12, 1), sic_delta=(16, 2, 1)):
    return dict(kind="det", rows=n_r, cols=n_t, qam=qam, n_sc=n_sc, n_sym=n_sym, chains=chains,
                sweeps=sweeps, snr=snr, seed=seed, init=init, delta=delta, sic_delta=sic_delta)


def _vpp(n_u, n_t, qam, chains, sweeps, seed, n_sc=N_SC, n_sym=N_SYM):
    return dict(kind="vpp", rows=n_u, cols=n_t, qam=qam, n_sc=n_sc, n_sym=n_sym, chains=chains,
                sweeps=sweeps, snr=None, seed=seed, init=0)


# Each workload is a list of groups; a group is one slot launch (its jobs share
# the launch).  Reference schedules: 4x4 32x100, 8x8 64x200, 16x16 128x400;
# 64-QAM anneals start from the MMSE fallback (random starts stay trapped with
# binary weights).
WORKLOADS = {
    # the target configuration: 16x16 64-QAM slots over the SNR grid
    "det-16x16-64qam": [[_det(16, 16, 64, 128, 400, s, 3001, 1)] for s in (15.0, 20.0, 25.0, 30.0)],
    "det-8x8-16qam": [[_det(8, 8, 16, 64, 200, s, 2001, 0)] for s in (5.0, 10.0, 15.0, 20.0, 25.0)],
    # the paper's high-connectivity case: 32x32, 10 MHz at 30 kHz (24 resource
    # blocks = 288 subcarriers), 16-QAM, 128 anneals; plain path only (the
    # persistent kernel has no 64-dimension variant)
    "det-32x32-16qam": [[_det(32, 32, 16, 128, 100, 15.0, 3501, 0, n_sc=288)]],
    "det-4x4-qpsk": [[_det(4, 4, 4, 32, 100, 10.0, 0, 0, n_sc=64, n_sym=1)]],
    # downlink VPP, two sizes batched in one launch
    "vpp-8x8+16x16-16qam": [[_vpp(8, 8, 16, 64, 200, 4001), _vpp(16, 16, 16, 128, 400, 4002)]],
}


def qbits(qam: int) -> int:
    return {4: 1, 16: 2, 64: 3}[qam]


def job_shape(j):
    """(K, q, instances, flip attempts per slot) of a job at its reference schedule."""
    if j["kind"] == "det":
        K, q = 2 * j["cols"], qbits(j["qam"])
    else:
        K, q = 2 * j["rows"], 2
    n = j["n_sc"] * j["n_sym"]
    return K, q, n, float(n) * j["chains"] * j["sweeps"] * K * q


def ops_per_attempt(K: int, q: int) -> float:
    """Algorithmic 32-bit lane operations of one flip attempt: Philox4x32-10
    share 7.5 (10 rounds x (2 wide multiplies + 4 XOR) per 8 draws), draw
    extraction 1, energy change and scaling 3, threshold index and compare 3,
    state update 4, and the per-visit field row K/q (K fused multiply-adds per
    dimension, shared by its q attempts)."""
    return 18.5 + K / q


def sched_work(j, sc):
    """(flip attempts, algorithmic lane operations) of one job's anneals under
    schedule sc; moves around a guess anneal two unit-weight spins per real
    dimension in each stage."""
    K, q, n, _ = job_shape(j)
    st = sc.get("stages", 0)
    if st:
        q = 2
    a = float(n) * sc["chains"] * sc["sweeps"] * K * q * max(st, 1)
    if sc.get("guesses", 0) == 3:          # MMGaP-E: a search from each guess
        a *= 2
    return a, a * ops_per_attempt(K, q)


def guess_arg(sc) -> int:
    """det_job's guesses for a schedule: 0 unless it searches from the MMSE-SIC
    guess (alone or in MMGaP-E)."""
    g = sc.get("guesses", 0)
    return g if g > 1 else 0


def sched_desc(s) -> str:
    g = s.get("guesses", 0)
    if not g:
        return f"{s['chains']} chains x {s['sweeps']} sweeps, " \
               f"{'fallback' if s['init'] else 'random'} start"
    src = {1: "around the MMSE guess", 2: "around the MMSE-SIC guess",
           3: "from both guesses, better answer (MMGaP-E)"}[g]
    return f"{s['chains']} chains x {s['sweeps']} sweeps x {s['stages']} stage(s) {src}"


def levels_to_symbols(lv: np.ndarray, qam: int) -> np.ndarray:
    q = qbits(qam)
    n_t = lv.shape[-1] // 2
    top = (1 << q) - 1
    pI = (lv[..., :n_t].astype(np.int64) + top) // 2
    pQ = (lv[..., n_t:].astype(np.int64) + top) // 2
    return (((pI ^ (pI >> 1)) << q) | (pQ ^ (pQ >> 1))).astype(np.uint8)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for fn in ("kernels.hip", "kernels.h"):
        with open(os.path.join(ROOT, "paper_2510_01579_amd", "csrc", fn), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source; else None."""
    fn = os.path.join(ROOT, "profiles", "anneal_traffic.json")
    if not os.path.exists(fn):
        return None
    with open(fn) as fh:
        rec = json.load(fh).get(f"{workload}/{kernel}")
    if not rec or rec.get("kernel_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def make_inputs(specs):
    from workload import synth as W
    out = []
    for j in specs:
        if j["kind"] == "det":
            d = W.det_slot(j["seed"], j["rows"], j["cols"], j["qam"], j["n_sc"], j["n_sym"],
                           j["snr"])
            beta2 = W.linear_beta2(j["sweeps"], *W.det_beta_range(j["qam"], j["rows"],
                                                                  d.noise_var))
            out.append(dict(spec=j, raw=d, H=d.H, y=d.y, noise_var=d.noise_var, beta2=beta2,
                            seed=W.job_seed(j["seed"])))
        else:
            s = W.vpp_slot(j["seed"], j["rows"], j["cols"], j["qam"], j["n_sc"], j["n_sym"])
            beta2 = W.linear_beta2(j["sweeps"], *W.vpp_beta_range(j["qam"], j["cols"]))
            out.append(dict(spec=j, raw=s, H=s.H, y=s.u, noise_var=0.0, beta2=beta2,
                            seed=W.job_seed(j["seed"])))
    return out


def cpu_baseline(inputs, scheds, target_s: float, cim=None):
    """The oracle as it stands, on a bounded random sample of the workload's
    instances (spread over its jobs in proportion to their instance counts),
    with the schedules of the reported leg."""
    from oracle import oracle as O
    threads = O.max_threads()
    rng = np.random.default_rng(1)
    sizes = [job_shape(inp["spec"])[2] for inp in inputs]
    total = sum(sizes)

    def run(frac):
        n_done = 0
        t0 = time.perf_counter()
        for inp, sc, n_all in zip(inputs, scheds, sizes):
            j = inp["spec"]
            m = max(1, min(n_all, int(round(frac * n_all))))
            ids = np.sort(rng.choice(n_all, m, replace=False)).astype(np.uint32)
            if j["kind"] == "det" and sc.get("guesses", 0) > 1:
                O.detect_e(inp["H"], inp["y"], inp["noise_var"], j["qam"], sc["chains"],
                           sc["sweeps"], sc["beta2"], inp["seed"], stages=sc["stages"],
                           inst_ids=ids, init_mode=sc["init"], cim=cim, guesses=sc["guesses"])
            elif j["kind"] == "det" and sc.get("stages"):
                O.detect_delta(inp["H"], inp["y"], inp["noise_var"], j["qam"], sc["chains"],
                               sc["sweeps"], sc["beta2"], inp["seed"], stages=sc["stages"],
                               inst_ids=ids, init_mode=sc["init"], cim=cim)
            elif j["kind"] == "det":
                O.detect(inp["H"], inp["y"], inp["noise_var"], j["qam"], sc["chains"],
                         sc["sweeps"], sc["beta2"], inp["seed"], inst_ids=ids,
                         init_mode=sc["init"], cim=cim)
            else:
                O.vpp_precode(inp["H"], inp["y"], j["qam"], sc["chains"], sc["sweeps"],
                              sc["beta2"], inp["seed"], inst_ids=ids, init_mode=sc["init"],
                              cim=cim)
            n_done += m
        return n_done, time.perf_counter() - t0

    n0, t_probe = run(min(1.0, 8.0 * threads / total))
    frac = min(1.0, target_s / max(t_probe, 1e-6) * n0 / total)
    n, dt = run(frac)
    return {"value": n / dt, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} of {total} instances of the same slot(s) (random subset), "
                      f"same schedules as the reported leg, {dt:.1f} s on {threads} threads"}


# serving mix: slot jobs, 60% detection / 40% VPP, sizes {8x8, 16x16},
# modulations {QPSK, 16-QAM, 64-QAM} uniform, SNR uniform 5-30 dB (detection)
SERVE_RATE = 2000.0          # offered slots per second
SERVE_DEADLINE_MS = 0.5      # one slot


def serve_classes():
    return [(kind, n, qam) for kind in ("det", "vpp") for n in (8, 16) for qam in (4, 16, 64)]


def serve_mix(M, torch, n_sat: int, n_arr: int, n_full: int):
    """The native serving loop on a stream of slot jobs drawn from the mix, with
    the tuner's schedules (moves around the MMSE guess where the tuner chose
    them).  Three phases: every job queued at once (the sustainable slot rate),
    Poisson arrivals at min(2000/s, 0.8 x sustainable), and a burst at the full
    2000/s.  Latency = submission to observed completion."""
    from workload import synth as W
    rng = np.random.default_rng(5)
    dev = torch.device("cuda", 0)
    ctx = M.Context(0)
    classes = serve_classes()
    pool = {}
    for ci, (kind, n, qam) in enumerate(classes):
        for r in range(2):
            seed = 6000 + 10 * ci + r
            if kind == "det":
                snr = float(rng.uniform(5.0, 30.0))
                d = W.det_slot(seed, n, n, qam, N_SC, N_SYM, snr)
                pool[(ci, r)] = dict(H=torch.from_numpy(d.H).to(dev),
                                     y=torch.from_numpy(d.y).to(dev), nv=d.noise_var,
                                     sched=M.tuned_schedule(M.KIND_DET, n, n, qam, d.noise_var))
            else:
                sl = W.vpp_slot(seed, n, n, qam, N_SC, N_SYM)
                pool[(ci, r)] = dict(H=torch.from_numpy(sl.H).to(dev),
                                     y=torch.from_numpy(sl.u).to(dev), nv=0.0,
                                     sched=M.tuned_schedule(M.KIND_VPP, n, n, qam))
    torch.cuda.synchronize()

    def draw_job(k):
        kind = "det" if rng.random() < 0.6 else "vpp"
        n = int(rng.choice([8, 16]))
        qam = int(rng.choice([4, 16, 64]))
        ci = classes.index((kind, n, qam))
        p = pool[(ci, int(rng.integers(2)))]
        sc = p["sched"]
        if kind == "det":
            return ctx.det_job(p["H"], p["y"], qam, p["nv"], sc["chains"], sc["sweeps"],
                               sc["beta2"], W.job_seed(k), init=sc["init"], metric=False,
                               stages=sc["stages"], guesses=guess_arg(sc))
        return ctx.vpp_job(p["H"], p["y"], qam, sc["chains"], sc["sweeps"], sc["beta2"],
                           W.job_seed(k), want_x=False, want_gamma=False, init=sc["init"])

    def arrivals(rate, n, base):
        gaps = rng.exponential(1.0 / rate, size=n)
        jobs = [draw_job(base + k) for k in range(n)]
        torch.cuda.synchronize()
        ctx.server_stats(SERVE_DEADLINE_MS, reset=True)     # a new accounting period
        ids = []
        t0 = time.perf_counter()
        t_next = t0
        for k in range(n):
            t_next += gaps[k]
            while time.perf_counter() < t_next:
                pass
            ids.append(ctx.server_submit(jobs[k]))
        ctx.server_drain()
        el = time.perf_counter() - t0
        lat = np.array([ctx.server_poll(i)[1] for i in ids]) / 1e3
        return lat, el, ctx.server_stats(SERVE_DEADLINE_MS)

    ctx.server_start(max_inflight=3, arena_bytes=2 << 30)
    try:
        ids = [ctx.server_submit(draw_job(k)) for k in range(6)]       # warmup
        ctx.server_drain()
        for i in ids:
            ctx.server_poll(i)
        jobs = [draw_job(100 + k) for k in range(n_sat)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ids = [ctx.server_submit(j) for j in jobs]
        ctx.server_drain()
        makespan = time.perf_counter() - t0
        for i in ids:
            ctx.server_poll(i)
        sustainable = n_sat / makespan
        rate = min(SERVE_RATE, 0.8 * sustainable)
        lat, elapsed, acct = arrivals(rate, n_arr, 1000)
        lat_full, _, acct_full = arrivals(SERVE_RATE, n_full, 5000)
    finally:
        ctx.server_stop()
        ctx.close()
    return {
        "workload": "slot jobs of 3276 subcarriers x 12 symbols, 60% uplink detection / 40% "
                    "VPP, sizes 8x8 and 16x16, QPSK/16-QAM/64-QAM uniform, detection SNR "
                    "uniform 5-30 dB, i.i.d. Rayleigh; tuned schedules (searches around a "
                    "guess and MMGaP-E where the tuner chose them)",
        "path": "native serving loop: FIFO admission into an HBM arena, batches recorded as "
                "HIP graphs on 3 streams (search launches for jobs that search around a "
                "guess, the persistent fused kernels for the rest)",
        "sustainable_slots_per_s": sustainable,
        "sustainable_solves_per_s": sustainable * N_SC * N_SYM,
        "saturation_jobs": n_sat,
        "offered_slots_per_s": rate,
        "arrivals": n_arr,
        "arrival_window_s": elapsed,
        "p50_slot_ms": float(np.percentile(lat, 50)),
        "p99_slot_ms": float(np.percentile(lat, 99)),
        "deadline_ms": SERVE_DEADLINE_MS,
        "frac_within_deadline": float(np.mean(lat <= SERVE_DEADLINE_MS)),
        "deadline_misses": acct["missed"],
        "server_accounting": acct,
        "at_target_rate": {"slots_per_s": SERVE_RATE, "arrivals": n_full,
                           "p50_slot_ms": float(np.percentile(lat_full, 50)),
                           "p99_slot_ms": float(np.percentile(lat_full, 99)),
                           "frac_within_deadline": float(np.mean(lat_full <= SERVE_DEADLINE_MS)),
                           "deadline_misses": acct_full["missed"],
                           "server_accounting": acct_full},
    }


def run_serving(args, M, torch):
    """The serving mix as its own benchmark line (--workload serve-mix)."""
    n_sat = max(args.steps, 12)
    res = serve_mix(M, torch, n_sat, max(args.steps * 2, 20), max(args.steps, 20))
    return {
        "metric": METRIC, "value": res["sustainable_solves_per_s"], "unit": "solves/s",
        "n_gpus": 1, "steps": n_sat, "warmup": 6,
        "ms_per_step": 1e3 / res["sustainable_slots_per_s"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "serving mix: " + res["workload"], "name": "serve-mix",
                   "path": res["path"]},
        "p50_slot_ms": res["p50_slot_ms"], "p99_slot_ms": res["p99_slot_ms"],
        "serve_mix": res, "roofline": None, "cpu_baseline": None,
    }


def build_bytes(j, n_sc=None) -> float:
    """Algorithmic HBM bytes of the detection build of one job (unpadded
    outputs, as mmgap_build_ising writes them): H and y in, couplings
    [n_sc][K][K] float32, fields [n][K] float32 and fallbacks [n][K] int8 out."""
    K = 2 * j["cols"]
    n_sc = j["n_sc"] if n_sc is None else n_sc
    n = n_sc * j["n_sym"]
    h = n_sc * j["rows"] * j["cols"] * 8
    y = n * j["rows"] * 8
    return float(h + y + n_sc * K * K * 4 + n * K * 4 + n * K)


def quality(inputs, outs):
    """Per job: symbol error rate (detection) or mean transmit energy (VPP)."""
    res = []
    for inp, o in zip(inputs, outs):
        j = inp["spec"]
        n = j["n_sc"] * j["n_sym"]
        if j["kind"] == "det":
            truth = inp["raw"].sym.reshape(n, j["cols"])
            res.append(float(np.mean(o["sym"] != truth)))
        else:
            res.append(float(np.mean(o["gamma"].astype(np.float64))))
    return res


def matched(q, ref):
    return all(a <= (1.0 + QUALITY_TOL) * b + 2e-5 for a, b in zip(q, ref))


def cim_ops_per_step(K: int, q: int, f_mvm: int) -> float:
    """Algorithmic 32-bit lane operations of one CIM-CAC Euler step of one
    anneal with N = K q spins and the auxiliary one: the update of every
    amplitude and error variable, 15 operations each (square, linear and cubic
    terms, drift, gain, push, step, amplitude sum; shifted square, product,
    scaling, step, sum, floor), and, every f_mvm steps, the coupling terms --
    K q for the levels, K^2 for the K x K product, 7 per spin and K for the
    auxiliary spin."""
    N = K * q
    return 15.0 * (N + 1) + (K * q + K * K + 7.0 * N + K) / f_mvm


def run_cim(args, M, torch):
    """CIM-CAC leg (the paper's own anneal dynamics) on the plain path:
    `chains` anneals of M.CIM_STEPS Euler steps with the default constants per
    problem -- of the binary encoding where it has at most 64 spins, else (the
    16-user 64-QAM slots) of the moves around the sliced MMSE estimate, the
    paper's own formulation (one stage, 64 spins and the auxiliary one) --
    with the Metropolis plain leg at the reference schedule beside it for
    quality."""
    specs = [j for g in WORKLOADS[args.workload] for j in g]
    moves = []
    for j in specs:
        K, q = job_shape(j)[:2]
        KT = 8 if K <= 8 else (16 if K <= 16 else 32)
        if K > 32:
            raise SystemExit(f"--dynamics cim needs at most 32 real dimensions ({args.workload})")
        moves.append(j["kind"] == "det" and KT * q > 64)
    inputs = make_inputs(specs)
    dev = torch.device("cuda", 0)
    for inp in inputs:
        inp["H_d"] = torch.from_numpy(inp["H"]).to(dev)
        inp["y_d"] = torch.from_numpy(inp["y"]).to(dev)
    ctx = M.Context(0)
    chains, steps = args.cim_chains, M.CIM_STEPS
    cim = dict(M.CIM_DEFAULTS)

    def step(use_cim):
        outs = []
        for inp, mv in zip(inputs, moves):
            j = inp["spec"]
            ch, sw, b2, kw = (chains, steps, None, dict(cim=cim)) if use_cim else \
                (j["chains"], j["sweeps"], inp["beta2"], {})
            if use_cim and mv:
                outs.append(ctx.detect_delta(inp["H_d"], inp["y_d"], j["qam"], inp["noise_var"],
                                             ch, sw, None, inp["seed"], stages=1, **kw))
            elif j["kind"] == "det":
                outs.append(ctx.detect(inp["H_d"], inp["y_d"], j["qam"], inp["noise_var"], ch, sw,
                                       b2, inp["seed"], init=0 if use_cim else j["init"], **kw))
            else:
                outs.append(ctx.vpp_precode(inp["H_d"], inp["y_d"], j["qam"], ch, sw, b2,
                                            inp["seed"], **kw))
        return outs

    def timed(use_cim):
        for _ in range(args.warmup):
            step(use_cim)
        ctx.set_profiling(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(use_cim)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = np.array(ctx.profile(args.steps * len(inputs))).reshape(args.steps, len(inputs), 3)
        ctx.set_profiling(False)
        outs = step(use_cim)
        torch.cuda.synchronize()
        res = []
        for inp, o in zip(inputs, outs):
            names = ("sym", "metric") if inp["spec"]["kind"] == "det" else ("v", "x", "gamma")
            res.append({k: t.cpu().numpy() for k, t in zip(names, o)})
        return el, prof, res

    total_inst = sum(job_shape(i["spec"])[2] for i in inputs)
    c_el, c_prof, c_out = timed(True)
    m_el, m_prof, m_out = timed(False)
    anneal_ms = float(np.mean(c_prof[:, :, 1].sum(axis=1)))
    ops = 0.0
    for inp, mv in zip(inputs, moves):
        K, q, n = job_shape(inp["spec"])[:3]
        ops += n * chains * steps * cim_ops_per_step(K, 2 if mv else q, cim["f_mvm"])
    achieved = ops / (anneal_ms * 1e-3) / 1e12
    cpu = None
    if not args.no_cpu_baseline:
        scheds = [dict(chains=chains, sweeps=steps, beta2=None, init=0,
                       **(dict(stages=1, guesses=1) if mv else {})) for mv in moves]
        cpu = cpu_baseline(inputs, scheds, args.cpu_seconds, cim=cim)
    ctx.close()
    return {
        "metric": METRIC + " (CIM-CAC dynamics)",
        "value": args.steps * total_inst / c_el, "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": c_el / args.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "dynamics": "CIM-CAC",
                   "path": "plain: build, CIM-CAC anneal and select launches per slot" +
                           ("; moves around the MMSE guess (one stage) where the binary "
                            "encoding has more than 64 spins" if any(moves) else ""),
                   "schedule": f"{chains} anneals x {steps} Euler steps",
                   "constants": cim, "instances_per_step": total_inst},
        "stage_ms": {"build": float(np.mean(c_prof[:, :, 0].sum(axis=1))),
                     "anneal": anneal_ms,
                     "select": float(np.mean(c_prof[:, :, 2].sum(axis=1)))},
        "quality": quality(inputs, c_out),
        "metropolis_reference": {"ms_per_step": m_el / args.steps * 1e3,
                                 "value": args.steps * total_inst / m_el,
                                 "quality": quality(inputs, m_out)},
        "roofline": {"bound": "alu", "kernel": "k_cim", "achieved": achieved,
                     "peak": PEAK_ALU_OPS / 1e12, "unit": "T lane-ops/s",
                     "frac": achieved * 1e12 / PEAK_ALU_OPS,
                     "traffic": None, "kernel_ms": anneal_ms,
                     "ops_per_launch": ops},
        "cpu_baseline": cpu,
    }


def pct(lat):
    lat = np.asarray(lat, np.float64)
    return {"p50_slot_ms": float(np.percentile(lat, 50)),
            "p99_slot_ms": float(np.percentile(lat, 99))}


def main(argv=None) -> int:  # noqa: C901
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="det-16x16-64qam",
                    choices=sorted(WORKLOADS) + ["serve-mix"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--dynamics", choices=("metropolis", "cim"), default="metropolis",
                    help="cim: time the CIM-CAC anneals on the plain path instead")
    ap.add_argument("--cim-chains", type=int, default=32, help="anneals per instance (cim)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain leg")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip MMGaP-E, MMSE-SIC, critical path, 64-slot build, serving mix")
    ap.add_argument("--no-serve", action="store_true", help="skip the bounded serving mix")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy three times, so that "
                         "hardware counters of a kernel of known traffic can be read")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the hot path shards by subcarrier with no "
              "exchange, and it runs one GPU at a time (use --gpus 1)",
              file=sys.stderr)
        return 2

    import torch

    import paper_2510_01579_amd as M
    from workload import synth as W

    if args.dynamics == "cim":
        print(json.dumps(run_cim(args, M, torch)), flush=True)
        return 0
    if args.workload == "serve-mix":
        print(json.dumps(run_serving(args, M, torch)), flush=True)
        return 0

    groups = WORKLOADS[args.workload]
    specs = [j for g in groups for j in g]
    inputs = make_inputs(specs)
    gidx = []                                   # input indices of each group
    k = 0
    for g in groups:
        gidx.append(list(range(k, k + len(g))))
        k += len(g)
    dev = torch.device("cuda", 0)
    for inp in inputs:
        inp["H_d"] = torch.from_numpy(inp["H"]).to(dev)
        inp["y_d"] = torch.from_numpy(inp["y"]).to(dev)
    ctx = M.Context(0)
    total_inst = sum(job_shape(i["spec"])[2] for i in inputs)
    is_det = all(j["kind"] == "det" for j in specs)
    print(f"[bench] workload {args.workload}: {len(groups)} slot launches per step, "
          f"{total_inst} instances", file=sys.stderr, flush=True)

    def records_per_step(launch_group):
        """Profiled calls the library records in one pass over every group (one
        per anneal launch of the stage launches; one per search launch)."""
        ctx.set_profiling(True)
        for gi in range(len(groups)):
            launch_group(gi)
        torch.cuda.synchronize()
        n = len(ctx.profile(256))
        ctx.set_profiling(False)
        return n

    def timed(launch_group):
        """W warmup steps, then K timed steps; one HIP event pair around each
        group's launch on the current stream.  Returns (elapsed s, [K][G] ms)."""
        for _ in range(args.warmup):
            for gi in range(len(groups)):
                launch_group(gi)
        ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in groups] for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for st in range(args.steps):
            for gi in range(len(groups)):
                ev[st][gi][0].record()
                launch_group(gi)
                ev[st][gi][1].record()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        lat = np.array([[a.elapsed_time(b) for a, b in row] for row in ev])
        return el, lat

    def leg_record(el, lat, q, extra=None):
        rec = {"value": args.steps * total_inst / el, "unit": "solves/s",
               "ms_per_step": el / args.steps * 1e3, **pct(lat.reshape(-1)),
               "slot_ms_mean": [float(v) for v in lat.mean(axis=0)], "quality": q}
        rec.update(extra or {})
        return rec

    def host_outs(outs):
        return [{k: (None if t is None else t.cpu().numpy()) for k, t in o.items()}
                for o in outs]

    def fused_leg(scheds, graph=True, one_plan=False, blocks=0, persistent=True):
        """One plan (a HIP graph unless graph=False) per group with the given
        schedules per job; one_plan: every group's jobs in one plan, launched
        once per step; blocks: the plan's grid (0: the library's choice);
        persistent: every job on the persistent kernels, else jobs with stages
        take the build and search launches inside the plan."""
        plans, jobs = [], []
        for g in ([sum(gidx, [])] if one_plan else gidx):
            gj = []
            for i in g:
                inp, sc, j = inputs[i], scheds[i], inputs[i]["spec"]
                if j["kind"] == "det":
                    gj.append(ctx.det_job(inp["H_d"], inp["y_d"], j["qam"], inp["noise_var"],
                                          sc["chains"], sc["sweeps"], sc["beta2"], inp["seed"],
                                          init=sc["init"], stages=sc.get("stages", 0),
                                          guesses=guess_arg(sc)))
                else:
                    gj.append(ctx.vpp_job(inp["H_d"], inp["y_d"], j["qam"], sc["chains"],
                                          sc["sweeps"], sc["beta2"], inp["seed"],
                                          init=sc["init"]))
            plans.append(ctx.plan_create(gj, graph=graph, blocks=blocks, persistent=persistent))
            jobs.extend(gj)
        info = [p.plan_info() for p in plans]
        if one_plan:
            el, lat = timed(lambda gi: plans[0].plan_launch() if gi == 0 else None)
        else:
            el, lat = timed(lambda gi: plans[gi].plan_launch())
        torch.cuda.synchronize()
        outs = host_outs([jb["outputs"] for jb in jobs])
        for p in plans:
            p.plan_destroy()
        return el, lat, outs, info

    def same_bytes(a, b, keys):
        return all(x[k] is None and y[k] is None or x[k].tobytes() == y[k].tobytes()
                   for x, y in zip(a, b) for k in keys if k in x and k in y)

    ref_scheds = [dict(chains=i["spec"]["chains"], sweeps=i["spec"]["sweeps"],
                       init=i["spec"]["init"], beta2=i["beta2"], stages=0) for i in inputs]
    fusable = all(job_shape(j)[0] <= 32 for j in specs)
    legs = {}

    # ---- plain: per-size build, anneal and select launches, reference schedule
    plain = None
    q_ref = None
    if not args.no_plain or not fusable:
        def plain_group(gi):
            outs = []
            for i in gidx[gi]:
                inp, j = inputs[i], inputs[i]["spec"]
                if j["kind"] == "det":
                    o = ctx.detect(inp["H_d"], inp["y_d"], j["qam"], inp["noise_var"],
                                   j["chains"], j["sweeps"], inp["beta2"], inp["seed"],
                                   init=j["init"])
                    outs.append(dict(sym=o[0], metric=o[1]))
                else:
                    o = ctx.vpp_precode(inp["H_d"], inp["y_d"], j["qam"], j["chains"],
                                        j["sweeps"], inp["beta2"], inp["seed"])
                    outs.append(dict(v=o[0], x=o[1], gamma=o[2]))
            return outs

        print("[bench] plain leg", file=sys.stderr, flush=True)
        ctx.set_profiling(True)
        el, lat = timed(plain_group)
        prof = np.array(ctx.profile(args.steps * len(specs))).reshape(args.steps, len(specs), 3)
        ctx.set_profiling(False)
        p_out = host_outs([o for gi in range(len(groups)) for o in plain_group(gi)])
        q_ref = quality(inputs, p_out)
        plain = leg_record(el, lat, q_ref, {
            "schedule": "reference",
            "stage_ms": {"build": float(np.mean(prof[:, :, 0].sum(axis=1))),
                         "anneal": float(np.mean(prof[:, :, 1].sum(axis=1))),
                         "select": float(np.mean(prof[:, :, 2].sum(axis=1)))}})
        legs["plain"] = (el, lat, ref_scheds)

    # ---- fused: the same schedule in one persistent launch per slot
    fused = None
    if fusable:
        print("[bench] fused leg", file=sys.stderr, flush=True)
        el, lat, f_out, info = fused_leg(ref_scheds)
        q_f = quality(inputs, f_out)
        if q_ref is None:
            q_ref = q_f
        fused = leg_record(el, lat, q_f, {
            "work_items": [a for a, _ in info], "workgroups": [b for _, b in info],
            "outputs_identical_to_plain": None if plain is None else
            same_bytes(p_out, f_out, ("sym", "metric", "v", "x", "gamma"))})
        legs["fused"] = (el, lat, ref_scheds)

    # ---- tuned: the tuner's schedule per job (binary encoding or stages); the
    # persistent leg where every job fits the persistent kernels
    tuned = None
    t_scheds = None
    t_out = None
    if fusable or is_det:
        t_scheds = []
        for inp in inputs:
            j = inp["spec"]
            kind = M.KIND_DET if j["kind"] == "det" else M.KIND_VPP
            ts = M.tuned_schedule(kind, j["rows"], j["cols"], j["qam"], inp["noise_var"])
            t_scheds.append(ts if ts["tuned"] else ref_scheds[len(t_scheds)])
    if fusable:
        print("[bench] tuned leg", file=sys.stderr, flush=True)
        el, lat, t_out, _ = fused_leg(t_scheds)
        t_out_ref = t_out
        q_t = quality(inputs, t_out)
        tuned = leg_record(el, lat, q_t, {
            "schedules": [sched_desc(s) for s in t_scheds],
            "quality_matched": matched(q_t, q_ref)})
        legs["tuned"] = (el, lat, t_scheds)

    # ---- the tuned stages through the multi-launch entry point
    delta_sep = None
    if t_scheds is not None and is_det and all(s.get("stages") and s.get("guesses", 1) <= 1
                                               for s in t_scheds):
        def delta_group(gi):
            outs = []
            for i in gidx[gi]:
                inp, sc, j = inputs[i], t_scheds[i], inputs[i]["spec"]
                o = ctx.detect_delta(inp["H_d"], inp["y_d"], j["qam"], inp["noise_var"],
                                     sc["chains"], sc["sweeps"], sc["beta2"], inp["seed"],
                                     stages=sc["stages"], init=sc["init"])
                outs.append(dict(sym=o[0], metric=o[1]))
            return outs

        print("[bench] delta leg (separate launches)", file=sys.stderr, flush=True)
        n_stage = records_per_step(delta_group)
        ctx.set_profiling(True)
        el, lat = timed(delta_group)
        md = max(1, min(args.steps, 256 // n_stage))      # the library keeps 256 records
        dprof = np.array(ctx.profile(md * n_stage)).reshape(md, n_stage, 3)
        ctx.set_profiling(False)
        d_out = host_outs([o for gi in range(len(groups)) for o in delta_group(gi)])
        q_d = quality(inputs, d_out)
        delta_sep = leg_record(el, lat, q_d, {
            "stage_ms": {"build": float(np.mean(dprof[:, :, 0].sum(axis=1))),
                         "anneal": float(np.mean(dprof[:, :, 1].sum(axis=1))),
                         "select": float(np.mean(dprof[:, :, 2].sum(axis=1)))},
            "outputs_identical_to_tuned": None if t_out is None else
            same_bytes(d_out, t_out, ("sym", "metric")),
            "quality_matched": matched(q_d, q_ref)})
        legs["delta_separate"] = (el, lat, t_scheds)

    # ---- the tuner's choice among every formulation (MMGaP-E and the MMSE-SIC
    # guess included) through the separate-launch entry points
    tuned_sep = None
    tuned_plan = None
    stage_launch_ms = None
    if t_scheds is not None and is_det:
        a_scheds = []
        for inp, ts in zip(inputs, t_scheds):
            j = inp["spec"]
            sa = M.tuned_schedule(M.KIND_DET, j["rows"], j["cols"], j["qam"], inp["noise_var"],
                                  any_formulation=True)
            a_scheds.append(sa if sa["tuned"] else ts)
        # (also every tuned formulation of jobs the persistent kernels cannot take)
        if any(s.get("guesses", 0) > 1 for s in a_scheds) or not fusable:
            def sep_group(gi):
                outs = []
                for i in gidx[gi]:
                    inp, sc, j = inputs[i], a_scheds[i], inputs[i]["spec"]
                    g = sc.get("guesses", 0)
                    if g > 1:
                        o = ctx.detect_e(inp["H_d"], inp["y_d"], j["qam"], inp["noise_var"],
                                         sc["chains"], sc["sweeps"], sc["beta2"], inp["seed"],
                                         stages=sc["stages"], init=sc["init"], guesses=g)
                    elif sc.get("stages"):
                        o = ctx.detect_delta(inp["H_d"], inp["y_d"], j["qam"], inp["noise_var"],
                                             sc["chains"], sc["sweeps"], sc["beta2"],
                                             inp["seed"], stages=sc["stages"], init=sc["init"])
                    else:
                        o = ctx.detect(inp["H_d"], inp["y_d"], j["qam"], inp["noise_var"],
                                       sc["chains"], sc["sweeps"], sc["beta2"], inp["seed"],
                                       init=sc["init"])
                    outs.append(dict(sym=o[0], metric=o[1]))
                return outs

            print("[bench] tuned leg, every formulation (separate launches)", file=sys.stderr,
                  flush=True)
            n_calls = records_per_step(sep_group)
            ctx.set_profiling(True)
            el, lat = timed(sep_group)
            m = max(1, min(args.steps, 256 // n_calls))      # the library keeps 256 records
            sprof = np.array(ctx.profile(m * n_calls)).reshape(m, n_calls, 3)
            ctx.set_profiling(False)
            s_out = host_outs([o for gi in range(len(groups)) for o in sep_group(gi)])
            q_s = quality(inputs, s_out)
            tuned_sep = leg_record(el, lat, q_s, {
                "schedules": [sched_desc(s) for s in a_scheds],
                "stage_ms": {"anneal": float(np.mean(sprof[:, :, 1].sum(axis=1)))},
                "quality_matched": matched(q_s, q_ref)})
            legs["tuned_separate"] = (el, lat, a_scheds)
            # the same formulations as one HIP graph per slot: the build, the
            # MMSE-SIC launch and the search (or the persistent kernel for the
            # binary encoding, or the plain launches above 32 dimensions)
            # replayed; batches take no stages above 32 dimensions
            if fusable or all(not s.get("stages") for s in a_scheds):
                print("[bench] tuned leg, every formulation (one graph per slot)",
                      file=sys.stderr, flush=True)
                el, lat, tp_out, _ = fused_leg(a_scheds, persistent=False)
                q_tp = quality(inputs, tp_out)
                tuned_plan = leg_record(el, lat, q_tp, {
                    "schedules": [sched_desc(s) for s in a_scheds],
                    "outputs_identical_to_tuned_separate": same_bytes(tp_out, s_out,
                                                                      ("sym", "metric")),
                    "quality_matched": matched(q_tp, q_ref)})
                legs["tuned_plan"] = (el, lat, a_scheds)
            if not args.no_extras:
                # the same jobs with every stage as separate launches
                ctx.set_stage_launches(True)
                try:
                    el_st, _ = timed(sep_group)
                    st_out = host_outs([o for gi in range(len(groups)) for o in sep_group(gi)])
                finally:
                    ctx.set_stage_launches(False)
                stage_launch_ms = (el_st / args.steps * 1e3,
                                   same_bytes(st_out, s_out, ("sym", "metric")))

    # ---- ablation: the result-invariant choices, one at a time, at the schedules
    # above (the survey's split of the speed-up over the plain path)
    ablation = None
    if tuned is not None and plain is not None and not args.no_extras:
        print("[bench] ablation", file=sys.stderr, flush=True)

        def step_ms(el):
            return el / args.steps * 1e3

        rows = [{"step": "plain: build, anneal, select launches per slot, reference schedule",
                 "ms_per_step": plain["ms_per_step"]},
                {"step": "fusion + LDS: one persistent launch per slot (HIP graph), same schedule",
                 "ms_per_step": fused["ms_per_step"], "identical_outputs": fused[
                     "outputs_identical_to_plain"]}]
        el_ng, _, o_ng, _ = fused_leg(t_scheds, graph=False)
        rows.append({"step": "tuned schedule table (changes SER): one persistent launch per "
                             "slot, no HIP graph", "ms_per_step": step_ms(el_ng)})
        rows.append({"step": "+ HIP graph per slot (the tuned leg)",
                     "ms_per_step": tuned["ms_per_step"],
                     "identical_outputs": same_bytes(o_ng, t_out_ref, ("sym", "metric"))})
        if len(groups) > 1:
            el_one, _, o_one, _ = fused_leg(t_scheds, one_plan=True)
            rows.append({"step": "mixed-size packing: every slot of the step in one persistent "
                                 "launch (HIP graph)", "ms_per_step": step_ms(el_one),
                         "identical_outputs": same_bytes(o_one, t_out_ref, ("sym", "metric"))})
        el_b, _, o_b, _ = fused_leg(t_scheds, blocks=256)
        rows.append({"step": "mapping: one workgroup per CU instead of the library's resident "
                             "count (per slot, HIP graph)", "ms_per_step": step_ms(el_b),
                     "identical_outputs": same_bytes(o_b, t_out_ref, ("sym", "metric"))})
        if tuned_sep is not None and stage_launch_ms is not None:
            rows.append({"step": "separate launches at the fastest tuned formulation, every "
                                 "stage as its own launches", "ms_per_step": stage_launch_ms[0],
                         "identical_outputs": stage_launch_ms[1]})
            rows.append({"step": "+ one search launch per slot for moves around a guess and "
                                 "MMGaP-E (the tuned_separate leg)",
                         "ms_per_step": tuned_sep["ms_per_step"]})
            if tuned_plan is not None:
                rows.append({"step": "+ the slot's launches as one HIP graph (the tuned_plan leg)",
                             "ms_per_step": tuned_plan["ms_per_step"],
                             "identical_outputs": tuned_plan[
                                 "outputs_identical_to_tuned_separate"]})
        ablation = {"schedules_fused": [sched_desc(s) for s in t_scheds], "rows": rows}

    # ---- detection extras: MMGaP-E, MMSE-SIC, the SIC-guess search
    extras = {}
    if is_det and not args.no_extras and all(j["n_sc"] * j["n_sym"] > 0 for j in specs):
        def delta_sched(inp, which):
            j = inp["spec"]
            ch, sw, st = j[which]
            return dict(chains=ch, sweeps=sw, stages=st, init=0, beta2=W.linear_beta2(
                sw, *W.det_beta_range(j["qam"], j["rows"], inp["noise_var"])))

        e_sched = [delta_sched(inp, "delta") for inp in inputs]
        s_sched = [delta_sched(inp, "sic_delta") for inp in inputs]

        def e_group(scheds, guesses):
            def go(gi):
                return [ctx.detect_e(inputs[i]["H_d"], inputs[i]["y_d"],
                                     inputs[i]["spec"]["qam"], inputs[i]["noise_var"],
                                     scheds[i]["chains"], scheds[i]["sweeps"],
                                     scheds[i]["beta2"], inputs[i]["seed"],
                                     stages=scheds[i]["stages"], guesses=guesses)
                        for i in gidx[gi]]
            return go

        def sic_group(gi):
            return [ctx.detect_sic(inputs[i]["H_d"], inputs[i]["y_d"], inputs[i]["spec"]["qam"],
                                   inputs[i]["noise_var"]) for i in gidx[gi]]

        def q_of(go):
            outs = [o for gi in range(len(groups)) for o in go(gi)]
            return quality(inputs, [{"sym": o[0].cpu().numpy()} for o in outs])

        # the legs around MMSE-SIC need at most 16 users, the critical path's
        # persistent plan at most 32 real dimensions
        sic_ok = fusable and all(j["cols"] <= 16 for j in specs)
        sdesc = lambda s, g: f"{s['chains']} chains x {s['sweeps']} sweeps x {s['stages']} " \
                            f"stage(s) from {g}"
    if is_det and not args.no_extras and all(j["n_sc"] * j["n_sym"] > 0 for j in specs) \
            and sic_ok:
        print("[bench] MMGaP-E, MMSE-SIC, SIC-guess search", file=sys.stderr, flush=True)
        el, lat = timed(e_group(e_sched, M.GUESS_MMSE | M.GUESS_SIC))
        q = q_of(e_group(e_sched, M.GUESS_MMSE | M.GUESS_SIC))
        extras["mmgap_e"] = leg_record(el, lat, q, {
            "schedule": sdesc(e_sched[0], "the MMSE and the MMSE-SIC guess, better answer"),
            "quality_matched": matched(q, q_ref)})
        el, lat = timed(e_group(s_sched, M.GUESS_SIC))
        q = q_of(e_group(s_sched, M.GUESS_SIC))
        extras["sic_guess_search"] = leg_record(el, lat, q, {
            "schedule": sdesc(s_sched[0], "the MMSE-SIC guess"), "quality_matched": matched(q, q_ref)})
        el, lat = timed(sic_group)
        extras["mmse_sic"] = leg_record(el, lat, q_of(sic_group),
                                        {"schedule": "no anneal: ordered MMSE-SIC alone"})

        # critical path (paper §5.3): one subcarrier's 12 instances alone on the
        # GPU, for the tuned stages (MMGaP) and for MMGaP-E, from the middle slot
        mid = inputs[gidx[len(groups) // 2][0]]
        j = mid["spec"]
        H1, y1 = mid["H_d"][:1].contiguous(), mid["y_d"][:1].contiguous()
        ts = t_scheds[gidx[len(groups) // 2][0]] if t_scheds else e_sched[0]
        st1 = ts.get("stages", 0)
        reps = 50

        def lat_of(fn):
            for _ in range(5):
                fn()
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(reps)]
            for a, b in ev:
                a.record()
                fn()
                b.record()
            torch.cuda.synchronize()
            return pct([a.elapsed_time(b) for a, b in ev])

        job1 = ctx.det_job(H1, y1, j["qam"], mid["noise_var"], ts["chains"], ts["sweeps"],
                           ts["beta2"], mid["seed"], init=ts["init"], stages=st1,
                           guesses=guess_arg(ts))
        plan1 = ctx.plan_create([job1], graph=True)
        cp = {"instances": int(j["n_sym"]), "snr_db": j["snr"],
              "fused_tuned": dict(schedule=sched_desc(ts), **lat_of(plan1.plan_launch))}
        plan1.plan_destroy()
        if st1 and ts.get("guesses", 0) > 1:
            cp["mmgap_separate"] = lat_of(lambda: ctx.detect_e(
                H1, y1, j["qam"], mid["noise_var"], ts["chains"], ts["sweeps"], ts["beta2"],
                mid["seed"], stages=st1, guesses=ts["guesses"]))
        elif st1:
            cp["mmgap_separate"] = lat_of(lambda: ctx.detect_delta(
                H1, y1, j["qam"], mid["noise_var"], ts["chains"], ts["sweeps"], ts["beta2"],
                mid["seed"], stages=st1))
        es = e_sched[0]
        cp["mmgap_e"] = dict(schedule=sdesc(es, "both guesses, one after the other"),
                             **lat_of(lambda: ctx.detect_e(
                                 H1, y1, j["qam"], mid["noise_var"], es["chains"], es["sweeps"],
                                 es["beta2"], mid["seed"], stages=es["stages"])))
        # the paper's critical path runs MMGaP-E's two guesses in parallel: the
        # stage launches put the MMSE-SIC guess and its chain on the context's
        # second stream, beside the build and the chain from the MMSE guess
        # (outputs identical to the one-launch search)
        ctx.set_stage_launches(True)
        try:
            cp["mmgap_e_parallel"] = dict(
                schedule=sdesc(es, "both guesses in parallel on two streams"),
                **lat_of(lambda: ctx.detect_e(
                    H1, y1, j["qam"], mid["noise_var"], es["chains"], es["sweeps"],
                    es["beta2"], mid["seed"], stages=es["stages"])))
        finally:
            ctx.set_stage_launches(False)
        extras["critical_path"] = cp

    if is_det and not args.no_extras and all(j["n_sc"] * j["n_sym"] > 0 for j in specs):
        # build over 64 slots (one launch): the HBM-bound contraction at scale
        jb = specs[0]
        n64 = 64 * jb["n_sc"]
        Hb = inputs[0]["H_d"].repeat(64, 1, 1)
        yb = inputs[0]["y_d"].repeat(64, 1, 1)
        for _ in range(2):
            ctx.build_ising(M.KIND_DET, Hb, yb, jb["qam"], inputs[0]["noise_var"])
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(5)]
        for a, b in ev:
            a.record()
            ctx.build_ising(M.KIND_DET, Hb, yb, jb["qam"], inputs[0]["noise_var"])
            b.record()
        torch.cuda.synchronize()
        b_ms = float(np.median([a.elapsed_time(b) for a, b in ev]))
        b_bytes = build_bytes(jb, n64)
        extras["build_64_slots"] = {
            "bound": "hbm", "kernel": "k_det_build", "slots": 64, "subcarriers": n64,
            "achieved": b_bytes / (b_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": b_bytes / (b_ms * 1e-3) / PEAK_HBM, "bytes_per_launch": b_bytes,
            "kernel_ms": b_ms}
        del Hb, yb
    ctx.close()

    # ---- the reported leg: the fastest whose quality matches the plain leg's
    cands = [("fused", fused)] if fused is not None else [("plain", plain)]
    if tuned is not None and tuned["quality_matched"]:
        cands.append(("tuned", tuned))
    if delta_sep is not None and delta_sep["quality_matched"]:
        cands.append(("delta_separate", delta_sep))
    if tuned_sep is not None and tuned_sep["quality_matched"]:
        cands.append(("tuned_separate", tuned_sep))
    if tuned_plan is not None and tuned_plan["quality_matched"]:
        cands.append(("tuned_plan", tuned_plan))
    sel_name, sel = min(cands, key=lambda c: c[1]["ms_per_step"])
    sel_el, sel_lat, sel_scheds = legs[sel_name]
    value = args.steps * total_inst / sel_el

    # roofline of the dominant kernel on the reported leg: the anneals' operations
    # per slot launch over the launch's measured duration (HIP events on the
    # launch stream; for separate launches the library's events around its anneal
    # launches)
    attempts = ops = 0.0
    for inp, sc in zip(inputs, sel_scheds):
        a, o = sched_work(inp["spec"], sc)
        attempts += a
        ops += o
    if sel_name == "plain":
        kern_ms = plain["stage_ms"]["anneal"]
    elif sel_name == "delta_separate":
        kern_ms = delta_sep["stage_ms"]["anneal"]
    elif sel_name in ("tuned_separate", "tuned_plan"):
        # the same kernels and schedules: the library's events around the
        # search and anneal launches of the separate-launch leg
        kern_ms = tuned_sep["stage_ms"]["anneal"]
    else:
        kern_ms = float(sel_lat.mean(axis=0).sum())
    achieved = ops / (kern_ms * 1e-3)
    kname = {"plain": "k_anneal",
             "delta_separate": "k_search (moves around the guess, one launch per slot)",
             "tuned_separate": "k_search and k_anneal (tuned formulations: one search "
                               "launch per slot for moves around a guess and MMGaP-E)",
             "tuned_plan": "k_search and k_anneal (tuned formulations: one search launch per "
                           "slot for moves around a guess and MMGaP-E; kernel time from the "
                           "separate-launch leg's events around the same launches)"}.get(
        sel_name, "k_fused" + (" (moves around the guess)" if any(s.get("stages")
                                                                   for s in sel_scheds) else ""))
    if sel_name in ("tuned_separate", "tuned_plan") and not any(s.get("stages")
                                                                for s in sel_scheds):
        kname = "k_anneal (tuned schedules of the binary encoding: build, anneal and " \
                "selection launches per slot)"
    tkey = {"plain": "k_anneal", "delta_separate": "k_search_delta",
            "tuned_separate": "k_search_tuned_separate",
            "tuned_plan": "k_search_tuned_separate"}.get(
        sel_name, "k_fused_delta" if any(s.get("stages") for s in sel_scheds) else "k_fused")

    desc = []
    for j in specs:
        if j["kind"] == "det":
            desc.append(f"{j['rows']}x{j['cols']} {j['qam']}-QAM at {j['snr']:g} dB")
        else:
            desc.append(f"VPP {j['rows']}x{j['cols']} {j['qam']}-QAM")
    kinds = {j["kind"] for j in specs}
    head = ("uplink ML detection" if kinds == {"det"} else "downlink VPP" if kinds == {"vpp"}
            else "detection and VPP")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": sel_el / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{head}: " + "; ".join(desc) + f"; {specs[0]['n_sc']} subcarriers x "
                        f"{specs[0]['n_sym']} symbols per slot, i.i.d. Rayleigh, one slot per "
                        f"launch; reference " + ", ".join(sorted({f"{j['chains']} chains x "
                                                                 f"{j['sweeps']} sweeps"
                                                                 for j in specs})),
            "name": args.workload,
            "leg": sel_name,
            "path": {"plain": "plain: build, anneal and select launches per slot",
                     "fused": "fused: one persistent build+anneal+select launch per slot, "
                              "replayed as a HIP graph",
                     "tuned": "fused at the tuned schedules: one persistent launch per slot "
                              "(HIP graph), stages of moves around the MMSE guess inside it "
                              "where the tuner chose them",
                     "delta_separate": "the build, then every stage of the moves around the "
                                       "MMSE guess, the selections and the decode in one "
                                       "search launch",
                     "tuned_separate": "the tuned formulation per slot: the build (and the "
                                       "MMSE-SIC launch), then one search launch for every "
                                       "stage, both chains of MMGaP-E, the choice and the "
                                       "decode (moves around a guess), or anneal and select "
                                       "launches (binary encoding)",
                     "tuned_plan": "the tuned formulation per slot as one HIP graph: the build "
                                   "(and the MMSE-SIC launch) and one search launch for every "
                                   "stage, both chains of MMGaP-E, the choice and the decode "
                                   "(moves around a guess), or the persistent kernel (binary "
                                   "encoding)"
                     }[sel_name],
            "slots_per_step": len(groups),
            "instances_per_step": total_inst,
        },
        "p50_slot_ms": float(np.percentile(sel_lat, 50)),
        "p99_slot_ms": float(np.percentile(sel_lat, 99)),
        "deadline_ms": SERVE_DEADLINE_MS,
        "flip_attempts_per_s": attempts * args.steps / sel_el,
        "quality_kind": ["ser" if j["kind"] == "det" else "mean_gamma" for j in specs],
        "quality_per_slot": {"slot": desc, "plain": q_ref,
                             "reported": {"tuned": tuned, "delta_separate": delta_sep,
                                          "tuned_separate": tuned_sep, "tuned_plan": tuned_plan,
                                          "fused": fused, "plain": plain}[sel_name]["quality"]},
        "speedup_vs_plain": None if plain is None else value / plain["value"],
        "plain": plain,
        "fused_reference": fused,
        "tuned": tuned,
        "delta_separate": delta_sep,
        "tuned_separate": tuned_sep,
        "tuned_plan": tuned_plan,
        **extras,
        "ablation": ablation,
        "roofline": {
            "bound": "alu", "kernel": kname,
            "achieved": achieved / 1e12, "peak": PEAK_ALU_OPS / 1e12, "unit": "T lane-ops/s",
            "frac": achieved / PEAK_ALU_OPS,
            "traffic": stored_traffic(args.workload, tkey),
            "kernel_ms": kern_ms, "ops_per_step": ops, "attempts_per_step": attempts,
        },
        "cpu_baseline": None,
    }
    if is_det and not args.no_extras and not args.no_serve:
        print("[bench] serving mix", file=sys.stderr, flush=True)
        out["serve_mix"] = serve_mix(M, torch, 12, 20, 20)
    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(inputs, sel_scheds, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
