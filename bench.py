#!/usr/bin/env python3
"""Benchmark of the Ising hot path (ML-MIMO detection / VPP precoding) on one MI355X.

A step is one 5G slot of every job of the workload through the whole path --
Gram/field build, annealing, selection and decode -- on synthetic i.i.d.
Rayleigh channels (inputs resident in HBM before the timed region).  Two legs
run on the same inputs and schedules:
  * fused: one persistent launch per slot (a batch plan replayed as a HIP graph);
  * plain: the per-size entry points, one build, anneal and select launch each.
Their outputs must be identical.  The JSON line reports the fused leg's
whole-job throughput (Ising solves/s) and slot latency percentiles, the plain
leg beside it, the roofline position of the dominant kernel (VALU-bound), and
the CPU oracle timed on a bounded sample of the same workload.

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

N_SC, N_SYM = 3276, 12


def _det(n_r, n_t, qam, chains, sweeps, snr, seed, init, n_sc=N_SC, n_sym=N_SYM):
    return dict(kind="det", rows=n_r, cols=n_t, qam=qam, n_sc=n_sc, n_sym=n_sym, chains=chains,
                sweeps=sweeps, snr=snr, seed=seed, init=init)


def _vpp(n_u, n_t, qam, chains, sweeps, seed, n_sc=N_SC, n_sym=N_SYM):
    return dict(kind="vpp", rows=n_u, cols=n_t, qam=qam, n_sc=n_sc, n_sym=n_sym, chains=chains,
                sweeps=sweeps, snr=None, seed=seed, init=0)


WORKLOADS = {
    # the configuration the metric is quoted on: one slot, 8x8 16-QAM
    "det-8x8-16qam": [_det(8, 8, 16, 64, 200, 15.0, 2001, 0)],
    # 64-QAM anneals start from the MMSE fallback (random starts stay trapped)
    "det-16x16-64qam": [_det(16, 16, 64, 128, 400, 25.0, 3001, 1)],
    "det-4x4-qpsk": [_det(4, 4, 4, 32, 100, 10.0, 0, 0, n_sc=64, n_sym=1)],
    # downlink VPP, two sizes batched in one launch
    "vpp-8x8+16x16-16qam": [_vpp(8, 8, 16, 64, 200, 4001), _vpp(16, 16, 16, 64, 200, 4002)],
}


def qbits(qam: int) -> int:
    return {4: 1, 16: 2, 64: 3}[qam]


def job_shape(j):
    """(K, q, instances, flip attempts per slot) of a job."""
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


def cpu_baseline(inputs, target_s: float):
    """The oracle as it stands, on a bounded random sample of the workload's
    instances (spread over its jobs in proportion to their instance counts)."""
    from oracle import oracle as O
    threads = O.max_threads()
    rng = np.random.default_rng(1)
    sizes = [job_shape(inp["spec"])[2] for inp in inputs]
    total = sum(sizes)

    def run(frac):
        n_done = 0
        t0 = time.perf_counter()
        for inp, n_all in zip(inputs, sizes):
            j = inp["spec"]
            m = max(1, min(n_all, int(round(frac * n_all))))
            ids = np.sort(rng.choice(n_all, m, replace=False)).astype(np.uint32)
            if j["kind"] == "det":
                O.detect(inp["H"], inp["y"], inp["noise_var"], j["qam"], j["chains"],
                         j["sweeps"], inp["beta2"], inp["seed"], inst_ids=ids,
                         init_mode=j["init"])
            else:
                O.vpp_precode(inp["H"], inp["y"], j["qam"], j["chains"], j["sweeps"],
                              inp["beta2"], inp["seed"], inst_ids=ids)
            n_done += m
        return n_done, time.perf_counter() - t0

    n0, t_probe = run(min(1.0, 8.0 * threads / total))
    frac = min(1.0, target_s / max(t_probe, 1e-6) * n0 / total)
    n, dt = run(frac)
    return {"value": n / dt, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} of {total} instances of the same slot(s) (random subset), "
                      f"same chains and sweeps, {dt:.1f} s on {threads} threads"}


def main(argv=None) -> int:  # noqa: C901
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="det-8x8-16qam", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy three times, so that "
                         "hardware counters of a kernel of known traffic can be read")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the hot path shards by subcarrier with no "
              "exchange, and multi-GPU runs are not part of this build (use --gpus 1)",
              file=sys.stderr)
        return 2

    import torch

    import paper_2510_01579_amd as M

    specs = WORKLOADS[args.workload]
    inputs = make_inputs(specs)
    dev = torch.device("cuda", 0)
    for inp in inputs:
        inp["H_d"] = torch.from_numpy(inp["H"]).to(dev)
        inp["y_d"] = torch.from_numpy(inp["y"]).to(dev)
    ctx = M.Context(0)

    def plain_step():
        outs = []
        for inp in inputs:
            j = inp["spec"]
            if j["kind"] == "det":
                outs.append(ctx.detect(inp["H_d"], inp["y_d"], j["qam"], inp["noise_var"],
                                       j["chains"], j["sweeps"], inp["beta2"], inp["seed"],
                                       init=j["init"]))
            else:
                outs.append(ctx.vpp_precode(inp["H_d"], inp["y_d"], j["qam"], j["chains"],
                                            j["sweeps"], inp["beta2"], inp["seed"]))
        return outs

    jobs = []
    for inp in inputs:
        j = inp["spec"]
        if j["kind"] == "det":
            jobs.append(ctx.det_job(inp["H_d"], inp["y_d"], j["qam"], inp["noise_var"],
                                    j["chains"], j["sweeps"], inp["beta2"], inp["seed"],
                                    init=j["init"]))
        else:
            jobs.append(ctx.vpp_job(inp["H_d"], inp["y_d"], j["qam"], j["chains"], j["sweeps"],
                                    inp["beta2"], inp["seed"]))
    plan = ctx.plan_create(jobs, graph=True)
    n_items, n_blocks = plan.plan_info()

    def timed(step, steps):
        start = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        stop = [torch.cuda.Event(enable_timing=True) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            start[k].record()
            step()
            stop[k].record()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        return elapsed, np.array([a.elapsed_time(b) for a, b in zip(start, stop)])

    # fused leg (the reported value); the events bracket exactly one plan launch
    # (counter reset + persistent kernel) on the current stream
    for _ in range(args.warmup):
        plan.plan_launch()
    f_elapsed, f_lat = timed(plan.plan_launch, args.steps)
    fused_out = [{k: (None if t is None else t.cpu().numpy()) for k, t in jb["outputs"].items()}
                 for jb in jobs]

    plain = None
    identical = None
    if not args.no_plain:
        for _ in range(args.warmup):
            plain_step()
        ctx.set_profiling(True)
        p_elapsed, p_lat = timed(plain_step, args.steps)
        prof = np.array(ctx.profile(args.steps * len(inputs))).reshape(args.steps, len(inputs), 3)
        ctx.set_profiling(False)
        outs = plain_step()
        torch.cuda.synchronize()
        identical = True
        for inp, o, fo in zip(inputs, outs, fused_out):
            if inp["spec"]["kind"] == "det":
                pairs = [(o[0], fo["sym"]), (o[1], fo["metric"])]
            else:
                pairs = [(o[0], fo["v"]), (o[1], fo["x"]), (o[2], fo["gamma"])]
            for a, b in pairs:
                if a.cpu().numpy().tobytes() != b.tobytes():
                    identical = False
        anneal_ms = float(np.mean(prof[:, :, 1].sum(axis=1)))
        solves = args.steps * sum(job_shape(i["spec"])[2] for i in inputs)
        plain = {"value": solves / p_elapsed, "unit": "solves/s",
                 "ms_per_step": p_elapsed / args.steps * 1e3,
                 "p50_slot_ms": float(np.percentile(p_lat, 50)),
                 "p99_slot_ms": float(np.percentile(p_lat, 99)),
                 "stage_ms": {"build": float(np.mean(prof[:, :, 0].sum(axis=1))),
                              "anneal": anneal_ms,
                              "select": float(np.mean(prof[:, :, 2].sum(axis=1)))}}

    # quality: SER against the transmitted symbols (detection), mean transmit
    # energy against zero perturbation (VPP)
    quality = []
    for inp, fo in zip(inputs, fused_out):
        j = inp["spec"]
        n = j["n_sc"] * j["n_sym"]
        if j["kind"] == "det":
            fb = ctx.build_ising(M.KIND_DET, inp["H_d"], inp["y_d"], j["qam"],
                                 noise_var=inp["noise_var"])["x_fb"].cpu().numpy()
            truth = inp["raw"].sym.reshape(n, j["cols"])
            quality.append({"job": f"det {j['rows']}x{j['cols']} {j['qam']}-QAM",
                            "ser": float(np.mean(fo["sym"] != truth)),
                            "ser_mmse": float(np.mean(levels_to_symbols(fb, j["qam"]) != truth))})
        else:
            H = inp["H"].astype(np.complex128)
            u = inp["y"].astype(np.complex128)
            W = np.conj(np.swapaxes(H, 1, 2)) @ np.linalg.inv(H @ np.conj(np.swapaxes(H, 1, 2)))
            x0 = np.einsum("stu,smu->smt", W, u).reshape(n, -1)
            quality.append({"job": f"vpp {j['rows']}x{j['cols']} {j['qam']}-QAM",
                            "mean_gamma": float(np.mean(fo["gamma"])),
                            "mean_gamma_zf": float(np.mean(np.sum(np.abs(x0) ** 2, axis=1)))})
    plan.plan_destroy()
    ctx.close()

    total_inst = sum(job_shape(i["spec"])[2] for i in inputs)
    attempts = sum(job_shape(i["spec"])[3] for i in inputs)
    alg_ops = sum(job_shape(i["spec"])[3] * ops_per_attempt(*job_shape(i["spec"])[:2])
                  for i in inputs)
    fused_s = float(np.mean(f_lat)) / 1e3
    achieved = alg_ops / fused_s
    value = args.steps * total_inst / f_elapsed

    desc = []
    for j in specs:
        if j["kind"] == "det":
            desc.append(f"uplink ML detection {j['rows']}x{j['cols']} {j['qam']}-QAM, SNR "
                        f"{j['snr']:g} dB, " + ("random start" if j["init"] == 0 else
                                                "start from the MMSE fallback"))
        else:
            desc.append(f"downlink VPP {j['rows']}x{j['cols']} {j['qam']}-QAM")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": f_elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "; ".join(desc) + f"; {specs[0]['n_sc']} subcarriers x "
                        f"{specs[0]['n_sym']} symbols per slot, "
                        + ", ".join(f"{j['chains']} chains x {j['sweeps']} sweeps" for j in specs)
                        + ", i.i.d. Rayleigh",
            "name": args.workload,
            "path": "fused: one persistent build+anneal+select launch per slot, replayed as a "
                    "HIP graph",
            "instances_per_step": total_inst,
            "work_items": n_items,
            "workgroups": n_blocks,
        },
        "p50_slot_ms": float(np.percentile(f_lat, 50)),
        "p99_slot_ms": float(np.percentile(f_lat, 99)),
        "flip_attempts_per_s": attempts * args.steps / f_elapsed,
        "plain": plain,
        "speedup_vs_plain": None if plain is None else value / plain["value"],
        "outputs_identical_to_plain": identical,
        "quality": quality,
        "roofline": {
            "bound": "alu",
            "kernel": "k_fused",
            "achieved": achieved / 1e12,
            "peak": PEAK_ALU_OPS / 1e12,
            "unit": "T lane-ops/s",
            "frac": achieved / PEAK_ALU_OPS,
            "traffic": stored_traffic(args.workload, "k_fused"),
            "kernel_ms": fused_s * 1e3,
            "ops_per_launch": alg_ops,
            "attempts_per_launch": attempts,
        },
        "cpu_baseline": None,
    }
    if args.copy_calibration:
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inputs, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
