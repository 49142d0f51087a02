"""The serving loop against the oracle directly, on a mix shaped like the
serving workload: uplink detection and downlink VPP jobs of 8x8 and 16x16
with QPSK, 16-QAM and 64-QAM, the tuner's schedules for each job's class and
SNR (the binary encoding or moves around the MMSE guess in stages), several
jobs per batch, jobs submitted from a second thread while batches run.

Every served job is compared with the oracle on 40 sampled instances plus its
first and last: identical symbols / perturbations (the spec bar of
>= 99.99% of instances admits no mismatch at this sample size), float64
metrics, transmit vectors and energies within 1e-4 relative (the paper's
post-processing output, §3.2; VPP §3.3).
"""
import sys
import threading
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from workload import synth as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts only with -m gpu
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2510_01579_amd as M

N_SC, N_SYM = 512, 12

# (kind, n, qam, snr_db or None, forced (chains, sweeps, stages) or None)
MIX = [
    ("det", 8, 4, 8.0, None),
    ("det", 8, 16, 15.0, None),
    ("vpp", 8, 16, None, None),
    ("det", 8, 64, 25.0, None),
    ("det", 16, 4, 10.0, None),
    ("vpp", 16, 4, None, None),
    ("det", 16, 16, 20.0, None),
    ("det", 16, 64, 28.0, None),
    ("vpp", 16, 64, None, None),
    ("det", 16, 64, 18.0, (16, 8, 2)),
]


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def make_job(ctx, k, spec):
    kind, n, qam, snr, forced = spec
    seed = 1500 + k
    if kind == "det":
        d = W.det_slot(seed, n, n, qam, N_SC, N_SYM, snr)
        sc = M.tuned_schedule(M.KIND_DET, n, n, qam, d.noise_var)
        if forced:
            ch, sw, st = forced
            sc = dict(chains=ch, sweeps=sw, init=0, stages=st, beta2=W.linear_beta2(
                sw, *W.det_beta_range(qam, n, d.noise_var)))
        H, y = dev(d.H), dev(d.y)
        g = sc.get("guesses", 0)
        job = ctx.det_job(H, y, qam, d.noise_var, sc["chains"], sc["sweeps"], sc["beta2"],
                          W.job_seed(seed), init=sc["init"], stages=sc["stages"],
                          guesses=g if g > 1 else 0)
        return dict(kind=kind, raw=d, H=d.H, y=d.y, nv=d.noise_var, qam=qam, sched=sc,
                    seed=W.job_seed(seed), job=job)
    s = W.vpp_slot(seed, n, n, qam, N_SC, N_SYM)
    sc = M.tuned_schedule(M.KIND_VPP, n, n, qam)
    job = ctx.vpp_job(dev(s.H), dev(s.u), qam, sc["chains"], sc["sweeps"], sc["beta2"],
                      W.job_seed(seed), init=sc["init"])
    return dict(kind=kind, raw=s, H=s.H, y=s.u, nv=0.0, qam=qam, sched=sc,
                seed=W.job_seed(seed), job=job)


def oracle_ref(j, ids):
    sc = j["sched"]
    if j["kind"] == "det" and sc.get("guesses", 0) > 1:
        return O.detect_e(j["H"], j["y"], j["nv"], j["qam"], sc["chains"], sc["sweeps"],
                          sc["beta2"], j["seed"], stages=sc["stages"], inst_ids=ids,
                          init_mode=sc["init"], guesses=sc["guesses"])
    if j["kind"] == "det" and sc["stages"]:
        return O.detect_delta(j["H"], j["y"], j["nv"], j["qam"], sc["chains"], sc["sweeps"],
                              sc["beta2"], j["seed"], stages=sc["stages"], inst_ids=ids,
                              init_mode=sc["init"])
    if j["kind"] == "det":
        return O.detect(j["H"], j["y"], j["nv"], j["qam"], sc["chains"], sc["sweeps"],
                        sc["beta2"], j["seed"], inst_ids=ids, init_mode=sc["init"])
    return O.vpp_precode(j["H"], j["y"], j["qam"], sc["chains"], sc["sweeps"], sc["beta2"],
                         j["seed"], inst_ids=ids, init_mode=sc["init"])


def wait_all(ctx, ids, timeout=120.0):
    done = set()
    t0 = time.time()
    while len(done) < len(ids):
        for i in ids:
            if i not in done and ctx.server_poll(i)[0]:
                done.add(i)
        assert time.time() - t0 < timeout, "server did not complete the jobs"
        time.sleep(0.0005)


def test_served_mix_matches_the_oracle():
    ctx = M.Context(0)
    try:
        jobs = [make_job(ctx, k, s) for k, s in enumerate(MIX)]
        assert any(j["sched"]["stages"] for j in jobs) and any(
            j["kind"] == "det" and not j["sched"]["stages"] for j in jobs)
        torch.cuda.synchronize()
        note("server: C5-shaped mix of 10 jobs, 3 batches in flight, arrivals from a thread")
        ctx.server_start(max_inflight=3, max_batch_jobs=4)
        ids = [None] * len(jobs)
        try:
            ids[0] = ctx.server_submit(jobs[0]["job"])
            ids[1] = ctx.server_submit(jobs[1]["job"])

            def producer():
                for k in range(2, len(jobs)):
                    ids[k] = ctx.server_submit(jobs[k]["job"])
                    time.sleep(0.002)

            t = threading.Thread(target=producer)
            t.start()
            t.join()
            wait_all(ctx, ids)
        finally:
            ctx.server_stop()
        rng = np.random.default_rng(77)
        n = N_SC * N_SYM
        for k, j in enumerate(jobs):
            ids_k = np.unique(np.concatenate([[0, n - 1], rng.choice(n, 40, replace=False)]))
            ids_k = ids_k.astype(np.uint32)
            sc = j["sched"]
            note(f"job {k} {MIX[k][:4]} {sc['chains']}x{sc['sweeps']} stages {sc['stages']}")
            ref = oracle_ref(j, ids_k)
            out = {key: (None if t is None else t.cpu().numpy())
                   for key, t in j["job"]["outputs"].items()}
            if j["kind"] == "det":
                assert np.array_equal(out["sym"][ids_k], ref["sym"]), f"job {k}"
                assert np.allclose(out["metric"][ids_k].astype(np.float64), ref["metric"],
                                   rtol=1e-4, atol=1e-6), f"job {k}"
            else:
                assert np.array_equal(out["v"][ids_k], ref["v"]), f"job {k}"
                assert np.allclose(out["gamma"][ids_k].astype(np.float64), ref["gamma"],
                                   rtol=1e-4, atol=1e-6), f"job {k}"
                assert np.allclose(out["x"][ids_k].astype(np.complex128), ref["x"], rtol=1e-4,
                                   atol=1e-5), f"job {k}"
    finally:
        ctx.close()
