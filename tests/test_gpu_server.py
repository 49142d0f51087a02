"""GPU tests of the native serving loop (continuous batching).

Every job's outputs must be bit-identical to the single-job entry point on the
same arguments -- submitted alone, in a mix, under arena pressure, and while
other batches are running.
"""
import sys
import threading
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workload import synth as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts only with -m gpu
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2510_01579_amd as M


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


# (kind, rows, cols, qam, n_sc, n_sym, chains, sweeps, init)
MIX = [
    ("det", 8, 8, 16, 40, 12, 64, 20, 0),
    ("vpp", 8, 8, 16, 30, 12, 32, 15, 0),
    ("det", 16, 16, 64, 6, 12, 128, 6, 1),
    ("det", 4, 4, 4, 64, 1, 32, 30, 0),
    ("vpp", 16, 16, 4, 8, 5, 16, 10, 0),
    ("det", 8, 8, 64, 20, 7, 8, 25, 1),
]


def make_inputs(i, spec):
    kind, a, b, qam, n_sc, n_sym, chains, sweeps, init = spec
    if kind == "det":
        d = W.det_slot(1200 + i, a, b, qam, n_sc, n_sym, 20.0)
        beta2 = W.linear_beta2(sweeps, *W.det_beta_range(qam, a, d.noise_var))
        return dict(kind=kind, H=dev(d.H), y=dev(d.y), qam=qam, noise_var=d.noise_var,
                    chains=chains, sweeps=sweeps, beta2=beta2, seed=W.job_seed(70 + i), init=init)
    s = W.vpp_slot(1300 + i, a, b, qam, n_sc, n_sym)
    beta2 = W.linear_beta2(sweeps, *W.vpp_beta_range(qam, b))
    return dict(kind=kind, H=dev(s.H), y=dev(s.u), qam=qam, chains=chains, sweeps=sweeps,
                beta2=beta2, seed=W.job_seed(70 + i), init=init)


def job_of(ctx, inp):
    if inp["kind"] == "det":
        return ctx.det_job(inp["H"], inp["y"], inp["qam"], inp["noise_var"], inp["chains"],
                           inp["sweeps"], inp["beta2"], inp["seed"], init=inp["init"])
    return ctx.vpp_job(inp["H"], inp["y"], inp["qam"], inp["chains"], inp["sweeps"],
                       inp["beta2"], inp["seed"], init=inp["init"])


def single_call(ctx, inp):
    if inp["kind"] == "det":
        sym, met = ctx.detect(inp["H"], inp["y"], inp["qam"], inp["noise_var"], inp["chains"],
                              inp["sweeps"], inp["beta2"], inp["seed"], init=inp["init"])
        out = dict(sym=sym, metric=met)
    else:
        v, x, g = ctx.vpp_precode(inp["H"], inp["y"], inp["qam"], inp["chains"], inp["sweeps"],
                                  inp["beta2"], inp["seed"], init=inp["init"])
        out = dict(v=v, x=x, gamma=g)
    torch.cuda.synchronize()
    return {k: t.cpu().numpy() for k, t in out.items()}


def assert_same(job, ref, label):
    for k, r in ref.items():
        g = job["outputs"][k].cpu().numpy()
        assert g.tobytes() == r.tobytes(), f"{label}: {k} differs"


def wait_all(ctx, ids, timeout=60.0):
    lat = {}
    t0 = time.time()
    while len(lat) < len(ids):
        for i in ids:
            if i in lat:
                continue
            done, us = ctx.server_poll(i)
            if done:
                lat[i] = us
        assert time.time() - t0 < timeout, "server did not complete the jobs"
        time.sleep(0.0005)
    return lat


@pytest.fixture(scope="module")
def ctx():
    c = M.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def mix(ctx):
    inputs = [make_inputs(i, s) for i, s in enumerate(MIX)]
    return inputs, [single_call(ctx, inp) for inp in inputs]


def test_server_mix_equals_single_calls(ctx, mix):
    inputs, refs = mix
    note("server: mixed jobs, 2 in flight")
    ctx.server_start(max_inflight=2)
    try:
        for rep in range(2):
            jobs = [job_of(ctx, inp) for inp in inputs]
            ids = [ctx.server_submit(j) for j in jobs]
            lat = wait_all(ctx, ids)
            assert all(v > 0 for v in lat.values())
            for i, j in enumerate(jobs):
                assert_same(j, refs[i], f"rep {rep} job {i} {MIX[i]}")
    finally:
        ctx.server_stop()


def test_server_job_alone_equals_in_mix(ctx, mix):
    inputs, refs = mix
    note("server: each job alone")
    ctx.server_start(max_inflight=1)
    try:
        for i in (0, 2, 4):
            j = job_of(ctx, inputs[i])
            wait_all(ctx, [ctx.server_submit(j)])
            assert_same(j, refs[i], f"alone job {i}")
    finally:
        ctx.server_stop()


def test_server_arena_pressure_and_arrivals_during_batches(ctx, mix):
    """An arena that holds about two jobs: the rest wait for memory; jobs are
    submitted from another thread while batches run."""
    inputs, refs = mix
    note("server: small arena, arrivals from a second thread")
    # the largest job of the mix needs about 115 KB of arena
    ctx.server_start(max_inflight=3, arena_bytes=256 << 10, max_batch_jobs=2)
    try:
        jobs = [job_of(ctx, inputs[i % len(inputs)]) for i in range(18)]
        ids = [None] * len(jobs)
        torch.cuda.synchronize()

        def producer():
            # the main thread only waits for this one meanwhile
            for k in range(len(jobs)):
                ids[k] = ctx.server_submit(jobs[k])
                time.sleep(0.001)

        t = threading.Thread(target=producer)
        t.start()
        t.join()
        ctx.server_drain()
        wait_all(ctx, ids)
        for k, j in enumerate(jobs):
            assert_same(j, refs[k % len(inputs)], f"job {k}")
    finally:
        ctx.server_stop()


def test_server_errors(ctx, mix):
    inputs, _ = mix
    note("server: error paths")
    with pytest.raises(M.MmgapError) as e:
        ctx.server_submit(job_of(ctx, inputs[0]))
    assert e.value.code == -1                       # no server
    ctx.server_start(max_inflight=1, arena_bytes=1 << 16)
    try:
        with pytest.raises(M.MmgapError) as e:
            ctx.server_start()
        assert e.value.code == -5                   # already running
        with pytest.raises(M.MmgapError) as e:
            ctx.server_submit(job_of(ctx, inputs[0]))
        assert e.value.code == -2                   # can never fit the arena
        with pytest.raises(M.MmgapError) as e:
            ctx.server_poll(12345)
        assert e.value.code == -1
    finally:
        ctx.server_stop()
    ctx.server_stop()                               # stopping twice is harmless


def test_server_runs_detection_around_a_guess(ctx, mix):
    """Jobs with stages >= 1 (moves around the MMSE guess) served beside plain
    jobs equal mmgap_detect_delta on the same arguments."""
    inputs, refs = mix
    note("server: jobs with stages around the MMSE guess in a mix")
    specs = [(8, 8, 64, 12, 12, 16, 12, 1), (16, 16, 64, 4, 12, 16, 8, 2), (4, 4, 16, 30, 5, 32, 20, 3)]
    dins, drefs = [], []
    for i, (a, b, qam, n_sc, n_sym, chains, sweeps, stages) in enumerate(specs):
        d = W.det_slot(1400 + i, a, b, qam, n_sc, n_sym, 25.0)
        beta2 = W.linear_beta2(sweeps, *W.det_beta_range(qam, a, d.noise_var))
        inp = dict(H=dev(d.H), y=dev(d.y), qam=qam, noise_var=d.noise_var, chains=chains,
                   sweeps=sweeps, beta2=beta2, seed=W.job_seed(90 + i), stages=stages)
        sym, met = ctx.detect_delta(inp["H"], inp["y"], qam, d.noise_var, chains, sweeps, beta2,
                                    inp["seed"], stages=stages)
        torch.cuda.synchronize()
        dins.append(inp)
        drefs.append(dict(sym=sym.cpu().numpy(), metric=met.cpu().numpy()))
    ctx.server_start(max_inflight=2)
    try:
        jobs = [ctx.det_job(p["H"], p["y"], p["qam"], p["noise_var"], p["chains"], p["sweeps"],
                            p["beta2"], p["seed"], stages=p["stages"]) for p in dins]
        plain = [job_of(ctx, inputs[i]) for i in (0, 1)]
        ids = [ctx.server_submit(j) for j in jobs[:2] + plain + jobs[2:]]
        wait_all(ctx, ids)
        for k, j in enumerate(jobs):
            assert_same(j, drefs[k], f"delta job {k} {specs[k]}")
        for k, j in zip((0, 1), plain):
            assert_same(j, refs[k], f"plain job {k}")
    finally:
        ctx.server_stop()


def test_server_latency_accounting(ctx, mix):
    """mmgap_server_stats counts every completed job and those above the
    deadline, with the nearest-rank percentiles of the latencies the polls
    report (the accounting of admission.h, which tests/test_serve_sim_cpu.py
    checks on a simulated device)."""
    import math
    inputs, _ = mix
    note("server: latency accounting")
    ctx.server_start(max_inflight=2)
    try:
        s0 = ctx.server_stats(0.5)
        assert s0["completed"] == 0 and s0["missed"] == 0 and s0["max_ms"] == 0.0
        jobs = [job_of(ctx, inp) for inp in inputs]
        ids = [ctx.server_submit(j) for j in jobs]
        lat = sorted(wait_all(ctx, ids).values())           # microseconds
        n = len(lat)
        k = next(i for i in range(n // 2, n) if lat[i - 1] < lat[i])
        d_us = 0.5 * (lat[k - 1] + lat[k])                  # strictly between two latencies
        s = ctx.server_stats(d_us / 1e3)
        assert s["completed"] == n
        assert s["missed"] == sum(1 for v in lat if v > d_us) == n - k
        rank = lambda p: lat[max(1, math.ceil(p / 100 * n)) - 1]
        assert math.isclose(s["p50_ms"] * 1e3, rank(50), rel_tol=1e-12)
        assert math.isclose(s["p99_ms"] * 1e3, rank(99), rel_tol=1e-12)
        assert math.isclose(s["max_ms"] * 1e3, lat[-1], rel_tol=1e-12)
        s = ctx.server_stats(d_us / 1e3, reset=True)        # read, then a new period
        assert s["completed"] == n
        assert ctx.server_stats(d_us / 1e3)["completed"] == 0
        with pytest.raises(M.MmgapError) as e:
            ctx.server_stats(-1.0)
        assert e.value.code == -1
    finally:
        ctx.server_stop()
