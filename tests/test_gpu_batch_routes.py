"""Jobs that run with launches of their own inside a batch: CIM-CAC jobs (the
build, anneal and selection launches of the plain entry points; paper §2.3
Eqs. cim1/cim2), Metropolis jobs wider than 32 dimensions (the 32x32 shape of
§5.2.3 and 24 users, by the plain path's launches) and jobs with stages that
the one-launch search runs (moves around a guess, MMGaP-E; §2.3 Fig. 5, §3.2
Fig. 6), beside jobs of the persistent kernels.  Every job's outputs must equal its single-call entry
point's, bit for bit, in plans (on every graph replay) and in the server.
"""
import sys
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


@pytest.fixture(scope="module")
def ctx():
    c = M.Context(0)
    yield c
    c.close()


# (label, kind, rows, cols, qam, n_sc, n_sym, chains, sweeps, stages, guesses, cim)
SPECS = [
    ("cim det 8x8 16-QAM", "det", 8, 8, 16, 21, 12, 32, 64, 0, 0, {}),
    ("cim det 16x16 16-QAM, 64 spins", "det", 16, 16, 16, 7, 12, 16, 40, 0, 0, {"f_mvm": 1}),
    ("cim vpp 8x8 16-QAM", "vpp", 8, 8, 16, 11, 6, 32, 50, 0, 0, {}),
    ("search E 16x16 64-QAM", "det", 16, 16, 64, 9, 12, 16, 4, 3, 3, None),
    ("search SIC guess 8x8 64-QAM", "det", 8, 8, 64, 13, 12, 8, 2, 1, 2, None),
    ("search MMSE guess 8x8 16-QAM", "det", 8, 8, 16, 17, 12, 16, 6, 2, 0, None),
    ("persistent delta, 128 chains", "det", 8, 8, 16, 5, 4, 128, 4, 1, 0, None),
    ("persistent binary 8x8 16-QAM", "det", 8, 8, 16, 19, 12, 64, 20, 0, 0, None),
    ("plain 32x32 16-QAM, 64 dimensions", "det", 32, 32, 16, 3, 12, 64, 8, 0, 0, None),
    ("plain 24 users QPSK, 48 of 64 dimensions", "det", 24, 24, 4, 2, 5, 32, 6, 0, 0, None),
    ("persistent vpp 8x8 16-QAM", "vpp", 8, 8, 16, 9, 6, 32, 20, 0, 0, None),
]


def make(i, spec):
    label, kind, a, b, qam, n_sc, n_sym, chains, sweeps, stages, guesses, cim = spec
    if kind == "det":
        d = W.det_slot(6100 + i, a, b, qam, n_sc, n_sym, 20.0)
        beta2 = None if cim is not None else \
            W.linear_beta2(sweeps, *W.det_beta_range(qam, a, d.noise_var))
        return dict(kind=kind, H=dev(d.H), y=dev(d.y), qam=qam, noise_var=d.noise_var,
                    chains=chains, sweeps=sweeps, beta2=beta2, seed=W.job_seed(610 + i),
                    stages=stages, guesses=guesses, cim=cim)
    s = W.vpp_slot(6200 + i, a, b, qam, n_sc, n_sym)
    beta2 = None if cim is not None else W.linear_beta2(sweeps, *W.vpp_beta_range(qam, b))
    return dict(kind=kind, H=dev(s.H), y=dev(s.u), qam=qam, chains=chains, sweeps=sweeps,
                beta2=beta2, seed=W.job_seed(610 + i), stages=0, guesses=0, cim=cim)


def single(ctx, p):
    if p["kind"] == "vpp":
        v, x, g = ctx.vpp_precode(p["H"], p["y"], p["qam"], p["chains"], p["sweeps"], p["beta2"],
                                  p["seed"], cim=p["cim"])
        out = dict(v=v, x=x, gamma=g)
    elif p["guesses"]:
        s, m, fs = ctx.detect_e(p["H"], p["y"], p["qam"], p["noise_var"], p["chains"],
                                p["sweeps"], p["beta2"], p["seed"], stages=p["stages"],
                                guesses=p["guesses"])
        out = dict(sym=s, metric=m, from_sic=fs)
    elif p["stages"]:
        s, m = ctx.detect_delta(p["H"], p["y"], p["qam"], p["noise_var"], p["chains"],
                                p["sweeps"], p["beta2"], p["seed"], stages=p["stages"])
        out = dict(sym=s, metric=m)
    else:
        s, m = ctx.detect(p["H"], p["y"], p["qam"], p["noise_var"], p["chains"], p["sweeps"],
                          p["beta2"], p["seed"], cim=p["cim"])
        out = dict(sym=s, metric=m)
    torch.cuda.synchronize()
    return {k: t.cpu().numpy() for k, t in out.items()}


def job_of(ctx, p):
    if p["kind"] == "vpp":
        return ctx.vpp_job(p["H"], p["y"], p["qam"], p["chains"], p["sweeps"], p["beta2"],
                           p["seed"], cim=p["cim"])
    return ctx.det_job(p["H"], p["y"], p["qam"], p["noise_var"], p["chains"], p["sweeps"],
                       p["beta2"], p["seed"], stages=p["stages"], guesses=p["guesses"],
                       cim=p["cim"])


def check(job, ref, label):
    torch.cuda.synchronize()
    for k, r in ref.items():
        g = job["outputs"][k].cpu().numpy()
        assert g.shape == r.shape and g.tobytes() == r.tobytes(), f"{label}: {k} differs"


@pytest.fixture(scope="module")
def cases(ctx):
    inputs = [make(i, s) for i, s in enumerate(SPECS)]
    return inputs, [single(ctx, p) for p in inputs]


@pytest.mark.parametrize("i", range(len(SPECS)))
def test_job_alone_in_a_plan(ctx, cases, i):
    inputs, refs = cases
    note(f"plan, one job: {SPECS[i][0]}")
    job = job_of(ctx, inputs[i])
    plan = ctx.plan_create([job], graph=True)
    for rep in range(2):
        plan.plan_launch()
        check(job, refs[i], f"{SPECS[i][0]} replay {rep}")
    plan.plan_destroy()


def test_all_routes_in_one_plan_on_every_replay(ctx, cases):
    inputs, refs = cases
    note("plan with every route, graph replays")
    jobs = [job_of(ctx, p) for p in inputs]
    plan = ctx.plan_create(jobs, graph=True)
    for rep in range(3):
        for j in jobs:
            for t in j["outputs"].values():
                if t is not None:
                    t.zero_()
        plan.plan_launch()
        for k, j in enumerate(jobs):
            check(j, refs[k], f"{SPECS[k][0]} replay {rep}")
    plan.plan_destroy()


def test_all_routes_in_the_server(ctx, cases):
    inputs, refs = cases
    note("server with every route, 2 in flight")
    ctx.server_start(max_inflight=2)
    try:
        for rep in range(2):
            jobs = [job_of(ctx, p) for p in inputs]
            ids = [ctx.server_submit(j) for j in jobs]
            t0 = time.time()
            pending = set(ids)
            while pending:
                for jid in list(pending):
                    if ctx.server_poll(jid)[0]:
                        pending.discard(jid)
                assert time.time() - t0 < 60.0, "server did not complete the jobs"
                time.sleep(0.0005)
            for k, j in enumerate(jobs):
                check(j, refs[k], f"server rep {rep}: {SPECS[k][0]}")
    finally:
        ctx.server_stop()


def test_cim_with_stages_is_refused_in_batches(ctx, cases):
    note("CIM-CAC with stages refused in a batch")
    p = cases[0][0]
    job = ctx.det_job(p["H"], p["y"], p["qam"], p["noise_var"], 16, 20, None, 1, stages=1,
                      cim={})
    with pytest.raises(M.MmgapError) as e:
        ctx.plan_create([job])
    assert e.value.code == -4
