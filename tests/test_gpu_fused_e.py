"""GPU parity of MMGaP-E (paper §3.2 Fig. 6: stages of moves from the MMSE and
from the MMSE-SIC guess, the better answer) and of the search from the
MMSE-SIC guess alone inside persistent batch plans: a job with guesses != 0
must give sym, metric and from_sic bit-identical to mmgap_detect_e on the same
arguments (whose parity with the oracle is checked elsewhere), alone and mixed
with other jobs, on every replay of the plan's graph; sampled instances are
also checked against the oracle directly.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O
from workload import synth as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts only with -m gpu
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2510_01579_amd as M


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = M.Context(0)
    yield c
    c.close()


@pytest.fixture(params=[True, False], ids=["persistent", "routed"])
def persistent(request):
    """Plans with every job on the persistent kernels, or with the jobs the
    one-launch search can run routed to it (the default)."""
    return request.param


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


# (rows, cols, qam, n_sc, n_sym, snr, chains, sweeps, stages, guesses)
CASES = [
    (8, 8, 16, 13, 12, 15.0, 16, 8, 2, 3),       # KT 16, four instances per wavefront
    (16, 16, 64, 9, 12, 20.0, 4, 8, 3, 3),       # KT 32, sixteen instances per wavefront
    (16, 16, 64, 7, 12, 25.0, 4, 2, 1, 2),       # the MMSE-SIC guess alone
    (4, 4, 4, 33, 1, 10.0, 8, 4, 2, 1),          # KT 8, the MMSE guess through guesses
    (8, 8, 64, 5, 5, 25.0, 64, 4, 2, 3),         # one wavefront per instance
    (16, 16, 16, 3, 4, 15.0, 128, 3, 1, 3),      # two wavefronts per instance
    (12, 6, 16, 11, 3, 12.0, 16, 6, 2, 3),       # n_r != n_t, K 12 padded to 16
]


def make(i, spec):
    n_r, n_t, qam, n_sc, n_sym, snr, chains, sweeps, stages, guesses = spec
    d = W.det_slot(2700 + i, n_r, n_t, qam, n_sc, n_sym, snr)
    beta2 = W.linear_beta2(sweeps, *W.det_beta_range(qam, n_r, d.noise_var))
    return dict(H=dev(d.H), y=dev(d.y), qam=qam, noise_var=d.noise_var, chains=chains,
                sweeps=sweeps, beta2=beta2, seed=W.job_seed(270 + i), stages=stages,
                guesses=guesses, raw=d)


def single(ctx, inp):
    sym, met, fs = ctx.detect_e(inp["H"], inp["y"], inp["qam"], inp["noise_var"], inp["chains"],
                                inp["sweeps"], inp["beta2"], inp["seed"], stages=inp["stages"],
                                guesses=inp["guesses"])
    torch.cuda.synchronize()
    return dict(sym=sym.cpu().numpy(), metric=met.cpu().numpy(), from_sic=fs.cpu().numpy())


def job_of(ctx, inp):
    return ctx.det_job(inp["H"], inp["y"], inp["qam"], inp["noise_var"], inp["chains"],
                       inp["sweeps"], inp["beta2"], inp["seed"], stages=inp["stages"],
                       guesses=inp["guesses"])


def outs(job):
    torch.cuda.synchronize()
    return {k: t.cpu().numpy() for k, t in job["outputs"].items() if t is not None}


def assert_same(got, ref, label):
    for k, r in ref.items():
        g = got[k]
        assert g.shape == r.shape and g.tobytes() == r.tobytes(), \
            f"{label}: {k} differs in {int(np.sum(np.any((g != r).reshape(len(g), -1), axis=1)))} rows"


@pytest.mark.parametrize("i", range(len(CASES)))
def test_plan_job_equals_detect_e(ctx, i, persistent):
    spec = CASES[i]
    note(f"fused E job {spec}")
    inp = make(i, spec)
    ref = single(ctx, inp)
    job = job_of(ctx, inp)
    plan = ctx.plan_create([job], graph=True, persistent=persistent)
    for rep in range(2):
        for t in job["outputs"].values():
            t.zero_()
        plan.plan_launch()
        assert_same(outs(job), ref, f"case {i} replay {rep}")
    plan.plan_destroy()


def test_e_jobs_in_a_mix_on_every_replay(ctx, persistent):
    note("fused E jobs beside delta, binary and VPP jobs, graph replays")
    inputs = [make(i, s) for i, s in enumerate(CASES[:4])]
    refs = [single(ctx, inp) for inp in inputs]
    jobs = [job_of(ctx, inp) for inp in inputs]
    d2 = W.det_slot(2790, 8, 8, 16, 9, 4, 15.0)
    b2 = W.linear_beta2(20, *W.det_beta_range(16, 8, d2.noise_var))
    H2, y2 = dev(d2.H), dev(d2.y)
    jobs.append(ctx.det_job(H2, y2, 16, d2.noise_var, 32, 20, b2, W.job_seed(2790), stages=2))
    jobs.append(ctx.det_job(H2, y2, 16, d2.noise_var, 64, 20, b2, W.job_seed(2791)))
    v = W.vpp_slot(2792, 8, 8, 16, 5, 3)
    bv = W.linear_beta2(20, *W.vpp_beta_range(16, 8))
    jobs.append(ctx.vpp_job(dev(v.H), dev(v.u), 16, 32, 20, bv, W.job_seed(2792)))
    d_ref = ctx.detect_delta(H2, y2, 16, d2.noise_var, 32, 20, b2, W.job_seed(2790), stages=2)
    b_ref = ctx.detect(H2, y2, 16, d2.noise_var, 64, 20, b2, W.job_seed(2791))
    torch.cuda.synchronize()
    plan = ctx.plan_create(jobs, graph=True, persistent=persistent)
    for rep in range(3):
        for j in jobs:
            for t in j["outputs"].values():
                if t is not None:
                    t.zero_()
        plan.plan_launch()
        for k, inp in enumerate(inputs):
            assert_same(outs(jobs[k]), refs[k], f"mix job {k} replay {rep}")
        o = outs(jobs[4])
        assert o["sym"].tobytes() == d_ref[0].cpu().numpy().tobytes()
        o = outs(jobs[5])
        assert o["sym"].tobytes() == b_ref[0].cpu().numpy().tobytes()
    plan.plan_destroy()


@pytest.mark.parametrize("i", [0, 1, 2])
def test_plan_job_matches_the_oracle_on_sampled_instances(ctx, i, persistent):
    spec = CASES[i]
    note(f"fused E job vs oracle {spec}")
    inp = make(i, spec)
    job = job_of(ctx, inp)
    plan = ctx.plan_create([job], graph=False, persistent=persistent)
    plan.plan_launch()
    got = outs(job)
    plan.plan_destroy()
    d = inp["raw"]
    n = d.y.shape[0] * d.y.shape[1]
    rng = np.random.default_rng(2799 + i)
    ids = np.unique(np.concatenate([[0, n - 1], rng.choice(n, size=min(n, 24), replace=False)]))
    ref = O.detect_e(d.H, d.y, d.noise_var, inp["qam"], inp["chains"], inp["sweeps"],
                     inp["beta2"], inp["seed"], stages=inp["stages"], inst_ids=ids,
                     guesses=inp["guesses"])
    assert np.array_equal(got["sym"][ids], ref["sym"])
    assert np.allclose(got["metric"][ids].astype(np.float64), ref["metric"], rtol=1e-4, atol=1e-6)
    assert np.array_equal(got["from_sic"][ids].astype(bool), ref["from_sic"])


def test_guess_arguments_are_checked(ctx):
    note("fused E argument checks")
    inp = make(0, CASES[0])
    bad = ctx.det_job(inp["H"], inp["y"], inp["qam"], inp["noise_var"], 16, 4, inp["beta2"][:4],
                      inp["seed"], stages=0, guesses=3)
    with pytest.raises(RuntimeError, match="stages"):
        ctx.plan_create([bad])
    bad = ctx.det_job(inp["H"], inp["y"], inp["qam"], inp["noise_var"], 16, 4, inp["beta2"][:4],
                      inp["seed"], stages=1, guesses=4)
    with pytest.raises(RuntimeError, match="guesses"):
        ctx.plan_create([bad])
