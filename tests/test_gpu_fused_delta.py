"""GPU parity of detection by moves around a guess (paper §2.3 Delta-Ising form,
§3.2 MMGaP-E stages) inside the persistent fused kernel: a batch job with
stages >= 1 must give outputs bit-identical to mmgap_detect_delta on the same
arguments (whose parity with the oracle is checked elsewhere), alone, mixed
with plain jobs, on every replay of the plan's graph, and at the full 16x16
64-QAM slot; one job is also checked against the oracle directly.
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


def host(t):
    torch.cuda.synchronize()
    return None if t is None else t.cpu().numpy()


# (rows, cols, qam, n_sc, n_sym, snr, chains, sweeps, stages, init); stages = 0
# is a plain job of the same shape
MIX = [
    (8, 8, 16, 13, 7, 15.0, 32, 30, 1, 0),      # KT 16, one wavefront per instance
    (8, 8, 64, 9, 5, 25.0, 64, 25, 3, 0),       # KT 16, 64-QAM clamp
    (16, 16, 64, 3, 3, 25.0, 32, 20, 2, 1),     # KT 32, chains started at the zero move
    (4, 4, 16, 21, 5, 12.0, 16, 30, 2, 0),      # KT 8, four instances per wavefront
    (6, 3, 16, 11, 4, 15.0, 128, 15, 2, 0),     # K 6 padded to 8, two wavefronts per instance
    (16, 16, 64, 2, 14, 25.0, 8, 12, 1, 0),     # KT 32, eight instances per wavefront
    (8, 8, 16, 7, 3, 15.0, 64, 20, 0, 0),       # plain jobs beside the delta ones
    (16, 16, 64, 3, 3, 25.0, 64, 10, 0, 1),
]


def make_inputs(i, spec):
    n_r, n_t, qam, n_sc, n_sym, snr, chains, sweeps, stages, init = spec
    d = W.det_slot(1700 + i, n_r, n_t, qam, n_sc, n_sym, snr)
    beta2 = W.linear_beta2(sweeps, *W.det_beta_range(qam, n_r, d.noise_var))
    return dict(H=dev(d.H), y=dev(d.y), qam=qam, noise_var=d.noise_var, chains=chains,
                sweeps=sweeps, beta2=beta2, seed=W.job_seed(70 + i), stages=stages, init=init,
                raw=d)


def job_of(ctx, inp):
    return ctx.det_job(inp["H"], inp["y"], inp["qam"], inp["noise_var"], inp["chains"],
                       inp["sweeps"], inp["beta2"], inp["seed"], init=inp["init"],
                       stages=inp["stages"])


def single_call(ctx, inp):
    args = (inp["H"], inp["y"], inp["qam"], inp["noise_var"], inp["chains"], inp["sweeps"],
            inp["beta2"], inp["seed"])
    if inp["stages"] > 0:
        sym, met = ctx.detect_delta(*args, stages=inp["stages"], init=inp["init"])
    else:
        sym, met = ctx.detect(*args, init=inp["init"])
    return dict(sym=host(sym), metric=host(met))


def outputs_of(job):
    torch.cuda.synchronize()
    return {k: (None if t is None else t.cpu().numpy()) for k, t in job["outputs"].items()}


def assert_same(got, ref, label):
    for k, r in ref.items():
        g = got[k]
        assert g is not None and r is not None, (label, k)
        assert g.shape == r.shape and g.view(np.uint8).tobytes() == r.view(np.uint8).tobytes(), \
            f"{label}: {k} differs in {int(np.sum(np.any((g != r).reshape(len(g), -1), axis=1)))} rows"


def clear(jobs):
    for j in jobs:
        for t in j["outputs"].values():
            if t is not None:
                t.zero_()


@pytest.fixture(scope="module")
def mix(ctx):
    inputs = [make_inputs(i, s) for i, s in enumerate(MIX)]
    refs = [single_call(ctx, inp) for inp in inputs]
    return inputs, refs


def test_fused_delta_batch_equals_single_calls_on_every_replay(ctx, mix, persistent):
    inputs, refs = mix
    note(f"fused delta batch of {len(inputs)} jobs, graph replays")
    jobs = [job_of(ctx, inp) for inp in inputs]
    plan = ctx.plan_create(jobs, graph=True, persistent=persistent)
    for rep in range(3):
        clear(jobs)
        a = torch.randn(256, 256, device="cuda:0")
        (a @ a).sum().item()                         # eager work between replays
        torch.cuda.synchronize()
        plan.plan_launch()
        for i, j in enumerate(jobs):
            assert_same(outputs_of(j), refs[i], f"replay {rep} job {i} {MIX[i]}")
    plan.plan_destroy()


def test_fused_delta_direct_launch_few_workgroups(ctx, mix, persistent):
    inputs, refs = mix
    note("fused delta batch, direct launch, 2 workgroups")
    jobs = [job_of(ctx, inp) for inp in inputs]
    plan = ctx.plan_create(jobs, graph=False, blocks=2, persistent=persistent)
    plan.plan_launch()
    for i, j in enumerate(jobs):
        assert_same(outputs_of(j), refs[i], f"job {i} {MIX[i]}")
    plan.plan_destroy()


def test_fused_delta_job_alone(ctx, mix):
    inputs, refs = mix
    note("fused delta single-job plans")
    for i in (1, 3, 5):
        job = job_of(ctx, inputs[i])
        plan = ctx.plan_create([job])
        plan.plan_launch()
        assert_same(outputs_of(job), refs[i], f"alone job {i}")
        plan.plan_destroy()


def test_fused_delta_matches_oracle_directly(ctx, mix, persistent):
    inputs, _ = mix
    note("fused delta vs oracle, job 1")
    p = inputs[1]
    job = job_of(ctx, p)
    plan = ctx.plan_create([job], persistent=persistent)
    plan.plan_launch()
    got = outputs_of(job)
    plan.plan_destroy()
    d = p["raw"]
    ref = O.detect_delta(d.H, d.y, d.noise_var, p["qam"], p["chains"], p["sweeps"], p["beta2"],
                         p["seed"], stages=p["stages"], init_mode=p["init"])
    assert np.array_equal(got["sym"], ref["sym"])
    assert np.allclose(got["metric"].astype(np.float64), ref["metric"], rtol=1e-4, atol=1e-6)


def test_fused_delta_full_slot_16x16_64qam(ctx, persistent):
    """The 16x16 64-QAM slot (3276 x 12, 25 dB), 16 chains x 25 sweeps, two
    stages around the MMSE guess, chains started at the zero move: the plan
    equals the multi-launch entry point."""
    note("fused delta full slot 16x16 64-QAM 3276x12 16x25 2 stages init 1")
    d = W.det_slot(3001, 16, 16, 64, 3276, 12, 25.0)
    beta2 = W.linear_beta2(25, *W.det_beta_range(64, 16, d.noise_var))
    inp = dict(H=dev(d.H), y=dev(d.y), qam=64, noise_var=d.noise_var, chains=16, sweeps=25,
               beta2=beta2, seed=W.job_seed(3001), stages=2, init=1)
    ref = single_call(ctx, inp)
    job = job_of(ctx, inp)
    plan = ctx.plan_create([job], persistent=persistent)
    plan.plan_launch()
    assert_same(outputs_of(job), ref, "full slot")
    plan.plan_destroy()


def test_fused_delta_refusals(ctx):
    note("fused delta argument errors")
    s = W.vpp_slot(5, 4, 4, 16, 3, 2)
    b = np.ones(10, np.float32)
    job = ctx.vpp_job(dev(s.H), dev(s.u), 16, 32, 10, b, 1)
    job["job"].stages = 1
    with pytest.raises(M.MmgapError) as e:            # VPP runs no stages
        ctx.plan_create([job])
    assert e.value.code == -4
    d = W.det_slot(6, 4, 4, 16, 3, 2, 20.0)
    job = ctx.det_job(dev(d.H), dev(d.y), 16, d.noise_var, 32, 10, b, 1, stages=65)
    with pytest.raises(M.MmgapError) as e:
        ctx.plan_create([job])
    assert e.value.code == -4
