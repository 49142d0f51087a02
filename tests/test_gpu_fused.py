"""GPU parity of the persistent fused path (batch plans, one launch per batch).

Every job of a batch must produce outputs bit-identical to the single-job entry
point on the same arguments (which the parity suite checks against the oracle),
whatever else is in the batch, on every replay of the plan's graph; two jobs are
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return None if t is None else t.cpu().numpy()


# (kind, rows, cols, qam, n_sc, n_sym, chains, sweeps, init); one job per fused
# variant (KT, q) plus padding (K = 6), ragged symbol counts and 1/2/4
# wavefronts per instance
MIX = [
    ("det", 4, 4, 4, 21, 5, 32, 30, 0),      # KT 8,  q 1
    ("det", 8, 8, 16, 13, 7, 96, 25, 0),     # KT 16, q 2, two wavefronts per instance
    ("det", 16, 16, 64, 3, 3, 64, 10, 1),    # KT 32, q 3, MMSE start
    ("vpp", 8, 8, 16, 9, 3, 192, 20, 0),     # KT 16, q 2, four wavefronts per instance
    ("vpp", 4, 6, 64, 7, 2, 32, 25, 0),      # KT 8,  q 2
    ("det", 4, 3, 16, 11, 4, 64, 20, 0),     # K 6 padded to 8, q 2
    ("det", 16, 8, 64, 5, 6, 128, 15, 1),    # KT 16, q 3
    ("det", 32, 16, 4, 4, 2, 64, 10, 0),     # KT 32, q 1
    ("det", 4, 4, 64, 6, 3, 32, 20, 0),      # KT 8,  q 3
    ("det", 8, 8, 4, 5, 4, 64, 12, 0),       # KT 16, q 1
    ("vpp", 16, 16, 16, 3, 2, 64, 10, 0),    # KT 32, q 2
    # several instances per wavefront: 16, 8 and 1 chains (4, 8 and 16 per wavefront)
    ("det", 8, 8, 16, 7, 12, 16, 20, 0),     # KT 16, q 2
    ("vpp", 8, 8, 64, 5, 9, 8, 15, 0),       # KT 16, q 2
    ("det", 16, 16, 16, 3, 14, 16, 8, 1),    # KT 32, q 2
    ("det", 4, 4, 16, 6, 33, 1, 10, 0),      # KT 8, q 2, ragged 33 = 2 x 16 + 1
]


def make_inputs(i, spec):
    kind, a, b, qam, n_sc, n_sym, chains, sweeps, init = spec
    if kind == "det":
        d = W.det_slot(900 + i, a, b, qam, n_sc, n_sym, 24.0 if qam == 64 else 12.0)
        beta2 = W.linear_beta2(sweeps, *W.det_beta_range(qam, a, d.noise_var))
        return dict(kind=kind, H=dev(d.H), y=dev(d.y), qam=qam, noise_var=d.noise_var,
                    chains=chains, sweeps=sweeps, beta2=beta2, seed=W.job_seed(50 + i),
                    init=init, raw=d)
    s = W.vpp_slot(950 + i, a, b, qam, n_sc, n_sym)
    beta2 = W.linear_beta2(sweeps, *W.vpp_beta_range(qam, b))
    return dict(kind=kind, H=dev(s.H), y=dev(s.u), qam=qam, chains=chains, sweeps=sweeps,
                beta2=beta2, seed=W.job_seed(50 + i), init=init, raw=s)


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
        return dict(sym=host(sym), metric=host(met))
    v, x, g = ctx.vpp_precode(inp["H"], inp["y"], inp["qam"], inp["chains"], inp["sweeps"],
                              inp["beta2"], inp["seed"], init=inp["init"])
    return dict(v=host(v), x=host(x), gamma=host(g))


def outputs_of(job):
    torch.cuda.synchronize()
    return {k: (None if t is None else t.cpu().numpy()) for k, t in job["outputs"].items()}


def assert_same(got, ref, label):
    for k, r in ref.items():
        g = got[k]
        assert g is not None and r is not None, (label, k)
        # bitwise equality, NaN-safe for the float outputs
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


def test_fused_mixed_batch_equals_single_calls_on_every_replay(ctx, mix):
    inputs, refs = mix
    note(f"fused mixed batch of {len(inputs)} jobs, graph replays")
    jobs = [job_of(ctx, inp) for inp in inputs]
    plan = ctx.plan_create(jobs, graph=True)
    n_items, blocks = plan.plan_info()
    def per_item(chains):
        if chains <= 32:
            lanes = max(4, 1 << (chains - 1).bit_length())
            return 4 * (64 // lanes)
        return 4 // (1 if chains <= 64 else 2 if chains <= 128 else 4)
    assert n_items == sum(s[4] * -(-s[5] // per_item(s[6])) for s in MIX)
    assert 1 <= blocks <= n_items
    for rep in range(3):
        clear(jobs)
        a = torch.randn(256, 256, device="cuda:0")
        (a @ a).sum().item()                         # eager work between replays
        torch.cuda.synchronize()
        plan.plan_launch()
        for i, j in enumerate(jobs):
            assert_same(outputs_of(j), refs[i], f"replay {rep} job {i} {MIX[i]}")
    plan.plan_destroy()


def test_fused_without_graph_and_few_workgroups(ctx, mix):
    inputs, refs = mix
    note("fused mixed batch, direct launch, 3 workgroups")
    jobs = [job_of(ctx, inp) for inp in inputs]
    plan = ctx.plan_create(jobs, graph=False, blocks=3)
    assert plan.plan_info()[1] == 3
    plan.plan_launch()
    for i, j in enumerate(jobs):
        assert_same(outputs_of(j), refs[i], f"job {i} {MIX[i]}")
    plan.plan_destroy()


def test_fused_job_alone_equals_job_in_mix(ctx, mix):
    inputs, refs = mix
    note("fused single-job plans")
    for i in (1, 3, 7):
        job = job_of(ctx, inputs[i])
        plan = ctx.plan_create([job])
        plan.plan_launch()
        assert_same(outputs_of(job), refs[i], f"alone job {i}")
        plan.plan_destroy()


def test_fused_matches_oracle_directly(ctx, mix):
    inputs, _ = mix
    note("fused vs oracle, jobs 0 and 3")
    jobs = [job_of(ctx, inputs[i]) for i in (0, 3)]
    plan = ctx.plan_create(jobs)
    plan.plan_launch()
    got0, got3 = outputs_of(jobs[0]), outputs_of(jobs[1])
    plan.plan_destroy()
    d, p0 = inputs[0]["raw"], inputs[0]
    ref = O.detect(d.H, d.y, d.noise_var, p0["qam"], p0["chains"], p0["sweeps"], p0["beta2"],
                   p0["seed"], init_mode=p0["init"])
    assert np.array_equal(got0["sym"], ref["sym"])
    assert np.allclose(got0["metric"].astype(np.float64), ref["metric"], rtol=1e-4, atol=1e-6)
    s, p3 = inputs[3]["raw"], inputs[3]
    ref = O.vpp_precode(s.H, s.u, p3["qam"], p3["chains"], p3["sweeps"], p3["beta2"], p3["seed"])
    assert np.array_equal(got3["v"], ref["v"])
    assert np.allclose(got3["gamma"].astype(np.float64), ref["gamma"], rtol=1e-4, atol=1e-6)


def test_fused_reads_inputs_at_launch_time(ctx):
    note("fused plan relaunched after rewriting its inputs in place")
    spec = ("det", 8, 8, 16, 17, 5, 64, 20, 0)
    a, b = make_inputs(20, spec), make_inputs(21, spec)
    job = job_of(ctx, a)
    plan = ctx.plan_create([job])
    plan.plan_launch()
    assert_same(outputs_of(job), single_call(ctx, a), "before rewrite")
    a["H"].copy_(b["H"])
    a["y"].copy_(b["y"])
    plan.plan_launch()
    ref_b = single_call(ctx, dict(b, seed=a["seed"], beta2=a["beta2"], noise_var=a["noise_var"]))
    assert_same(outputs_of(job), ref_b, "after rewrite")
    plan.plan_destroy()


def test_fused_full_slot_8x8_16qam_equals_plain(ctx):
    """The benchmark slot (3276 subcarriers x 12 symbols, 8x8 16-QAM, 64 x 200)
    through one fused launch: every instance equal to the plain path's."""
    note("fused full slot 8x8 16-QAM 3276x12 64x200")
    d = W.det_slot(2000, 8, 8, 16, 3276, 12, 15.0)
    beta2 = W.linear_beta2(200, *W.det_beta_range(16, 8, d.noise_var))
    inp = dict(kind="det", H=dev(d.H), y=dev(d.y), qam=16, noise_var=d.noise_var, chains=64,
               sweeps=200, beta2=beta2, seed=W.job_seed(2000), init=0)
    ref = single_call(ctx, inp)
    job = job_of(ctx, inp)
    plan = ctx.plan_create([job])
    plan.plan_launch()
    plan.plan_launch()
    assert_same(outputs_of(job), ref, "full slot")
    plan.plan_destroy()


def test_fused_empty_and_errors(ctx):
    note("fused empty plans and argument errors")
    plan = ctx.plan_create([])
    assert plan.plan_info() == (0, 0)
    plan.plan_launch()
    plan.plan_destroy()
    H = torch.zeros((0, 4, 4), dtype=torch.complex64, device="cuda:0")
    y = torch.zeros((0, 3, 4), dtype=torch.complex64, device="cuda:0")
    job = ctx.det_job(H, y, 16, 0.1, 32, 5, np.ones(5, np.float32), 1)
    plan = ctx.plan_create([job])
    plan.plan_launch()
    torch.cuda.synchronize()
    plan.plan_destroy()

    inp = make_inputs(30, ("det", 4, 4, 16, 3, 2, 257, 5, 0))
    with pytest.raises(M.MmgapError) as e:
        ctx.plan_create([job_of(ctx, inp)])
    assert e.value.code == -4
    inp = make_inputs(31, ("det", 4, 4, 16, 3, 2, 32, 5, 0))
    j = job_of(ctx, inp)
    j["job"].out0 = None
    with pytest.raises(M.MmgapError) as e:
        ctx.plan_create([j])
    assert e.value.code == -1
    small = M.Context(0, hbm_budget=1 << 16)
    try:
        big = make_inputs(32, ("det", 8, 8, 16, 400, 12, 64, 5, 0))
        with pytest.raises(M.MmgapError) as e:
            small.plan_create([job_of(small, big)])
        assert e.value.code == -2
    finally:
        small.close()
