"""Subcarrier shards of a slot (paper §5.3 "Execution Time": the subcarriers of
a slot are split over GPUs, each solving its share with no exchange).

A call on subcarriers [a, b) of a slot with schedule.inst_base = a * n_sym must
draw the random numbers of those instances in the whole-slot call, so the
shards' outputs, concatenated, are byte for byte the whole slot's -- for every
entry point that anneals (detection, VPP, moves around a guess, MMGaP-E, the
generic solver and the persistent batches).  The shards are also checked
against the oracle evaluated at the instances' slot-wide indices.
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

N_SC, N_SYM = 40, 12
CUTS = (0, 17, 31, N_SC)          # three shards, ragged


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


def shards(call, H, y):
    """Outputs of `call(H_part, y_part, inst_base)` over CUTS, concatenated."""
    parts = []
    for a, b in zip(CUTS[:-1], CUTS[1:]):
        outs = call(dev(H[a:b]), dev(y[a:b]), a * N_SYM)
        parts.append([host(o) for o in outs])
    return [None if p[0] is None else np.concatenate(p) for p in zip(*parts)]


def assert_bytes_equal(whole, parts):
    for w, p in zip(whole, parts):
        if w is None:
            assert p is None
        else:
            assert w.tobytes() == p.tobytes()


def test_detect_shards_equal_whole_slot(ctx):
    note("detect 8x8 16-QAM, 40 subcarriers in 3 shards")
    d = W.det_slot(8101, 8, 8, 16, N_SC, N_SYM, 15.0)
    b2 = W.linear_beta2(30, *W.det_beta_range(16, 8, d.noise_var))
    seed = W.job_seed(8101)
    whole = [host(o) for o in ctx.detect(dev(d.H), dev(d.y), 16, d.noise_var, 64, 30, b2, seed)]
    parts = shards(lambda H, y, ib: ctx.detect(H, y, 16, d.noise_var, 64, 30, b2, seed,
                                               inst_base=ib), d.H, d.y)
    assert_bytes_equal(whole, parts)
    # the last shard against the oracle at its slot-wide instance indices
    ids = np.arange(CUTS[-2] * N_SYM, N_SC * N_SYM, dtype=np.uint32)
    ref = O.detect(d.H, d.y, d.noise_var, 16, 64, 30, b2, seed, inst_ids=ids)
    assert np.array_equal(parts[0][ids], ref["sym"])
    assert np.allclose(parts[1][ids].astype(np.float64), ref["metric"], rtol=1e-4, atol=1e-6)


def test_shard_differs_without_offset(ctx):
    """Without inst_base a shard draws the streams of the slot's first
    instances: the offset is what makes the shards agree."""
    note("detect shard without inst_base")
    d = W.det_slot(8102, 4, 4, 4, 64, 1, 6.0)
    b2 = W.linear_beta2(6, *W.det_beta_range(4, 4, d.noise_var))
    seed = W.job_seed(8102)
    a = 32
    ids = np.arange(a, 64, dtype=np.uint32)
    with_off = host(ctx.detect(dev(d.H[a:]), dev(d.y[a:]), 4, d.noise_var, 8, 6, b2, seed,
                               inst_base=a)[0])
    without = host(ctx.detect(dev(d.H[a:]), dev(d.y[a:]), 4, d.noise_var, 8, 6, b2, seed)[0])
    ref = O.detect(d.H, d.y, d.noise_var, 4, 8, 6, b2, seed, inst_ids=ids)
    ref0 = O.detect(d.H[a:], d.y[a:], d.noise_var, 4, 8, 6, b2, seed)
    assert np.array_equal(with_off, ref["sym"])
    assert np.array_equal(without, ref0["sym"])


def test_vpp_shards_equal_whole_slot(ctx):
    note("VPP 8x8 16-QAM, 40 subcarriers in 3 shards")
    s = W.vpp_slot(8201, 8, 8, 16, N_SC, N_SYM)
    b2 = W.linear_beta2(25, *W.vpp_beta_range(16, 8))
    seed = W.job_seed(8201)
    whole = [host(o) for o in ctx.vpp_precode(dev(s.H), dev(s.u), 16, 64, 25, b2, seed)]
    parts = shards(lambda H, u, ib: ctx.vpp_precode(H, u, 16, 64, 25, b2, seed, inst_base=ib),
                   s.H, s.u)
    assert_bytes_equal(whole, parts)
    ids = np.arange(CUTS[1] * N_SYM, CUTS[2] * N_SYM, dtype=np.uint32)
    ref = O.vpp_precode(s.H, s.u, 16, 64, 25, b2, seed, inst_ids=ids)
    assert np.array_equal(parts[0][ids], ref["v"])


def test_delta_and_mmgap_e_shards_equal_whole_slot(ctx):
    note("detect_delta (2 stages) and detect_e, 16x16 64-QAM, 3 shards")
    d = W.det_slot(8301, 16, 16, 64, N_SC, N_SYM, 25.0)
    b2 = W.linear_beta2(6, *W.det_beta_range(64, 16, d.noise_var))
    seed = W.job_seed(8301)
    whole = [host(o) for o in ctx.detect_delta(dev(d.H), dev(d.y), 64, d.noise_var, 16, 6, b2,
                                               seed, stages=2)]
    parts = shards(lambda H, y, ib: ctx.detect_delta(H, y, 64, d.noise_var, 16, 6, b2, seed,
                                                     stages=2, inst_base=ib), d.H, d.y)
    assert_bytes_equal(whole, parts)
    ids = np.arange(CUTS[-2] * N_SYM, N_SC * N_SYM, dtype=np.uint32)
    ref = O.detect_delta(d.H, d.y, d.noise_var, 64, 16, 6, b2, seed, stages=2, inst_ids=ids)
    assert np.array_equal(parts[0][ids], ref["sym"])

    whole = [host(o) for o in ctx.detect_e(dev(d.H), dev(d.y), 64, d.noise_var, 16, 6, b2, seed,
                                           stages=1)]
    parts = shards(lambda H, y, ib: ctx.detect_e(H, y, 64, d.noise_var, 16, 6, b2, seed,
                                                 stages=1, inst_base=ib), d.H, d.y)
    assert_bytes_equal(whole, parts)
    ref = O.detect_e(d.H, d.y, d.noise_var, 64, 16, 6, b2, seed, stages=1, inst_ids=ids)
    assert np.array_equal(parts[0][ids], ref["sym"])


def test_solve_offset_matches_oracle_ids(ctx):
    note("solve K=16 q=2 with inst_base = 1000")
    n, ipg = 23, 1
    G, f = W.random_structured_ising(8401, n, ipg, 16)
    b2 = W.linear_beta2(12, 0.05, 2.0)
    seed = W.job_seed(8401)
    sp, E, win = ctx.solve(dev(G), dev(f), 16, 2, [2, 1], 64, 12, b2, seed, inst_base=1000)
    ids = np.arange(1000, 1000 + n, dtype=np.uint32)
    # the oracle's G index is inst_id / inst_per_G, so the couplings are laid out
    # at their slot-wide positions
    Gfull = np.zeros((1000 + n, 16, 16), np.float32)
    Gfull[1000:] = G
    ref = O.solve(Gfull, f, 16, 2, np.array([2, 1], np.int8), 64, 12, b2, seed, inst_ids=ids)
    assert np.array_equal(host(sp), ref["spins"])
    assert np.array_equal(host(E).view(np.uint32), ref["E"].view(np.uint32))
    assert np.array_equal(host(win), ref["win"])


def test_plan_of_shards_equals_whole_slot_plan(ctx):
    """The persistent batches: one plan holding the shards as separate jobs
    (detection around the MMSE guess and VPP) gives the whole-slot jobs' bytes."""
    note("fused plans: shards as jobs vs whole-slot jobs")
    d = W.det_slot(8501, 16, 16, 64, N_SC, N_SYM, 20.0)
    s = W.vpp_slot(8502, 8, 8, 16, N_SC, N_SYM)
    b2d = W.linear_beta2(6, *W.det_beta_range(64, 16, d.noise_var))
    b2v = W.linear_beta2(20, *W.vpp_beta_range(16, 8))
    sd, sv = W.job_seed(8501), W.job_seed(8502)
    Hd, yd, Hv, uv = dev(d.H), dev(d.y), dev(s.H), dev(s.u)
    whole = [ctx.det_job(Hd, yd, 64, d.noise_var, 16, 6, b2d, sd, stages=2),
             ctx.vpp_job(Hv, uv, 16, 64, 20, b2v, sv)]
    p = ctx.plan_create(whole, graph=True)
    p.plan_launch()
    torch.cuda.synchronize()
    jobs = []
    for a, b in zip(CUTS[:-1], CUTS[1:]):
        jobs.append(ctx.det_job(dev(d.H[a:b]), dev(d.y[a:b]), 64, d.noise_var, 16, 6, b2d, sd,
                                stages=2, inst_base=a * N_SYM))
        jobs.append(ctx.vpp_job(dev(s.H[a:b]), dev(s.u[a:b]), 16, 64, 20, b2v, sv,
                                inst_base=a * N_SYM))
    q = ctx.plan_create(jobs, graph=True)
    for _ in range(2):                       # two replays of the graph
        q.plan_launch()
        torch.cuda.synchronize()
        for k, name in ((0, "sym"), (0, "metric"), (1, "v"), (1, "x"), (1, "gamma")):
            w = host(whole[k]["outputs"][name])
            parts = np.concatenate([host(j["outputs"][name]) for j in jobs[k::2]])
            assert w.tobytes() == parts.tobytes(), name
    p.plan_destroy()
    q.plan_destroy()
