"""GPU parity of the CIM-CAC anneals (paper §2.3 Eqs. cim1/cim2, Euler
integration as in §3.2 and Appendix A) against the oracle: identical spins,
energies (bit for bit) and winning chains under the same Philox streams, for
the generic solver, detection and VPP, plus the argument checks.
"""
import math
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


def assert_rows_equal(gpu, ora, e_gpu=None, e_ora=None, frac=1e-4, tol=1e-5):
    gpu = np.asarray(gpu).reshape(len(gpu), -1)
    ora = np.asarray(ora).reshape(len(ora), -1)
    bad = np.where(np.any(gpu != ora, axis=1))[0]
    assert len(bad) <= int(math.floor(frac * len(gpu))), f"{len(bad)} of {len(gpu)} differ: {bad[:10]}"
    if len(bad):
        assert e_gpu is not None
        assert np.all(np.abs(np.asarray(e_gpu)[bad] - np.asarray(e_ora)[bad]) < tol)


SOLVE_CASES = [
    # K, q, w, chains, steps, n, inst_per_G, fallback, init, constants
    (8, 1, [1], 32, 128, 37, 1, False, 0, {}),
    (16, 2, [2, 1], 64, 64, 23, 4, True, 0, {}),
    (5, 2, [2, 1], 64, 40, 13, 1, True, 1, {"amp0": 0.5}),
    (16, 1, [1], 128, 30, 9, 3, True, 0, {"f_mvm": 1}),
    (32, 1, [1], 64, 25, 7, 7, True, 0, {"f_mvm": 3, "eps": 0.4}),
    (8, 4, [8, 4, 2, 1], 64, 30, 11, 1, False, 0, {"p": 1.1, "zeta": 0.5}),
    (8, 3, [4, 2, 1], 16, 50, 40, 8, True, 1, {}),        # four instances per wavefront
    (16, 2, [2, 1], 8, 40, 33, 8, True, 0, {"dt": 0.01}),  # eight per wavefront, ragged tail
    (4, 2, [2, 1], 1, 20, 130, 64, False, 0, {}),          # sixteen per wavefront
]


@pytest.mark.parametrize("K,q,w,chains,steps,n,ipg,fb,init,cim", SOLVE_CASES)
def test_cim_solve_matches_oracle(ctx, K, q, w, chains, steps, n, ipg, fb, init, cim):
    note(f"cim solve K={K} q={q} chains={chains} steps={steps} n={n} ipg={ipg} {cim}")
    n_G = (n + ipg - 1) // ipg
    G, f = W.random_structured_ising(300 + K * 10 + q, n_G, ipg, K)
    f = f[:n]
    rng = np.random.default_rng(K + 7 * q)
    x_fb = None
    if fb:
        x_fb = (rng.choice([-1, 1], size=(n, K, q)) * np.array(w)).sum(-1).astype(np.int8)
    seed = W.job_seed(500 + K * 10 + q)
    sp, E, win = ctx.solve(dev(G), dev(f), K, q, w, chains, steps, None, seed,
                           x_fallback=None if x_fb is None else dev(x_fb), inst_per_G=ipg,
                           init=init, cim=cim)
    ref = O.cim_solve(G, f, K, q, np.array(w, np.int8), chains, steps, cim, seed, x_fb=x_fb,
                      inst_per_G=ipg, init_mode=init)
    assert np.array_equal(host(sp), ref["spins"])
    assert np.array_equal(host(E).view(np.uint32), ref["E"].view(np.uint32))
    assert np.array_equal(host(win), ref["win"])


DET_CASES = [
    # n_r, n_t, qam, n_sc, n_sym, snr, chains, steps, init
    (4, 4, 4, 64, 1, 10.0, 32, 128, 0),     # the 4x4 QPSK slot with the paper's 32 anneals
    (8, 8, 4, 21, 3, 10.0, 32, 128, 0),
    (8, 8, 16, 13, 4, 15.0, 64, 128, 1),
    (16, 16, 4, 5, 2, 8.0, 32, 64, 0),
    (6, 3, 16, 9, 5, 15.0, 16, 100, 0),
]


@pytest.mark.parametrize("n_r,n_t,qam,n_sc,n_sym,snr,chains,steps,init", DET_CASES)
def test_cim_detect_matches_oracle(ctx, n_r, n_t, qam, n_sc, n_sym, snr, chains, steps, init):
    note(f"cim detect {n_r}x{n_t} qam={qam} {n_sc}x{n_sym} {chains}x{steps} init={init}")
    d = W.det_slot(700 + n_t + qam, n_r, n_t, qam, n_sc, n_sym, snr)
    seed = W.job_seed(9)
    sym, met = ctx.detect(dev(d.H), dev(d.y), qam, d.noise_var, chains, steps, None, seed,
                          init=init, cim={})
    ref = O.detect(d.H, d.y, d.noise_var, qam, chains, steps, None, seed, init_mode=init, cim={})
    met = host(met).astype(np.float64)
    assert_rows_equal(host(sym), ref["sym"], met, ref["metric"])
    assert np.allclose(met, ref["metric"], rtol=1e-4, atol=1e-6)


@pytest.mark.parametrize("n_u,n_t,n_sc,n_sym,chains,steps", [(8, 8, 11, 3, 32, 128),
                                                             (4, 6, 7, 2, 64, 80)])
def test_cim_vpp_matches_oracle(ctx, n_u, n_t, n_sc, n_sym, chains, steps):
    note(f"cim vpp {n_u}x{n_t} {n_sc}x{n_sym} {chains}x{steps}")
    s = W.vpp_slot(800 + n_u, n_u, n_t, 16, n_sc, n_sym)
    seed = W.job_seed(10)
    v, x, g = ctx.vpp_precode(dev(s.H), dev(s.u), 16, chains, steps, None, seed, cim={})
    ref = O.vpp_precode(s.H, s.u, 16, chains, steps, None, seed, cim={})
    gam = host(g).astype(np.float64)
    assert_rows_equal(host(v), ref["v"], gam, ref["gamma"])
    assert np.allclose(gam, ref["gamma"], rtol=1e-4, atol=1e-6)


def test_cim_full_slot_8x8_16qam_sampled(ctx):
    """The 8x8 16-QAM slot (3276 x 12) with 32 anneals of 128 steps, the
    launch the benchmark's CIM leg times; the oracle recomputes a sample."""
    note("cim full slot 8x8 16-QAM 3276x12 32x128")
    d = W.det_slot(2001, 8, 8, 16, 3276, 12, 15.0)
    seed = W.job_seed(2001)
    sym, met = ctx.detect(dev(d.H), dev(d.y), 16, d.noise_var, 32, 128, None, seed, cim={})
    sym, met = host(sym), host(met).astype(np.float64)
    rng = np.random.default_rng(3)
    ids = np.unique(np.concatenate([rng.choice(3276 * 12, 200, replace=False),
                                    [0, 11, 12, 3276 * 12 - 1]])).astype(np.uint32)
    ref = O.detect(d.H, d.y, d.noise_var, 16, 32, 128, None, seed, inst_ids=ids, cim={})
    assert_rows_equal(sym[ids], ref["sym"], met[ids], ref["metric"])
    assert np.allclose(met[ids], ref["metric"], rtol=1e-4, atol=1e-6)


def test_cim_arguments(ctx):
    note("cim argument errors")
    d = W.det_slot(5, 16, 16, 64, 3, 2, 20.0)
    H, y = dev(d.H), dev(d.y)
    with pytest.raises(M.MmgapError) as e:          # 16x16 64-QAM: 96 spins
        ctx.detect(H, y, 64, d.noise_var, 32, 10, None, 1, cim={})
    assert e.value.code == -4
    d = W.det_slot(6, 4, 4, 16, 3, 2, 20.0)
    H, y = dev(d.H), dev(d.y)
    for bad in ({"dt": 0.0}, {"f_mvm": 0}, {"eps": float("nan")}):
        with pytest.raises(M.MmgapError) as e:
            ctx.detect(H, y, 16, d.noise_var, 32, 10, None, 1, cim=bad)
        assert e.value.code == -1, bad
    job = ctx.det_job(H, y, 16, d.noise_var, 32, 10, None, 1, stages=1, cim={})
    with pytest.raises(M.MmgapError) as e:          # batches: CIM-CAC without stages only
        ctx.plan_create([job])
    assert e.value.code == -4


@pytest.mark.parametrize("dt,f_mvm", [(0.01, 1), (0.08, 4), (0.32, 1)])
def test_cim_chains_match_oracle(ctx, dt, f_mvm):
    """Every anneal's final spins, energy and divergence flag (the Appendix A
    study's raw data), including settings that diverge."""
    note(f"cim chains dt={dt} f_mvm={f_mvm}")
    from paper_2510_01579_amd import cim_integration as CI
    K = 16
    G, f = CI.instances(11, 48, K)
    steps = int(round(2.56 / dt))
    s, E, d = ctx.cim_chains(dev(G), dev(f), K, 1, [1], 2, steps, 5, cim=dict(dt=dt, f_mvm=f_mvm))
    ref = O.cim_chains(G, f, K, 1, np.array([1], np.int8), 2, steps, dict(dt=dt, f_mvm=f_mvm), 5)
    assert np.array_equal(host(d), ref["diverged"])
    assert np.array_equal(host(s), ref["spins"])
    assert np.array_equal(host(E).view(np.uint32), ref["E"].view(np.uint32))


def test_cim_integration_study_matches_oracle_metrics(ctx):
    note("cim integration study, 64 instances, 2 x 2 grid")
    from paper_2510_01579_amd import cim_integration as CI
    res = CI.run(ctx, n_inst=64, n_spins=12, seed=4, dts=(0.02, 0.16), fmvms=(1, 4))
    G, f = CI.instances(4, 64, 12)
    w = np.array([1], np.int8)
    ref = O.cim_chains(G, f, 12, 1, w, 1, 256, dict(dt=0.01, f_mvm=1), 5)
    for row in res["grid"]:
        r = O.cim_chains(G, f, 12, 1, w, 1, row["steps"], dict(dt=row["dt"], f_mvm=row["f_mvm"]), 5)
        m = O.cim_integration_metrics(ref["spins"], ref["diverged"], r["spins"], r["diverged"])
        assert row["p_diverge"] == m["p_diverge"]
        assert (row["p_error"] is None and m["compared"] == 0) or row["p_error"] == m["p_error"]


def test_cim_chains_arguments(ctx):
    note("cim chains argument errors")
    G = torch.zeros((2, 8, 8), dtype=torch.float32, device="cuda:0")
    f = torch.zeros((2, 8), dtype=torch.float32, device="cuda:0")
    import ctypes
    s, keep = M.Context._schedule(4, 10, np.ones(10, np.float32), 1, 0, None)   # Metropolis
    wv = (ctypes.c_byte * 1)(1)
    out = torch.empty((2, 4, 8), dtype=torch.int8, device="cuda:0")
    rc = M.lib().mmgap_cim_chains(ctx._h, 2, 8, 1, wv, M._ptr(G), 1, M._ptr(f), None,
                                  ctypes.byref(s), M._ptr(out), None, None, M._stream(ctx._dev()))
    assert rc == -1
    with pytest.raises(M.MmgapError) as e:                  # 96 spins
        ctx.cim_chains(torch.zeros((1, 32, 32), dtype=torch.float32, device="cuda:0"),
                       torch.zeros((1, 32), dtype=torch.float32, device="cuda:0"), 32, 3,
                       [4, 2, 1], 1, 10, 1)
    assert e.value.code == -4


def test_cim_chains_empty_and_padded(ctx):
    """No instances: nothing to do; K = 5 padded to 8: the padded spins are
    neither returned nor checked for divergence."""
    note("cim chains: empty and padded")
    G = torch.empty((0, 5, 5), dtype=torch.float32, device="cuda:0")
    f = torch.empty((0, 5), dtype=torch.float32, device="cuda:0")
    s, E, d = ctx.cim_chains(G, f, 5, 2, [2, 1], 4, 10, 1)
    assert s.shape == (0, 4, 10)
    Gn, fn = W.random_structured_ising(77, 9, 1, 5)
    s, E, d = ctx.cim_chains(dev(Gn), dev(fn), 5, 2, [2, 1], 3, 40, 2, cim=dict(dt=0.16))
    ref = O.cim_chains(Gn, fn, 5, 2, np.array([2, 1], np.int8), 3, 40, dict(dt=0.16), 2)
    assert np.array_equal(host(s), ref["spins"])
    assert np.array_equal(host(d), ref["diverged"])
    assert np.array_equal(host(E).view(np.uint32), ref["E"].view(np.uint32))
