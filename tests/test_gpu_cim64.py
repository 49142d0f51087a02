"""GPU parity of the CIM-CAC anneals of 33 to 64 spins (paper §2.3 Eqs.
cim1/cim2; the paper's 16-user move problem has 64 spins), two lanes per
anneal: identical spins, energies and divergence flags (bit for bit) and
winning chains against the oracle under the same Philox streams, for the
generic solver, every anneal's final state (diverging settings included),
detection by moves around the MMSE guess at 16x16 64-QAM, 8x8 64-QAM detection
(48 spins) and 16x16 VPP.
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
    (32, 2, [1, 1], 16, 64, 24, 12, True, 0, {}),          # 64 spins, 2 instances per wavefront
    (32, 2, [2, 1], 32, 40, 9, 3, False, 0, {"f_mvm": 1}), # 32 anneals: one instance per wavefront
    (20, 2, [1, 1], 48, 30, 7, 7, True, 1, {"amp0": 0.4}), # K 20 padded to 32; two wavefronts
    (16, 3, [4, 2, 1], 8, 50, 40, 8, True, 0, {}),         # 48 spins, four instances per wavefront
    (12, 3, [4, 2, 1], 64, 25, 5, 1, False, 0, {"f_mvm": 3, "eps": 0.4}),   # K 12 padded to 16
    (16, 4, [8, 4, 2, 1], 4, 30, 33, 11, True, 1, {"p": 1.1, "zeta": 0.5}),  # ragged tail
    (32, 2, [1, 1], 100, 20, 3, 1, True, 0, {"dt": 0.01}), # four wavefronts, last one partial
]


@pytest.mark.parametrize("K,q,w,chains,steps,n,ipg,fb,init,cim", SOLVE_CASES)
def test_cim64_solve_matches_oracle(ctx, K, q, w, chains, steps, n, ipg, fb, init, cim):
    note(f"cim64 solve K={K} q={q} chains={chains} steps={steps} n={n} ipg={ipg} {cim}")
    n_G = (n + ipg - 1) // ipg
    G, f = W.random_structured_ising(900 + K * 10 + q, n_G, ipg, K)
    f = f[:n]
    rng = np.random.default_rng(K + 11 * q)
    x_fb = None
    if fb:
        x_fb = (rng.choice([-1, 1], size=(n, K, q)) * np.array(w)).sum(-1).astype(np.int8)
    seed = W.job_seed(900 + K * 10 + q)
    sp, E, win = ctx.solve(dev(G), dev(f), K, q, w, chains, steps, None, seed,
                           x_fallback=None if x_fb is None else dev(x_fb), inst_per_G=ipg,
                           init=init, cim=cim)
    ref = O.cim_solve(G, f, K, q, np.array(w, np.int8), chains, steps, cim, seed, x_fb=x_fb,
                      inst_per_G=ipg, init_mode=init)
    assert np.array_equal(host(sp), ref["spins"])
    assert np.array_equal(host(E).view(np.uint32), ref["E"].view(np.uint32))
    assert np.array_equal(host(win), ref["win"])


@pytest.mark.parametrize("dt,f_mvm", [(0.02, 2), (0.32, 1)])
def test_cim64_chains_match_oracle(ctx, dt, f_mvm):
    """Every anneal's final spins, energy and divergence flag at 64 spins,
    including a step that diverges."""
    note(f"cim64 chains dt={dt} f_mvm={f_mvm}")
    K, q, w = 32, 2, [1, 1]
    G, f = W.random_structured_ising(41, 6, 4, K)
    steps = int(round(2.56 / dt))
    cim = dict(dt=dt, f_mvm=f_mvm)
    s, E, d = ctx.cim_chains(dev(G), dev(f), K, q, w, 6, steps, 5, inst_per_G=4, cim=cim)
    ref = O.cim_chains(G, f, K, q, np.array(w, np.int8), 6, steps, cim, 5, inst_per_G=4)
    assert np.array_equal(host(d), ref["diverged"])
    assert np.array_equal(host(s), ref["spins"])
    assert np.array_equal(host(E).view(np.uint32), ref["E"].view(np.uint32))


def test_cim64_moves_around_the_guess_16x16_64qam(ctx):
    """The paper's formulation: 16 users, moves around the MMSE guess (64 spins
    and the auxiliary one) annealed by CIM-CAC, two stages."""
    note("cim64 detect_delta 16x16 64-QAM 23x4 16 anneals x 64 steps, 2 stages")
    d = W.det_slot(3301, 16, 16, 64, 23, 4, 25.0)
    seed = W.job_seed(33)
    sym, met = ctx.detect_delta(dev(d.H), dev(d.y), 64, d.noise_var, 16, 64, None, seed,
                                stages=2, cim={})
    ref = O.detect_delta(d.H, d.y, d.noise_var, 64, 16, 64, None, seed, stages=2, cim={})
    met = host(met).astype(np.float64)
    assert_rows_equal(host(sym), ref["sym"], met, ref["metric"])
    assert np.allclose(met, ref["metric"], rtol=1e-4, atol=1e-6)


def test_cim64_detect_8x8_64qam(ctx):
    note("cim64 detect 8x8 64-QAM (48 spins) 13x4 32 anneals x 128 steps")
    d = W.det_slot(3302, 8, 8, 64, 13, 4, 25.0)
    seed = W.job_seed(34)
    sym, met = ctx.detect(dev(d.H), dev(d.y), 64, d.noise_var, 32, 128, None, seed, cim={})
    ref = O.detect(d.H, d.y, d.noise_var, 64, 32, 128, None, seed, cim={})
    met = host(met).astype(np.float64)
    assert_rows_equal(host(sym), ref["sym"], met, ref["metric"])
    assert np.allclose(met, ref["metric"], rtol=1e-4, atol=1e-6)


def test_cim64_vpp_16x16(ctx):
    note("cim64 vpp 16x16 16-QAM 5x3 32 anneals x 128 steps")
    s = W.vpp_slot(3303, 16, 16, 16, 5, 3)
    seed = W.job_seed(35)
    v, x, g = ctx.vpp_precode(dev(s.H), dev(s.u), 16, 32, 128, None, seed, cim={})
    ref = O.vpp_precode(s.H, s.u, 16, 32, 128, None, seed, cim={})
    gam = host(g).astype(np.float64)
    assert_rows_equal(host(v), ref["v"], gam, ref["gamma"])
    assert np.allclose(gam, ref["gamma"], rtol=1e-4, atol=1e-6)
