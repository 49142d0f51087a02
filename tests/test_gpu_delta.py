"""GPU parity of detection by moves around a guess (paper §2.3 Delta-Ising
form, §3.2 MMGaP-E stages; mmgap_detect_delta) against the oracle: the same
symbols and metrics per instance under the same Philox streams, with
Metropolis or CIM-CAC anneals, one or several stages, the MMSE or a given
first guess, and at the full 16x16 64-QAM slot size on sampled instances.
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


def assert_rows_equal(gpu, ora, e_gpu, e_ora, frac=1e-4, tol=1e-5):
    gpu = np.asarray(gpu).reshape(len(gpu), -1)
    ora = np.asarray(ora).reshape(len(ora), -1)
    bad = np.where(np.any(gpu != ora, axis=1))[0]
    assert len(bad) <= int(math.floor(frac * len(gpu))), f"{len(bad)} of {len(gpu)} differ: {bad[:10]}"
    if len(bad):
        assert np.all(np.abs(np.asarray(e_gpu)[bad] - np.asarray(e_ora)[bad]) < tol)


CASES = [
    # n_r, n_t, qam, n_sc, n_sym, snr, chains, sweeps, stages, cim, init
    (8, 8, 16, 17, 3, 15.0, 32, 50, 1, None, 0),
    (8, 8, 16, 11, 4, 20.0, 64, 40, 2, None, 0),
    (8, 8, 64, 9, 3, 25.0, 32, 50, 3, None, 0),
    (16, 16, 64, 4, 3, 25.0, 32, 30, 2, None, 1),
    (4, 4, 4, 64, 1, 10.0, 16, 40, 1, None, 0),          # four instances per wavefront
    (6, 3, 16, 9, 5, 15.0, 8, 30, 2, None, 0),           # K = 6 padded to 8
    (8, 8, 16, 13, 3, 20.0, 32, 128, 2, {}, 0),          # CIM-CAC anneals
    (8, 4, 64, 7, 3, 25.0, 64, 128, 1, {"f_mvm": 1}, 1),
]


@pytest.mark.parametrize("n_r,n_t,qam,n_sc,n_sym,snr,chains,sweeps,stages,cim,init", CASES)
def test_delta_detect_matches_oracle(ctx, n_r, n_t, qam, n_sc, n_sym, snr, chains, sweeps,
                                     stages, cim, init):
    note(f"delta {n_r}x{n_t} qam={qam} {n_sc}x{n_sym} {chains}x{sweeps} stages={stages} "
         f"cim={cim} init={init}")
    d = W.det_slot(1500 + n_t + qam, n_r, n_t, qam, n_sc, n_sym, snr)
    beta2 = None if cim is not None else \
        W.linear_beta2(sweeps, *W.det_beta_range(qam, n_r, d.noise_var))
    seed = W.job_seed(11)
    sym, met = ctx.detect_delta(dev(d.H), dev(d.y), qam, d.noise_var, chains, sweeps, beta2, seed,
                                stages=stages, init=init, cim=cim)
    ref = O.detect_delta(d.H, d.y, d.noise_var, qam, chains, sweeps, beta2, seed, stages=stages,
                         init_mode=init, cim=cim)
    met = host(met).astype(np.float64)
    assert_rows_equal(host(sym), ref["sym"], met, ref["metric"])
    assert np.allclose(met, ref["metric"], rtol=1e-4, atol=1e-6)


def test_delta_from_a_given_guess(ctx):
    note("delta from a given guess")
    d = W.det_slot(1601, 8, 8, 64, 10, 3, 25.0)
    n, K = 30, 16
    rng = np.random.default_rng(4)
    guess = (2 * rng.integers(0, 8, size=(n, K)) - 7).astype(np.int8)
    beta2 = W.linear_beta2(40, *W.det_beta_range(64, 8, d.noise_var))
    seed = W.job_seed(12)
    sym, met = ctx.detect_delta(dev(d.H), dev(d.y), 64, d.noise_var, 32, 40, beta2, seed,
                                stages=2, guess=dev(guess))
    ref = O.detect_delta(d.H, d.y, d.noise_var, 64, 32, 40, beta2, seed, stages=2, guess=guess)
    met = host(met).astype(np.float64)
    assert_rows_equal(host(sym), ref["sym"], met, ref["metric"])


def test_delta_full_slot_16x16_64qam_sampled(ctx):
    """The 16x16 64-QAM slot (3276 x 12, 25 dB) by two stages of 32 chains x 50
    sweeps around the MMSE guess; the oracle recomputes a sample, and every
    instance's metric is the float64 residual of its symbols."""
    note("delta full slot 16x16 64-QAM 3276x12 32x50 2 stages")
    d = W.det_slot(3001, 16, 16, 64, 3276, 12, 25.0)
    beta2 = W.linear_beta2(50, *W.det_beta_range(64, 16, d.noise_var))
    seed = W.job_seed(3001)
    sym, met = ctx.detect_delta(dev(d.H), dev(d.y), 64, d.noise_var, 32, 50, beta2, seed,
                                stages=2)
    sym, met = host(sym), host(met).astype(np.float64)
    rng = np.random.default_rng(5)
    ids = np.unique(np.concatenate([rng.choice(3276 * 12, 48, replace=False),
                                    [0, 11, 12, 3276 * 12 - 1]])).astype(np.uint32)
    ref = O.detect_delta(d.H, d.y, d.noise_var, 64, 32, 50, beta2, seed, stages=2, inst_ids=ids)
    assert_rows_equal(sym[ids], ref["sym"], met[ids], ref["metric"])
    li, lq = W.symbol_levels(sym, 64)
    m64 = O.det_metric(d.H, d.y, np.concatenate([li, lq], axis=1), 64)
    assert np.allclose(met, m64, rtol=1e-4, atol=1e-6)
    xmm = O.slice_levels(O.mmse(d.H, d.y, d.noise_var), 64).reshape(-1, 32)
    assert np.all(m64 <= O.det_metric(d.H, d.y, xmm, 64) * (1 + 1e-5) + 1e-6)


def test_delta_arguments(ctx):
    note("delta argument errors")
    d = W.det_slot(7, 4, 4, 16, 3, 2, 20.0)
    H, y = dev(d.H), dev(d.y)
    b = np.ones(10, np.float32)
    for stages in (0, 65):
        with pytest.raises(M.MmgapError) as e:
            ctx.detect_delta(H, y, 16, d.noise_var, 32, 10, b, 1, stages=stages)
        assert e.value.code == -4
    with pytest.raises(ValueError):
        ctx.detect_delta(H, y, 16, d.noise_var, 32, 10, b, 1,
                         guess=torch.zeros((6, 7), dtype=torch.int8, device="cuda:0"))
