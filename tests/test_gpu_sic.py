"""GPU parity of the ordered MMSE-SIC detector (paper §1/§4 baseline; reading of
the unstated ordering rule: smallest MMSE error variance first) and of MMGaP-E
(§3.2 Fig. 6: stages from the MMSE and from the MMSE-SIC guess, the better
answer) against the oracle: the same detection order, levels and symbols, and
metrics within float rounding; full 16x16 64-QAM slots on sampled instances.
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


def assert_rows_equal(gpu, ora, margin=None, frac=1e-4, tiny=1e-9):
    """Equal rows but for a fraction `frac`, and those only where a slicing
    decision of the oracle lay within `tiny` of its boundary (float64 sums in
    another order may then decide the other way)."""
    gpu = np.asarray(gpu).reshape(len(gpu), -1)
    ora = np.asarray(ora).reshape(len(ora), -1)
    bad = np.where(np.any(gpu != ora, axis=1))[0]
    assert len(bad) <= int(math.floor(frac * len(gpu))), f"{len(bad)} of {len(gpu)} differ: {bad[:10]}"
    if len(bad):
        assert margin is not None and np.all(np.asarray(margin)[bad] < tiny), bad[:10]


SIC_CASES = [
    # n_r, n_t, qam, n_sc, n_sym, snr
    (4, 4, 4, 64, 1, 10.0),
    (8, 8, 16, 37, 5, 15.0),
    (8, 4, 64, 21, 37, 25.0),      # three passes of 16 symbols, ragged tail
    (16, 16, 64, 9, 12, 25.0),
    (6, 3, 16, 15, 7, 12.0),
    (4, 1, 16, 11, 3, 10.0),       # one user
    (64, 16, 16, 5, 4, 5.0),       # 64 receive antennas
]


@pytest.mark.parametrize("n_r,n_t,qam,n_sc,n_sym,snr", SIC_CASES)
def test_sic_matches_oracle(ctx, n_r, n_t, qam, n_sc, n_sym, snr):
    note(f"sic {n_r}x{n_t} qam={qam} {n_sc}x{n_sym} snr={snr}")
    d = W.det_slot(2100 + n_r + n_t + qam, n_r, n_t, qam, n_sc, n_sym, snr)
    sym, met, lv, od = ctx.detect_sic(dev(d.H), dev(d.y), qam, d.noise_var, levels=True,
                                      order=True)
    ref = O.mmse_sic(d.H, d.y, d.noise_var, qam)
    assert np.array_equal(host(od), ref["order"])
    assert_rows_equal(host(lv), ref["levels"], ref["margin"])
    assert_rows_equal(host(sym), ref["sym"], ref["margin"])
    assert np.allclose(host(met).astype(np.float64), ref["metric"], rtol=1e-4, atol=1e-6)


def test_sic_full_slot_16x16_64qam_sampled(ctx):
    note("sic full slot 16x16 64-QAM 3276x12")
    d = W.det_slot(3001, 16, 16, 64, 3276, 12, 25.0)
    sym, met, lv, _ = ctx.detect_sic(dev(d.H), dev(d.y), 64, d.noise_var, levels=True)
    sym, met, lv = host(sym), host(met).astype(np.float64), host(lv)
    rng = np.random.default_rng(12)
    ids = np.unique(np.concatenate([rng.choice(3276 * 12, 300, replace=False),
                                    [0, 11, 12, 3276 * 12 - 1]])).astype(np.uint32)
    ref = O.mmse_sic(d.H, d.y, d.noise_var, 64, inst_ids=ids)
    assert_rows_equal(lv[ids], ref["levels"], ref["margin"], frac=0.01)
    assert np.array_equal(O.levels_to_symbols(lv, 64), sym)
    assert np.allclose(met, O.det_metric(d.H, d.y, lv, 64), rtol=1e-4, atol=1e-6)
    truth = d.sym.reshape(-1, 16)
    mmse = O.levels_to_symbols(O.slice_levels(O.mmse(d.H, d.y, d.noise_var), 64).reshape(-1, 32), 64)
    assert np.mean(sym != truth) < np.mean(mmse != truth)


E_CASES = [
    # n_r, n_t, qam, n_sc, n_sym, snr, chains, sweeps, stages
    (8, 8, 16, 11, 4, 18.0, 32, 30, 1),
    (8, 8, 64, 7, 3, 25.0, 16, 25, 2),
    (16, 16, 64, 3, 4, 25.0, 32, 20, 2),
    (6, 3, 16, 9, 5, 15.0, 64, 20, 1),
]


@pytest.mark.parametrize("n_r,n_t,qam,n_sc,n_sym,snr,chains,sweeps,stages", E_CASES)
def test_mmgap_e_matches_oracle(ctx, n_r, n_t, qam, n_sc, n_sym, snr, chains, sweeps, stages):
    note(f"mmgap-e {n_r}x{n_t} qam={qam} {n_sc}x{n_sym} {chains}x{sweeps} stages={stages}")
    d = W.det_slot(2200 + n_t + qam, n_r, n_t, qam, n_sc, n_sym, snr)
    beta2 = W.linear_beta2(sweeps, *W.det_beta_range(qam, n_r, d.noise_var))
    seed = W.job_seed(21)
    sym, met, fs = ctx.detect_e(dev(d.H), dev(d.y), qam, d.noise_var, chains, sweeps, beta2,
                                seed, stages=stages)
    ref = O.detect_e(d.H, d.y, d.noise_var, qam, chains, sweeps, beta2, seed, stages=stages)
    assert_rows_equal(host(sym), ref["sym"], ref["sic_margin"])
    fs = host(fs).astype(bool)
    bad = np.where(fs != ref["from_sic"])[0]
    assert np.all(ref["sic_margin"][bad] < 1e-9), bad
    assert np.allclose(host(met).astype(np.float64), ref["metric"], rtol=1e-4, atol=1e-6)


@pytest.mark.parametrize("guesses", [1, 2])
def test_mmgap_e_single_chain_matches_oracle(ctx, guesses):
    note(f"mmgap-e guesses={guesses} 8x8 64-QAM 9x4 16x20 2 stages")
    d = W.det_slot(2300 + guesses, 8, 8, 64, 9, 4, 25.0)
    beta2 = W.linear_beta2(20, *W.det_beta_range(64, 8, d.noise_var))
    seed = W.job_seed(22)
    sym, met, fs = ctx.detect_e(dev(d.H), dev(d.y), 64, d.noise_var, 16, 20, beta2, seed,
                                stages=2, guesses=guesses)
    ref = O.detect_e(d.H, d.y, d.noise_var, 64, 16, 20, beta2, seed, stages=2, guesses=guesses)
    assert_rows_equal(host(sym), ref["sym"], ref["sic_margin"])
    assert np.all(host(fs) == (1 if guesses == 2 else 0))
    assert np.allclose(host(met).astype(np.float64), ref["metric"], rtol=1e-4, atol=1e-6)


def test_mmgap_e_full_slot_16x16_64qam_sampled(ctx):
    note("mmgap-e full slot 16x16 64-QAM 3276x12 16x12 1 stage")
    d = W.det_slot(3001, 16, 16, 64, 3276, 12, 25.0)
    beta2 = W.linear_beta2(12, *W.det_beta_range(64, 16, d.noise_var))
    seed = W.job_seed(3001)
    sym, met, fs = ctx.detect_e(dev(d.H), dev(d.y), 64, d.noise_var, 16, 12, beta2, seed,
                                stages=1)
    sym, met, fs = host(sym), host(met).astype(np.float64), host(fs)
    rng = np.random.default_rng(13)
    ids = np.unique(np.concatenate([rng.choice(3276 * 12, 40, replace=False),
                                    [0, 3276 * 12 - 1]])).astype(np.uint32)
    ref = O.detect_e(d.H, d.y, d.noise_var, 64, 16, 12, beta2, seed, stages=1, inst_ids=ids)
    assert_rows_equal(sym[ids], ref["sym"], ref["sic_margin"], frac=0.03)
    li, lq = W.symbol_levels(sym, 64)
    assert np.allclose(met, O.det_metric(d.H, d.y, np.concatenate([li, lq], axis=1), 64),
                       rtol=1e-4, atol=1e-6)
    # never worse than the single-guess search from the MMSE estimate
    s1, m1 = ctx.detect_delta(dev(d.H), dev(d.y), 64, d.noise_var, 16, 12, beta2, seed, stages=1)
    assert np.all(met <= host(m1).astype(np.float64) * (1 + 1e-4) + 1e-6)


def test_sic_arguments(ctx):
    note("sic argument errors")
    d = W.det_slot(8, 4, 4, 16, 3, 2, 20.0)
    H, y = dev(d.H), dev(d.y)
    p = ctx._problem(M.KIND_DET, H, y, 16, d.noise_var, 0.0)
    met = torch.empty(6, dtype=torch.float32, device="cuda:0")
    rc = M.lib().mmgap_detect_sic(ctx._h, __import__("ctypes").byref(p), M._ptr(H), M._ptr(y),
                                  None, M._ptr(met), None, None, M._stream(ctx._dev()))
    assert rc == -1
    with pytest.raises(M.MmgapError) as e:
        ctx.detect_e(H, y, 16, d.noise_var, 32, 10, np.ones(10, np.float32), 1, stages=0)
    assert e.value.code == -4
    for g in (0, 4):
        with pytest.raises(M.MmgapError) as e:
            ctx.detect_e(H, y, 16, d.noise_var, 32, 10, np.ones(10, np.float32), 1, guesses=g)
        assert e.value.code == -1


def test_empty_and_largest_inputs(ctx):
    """Empty slots return without writing; the largest symbol count (64 per
    subcarrier: four detection passes of 16 lanes at 16 receive antennas) and
    one symbol per subcarrier match the oracle."""
    note("sic / mmgap-e / delta: empty and largest inputs")
    H0 = torch.empty((0, 8, 8), dtype=torch.complex64, device="cuda:0")
    y0 = torch.empty((0, 3, 8), dtype=torch.complex64, device="cuda:0")
    sym, met, lv, od = ctx.detect_sic(H0, y0, 16, 0.1, levels=True, order=True)
    assert sym.shape == (0, 8) and lv.shape == (0, 16)
    b = np.ones(4, np.float32)
    sym, met, fs = ctx.detect_e(H0, y0, 16, 0.1, 8, 4, b, 1)
    assert sym.shape == (0, 8)
    sym, met = ctx.detect_delta(H0, y0, 16, 0.1, 8, 4, b, 1)
    assert sym.shape == (0, 8)
    for n_sym in (64, 1):
        d = W.det_slot(2400 + n_sym, 16, 12, 16, 3, n_sym, 20.0)
        sym, met, lv, od = ctx.detect_sic(dev(d.H), dev(d.y), 16, d.noise_var, levels=True,
                                          order=True)
        ref = O.mmse_sic(d.H, d.y, d.noise_var, 16)
        assert np.array_equal(host(od), ref["order"])
        assert_rows_equal(host(lv), ref["levels"], ref["margin"])
        assert np.allclose(host(met).astype(np.float64), ref["metric"], rtol=1e-4, atol=1e-6)
