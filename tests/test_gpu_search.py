"""The one-launch search (every stage of moves around a guess, both chains of
MMGaP-E, the choice and the decode in one kernel; paper §2.3 Fig. 5, §3.2
Fig. 6) against the stage launches (move fields, anneal, selection, choice as
separate kernels): identical symbols, metrics and choices, over the padded
dimension counts 8/16/32, 1 to 64 chains (4 to 64 lanes per instance),
ragged wavefronts and workgroups, 1 to 4 stages, both initial states, the
MMSE, caller and MMSE-SIC guesses and receive antennas up to twice the lanes;
and a full 16x16 64-QAM slot at MMGaP-E 16 x 4 x 3 (the benchmark's 20 dB
schedule) against the oracle on sampled instances.
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


def both_paths(ctx, fn):
    """fn() with the one-launch search (the default), then with the stage launches."""
    a = [host(t) for t in fn()]
    ctx.set_stage_launches(True)
    try:
        b = [host(t) for t in fn()]
    finally:
        ctx.set_stage_launches(False)
    return a, b


def assert_same(a, b):
    for x, y in zip(a, b):
        if x is None:
            assert y is None
            continue
        assert x.dtype == y.dtype and x.shape == y.shape
        if x.dtype == np.float32:       # bit patterns, NaN and -0 included
            assert np.array_equal(x.view(np.uint32), y.view(np.uint32))
        else:
            assert np.array_equal(x, y)


CASES = [
    # n_r, n_t, qam, n_sc, n_sym, snr, chains, sweeps, stages, init
    (4, 4, 4, 37, 16, 8.0, 4, 6, 2, 0),       # KT 8, 4 lanes, 16 instances per wavefront
    (6, 3, 16, 29, 5, 14.0, 8, 5, 3, 1),      # K 6 < KT 8, 5 symbols: 64 lanes
    (8, 8, 16, 23, 12, 15.0, 16, 4, 3, 0),    # KT 16, 4 instances per wavefront
    (8, 8, 64, 19, 12, 25.0, 1, 3, 1, 1),     # one chain
    (12, 6, 64, 17, 7, 22.0, 32, 4, 2, 0),    # K 12 < KT 16, 32 lanes
    (16, 16, 64, 21, 12, 20.0, 16, 4, 3, 0),  # the benchmark's shape
    (16, 16, 64, 13, 12, 30.0, 48, 3, 1, 1),  # 48 chains: one instance per wavefront
    (16, 16, 16, 11, 12, 15.0, 64, 2, 4, 0),  # 64 chains, four stages
    (16, 12, 16, 9, 4, 18.0, 8, 5, 2, 1),     # K 24 < KT 32
    (16, 8, 16, 7, 8, 16.0, 8, 6, 2, 0),      # 8 lanes and 16 receive antennas (2 per lane)
    (32, 8, 16, 5, 8, 16.0, 8, 4, 1, 0),      # 32 antennas > 2 lanes: the stage launches run
]


@pytest.mark.parametrize("n_r,n_t,qam,n_sc,n_sym,snr,chains,sweeps,stages,init", CASES)
def test_search_equals_stage_launches(ctx, n_r, n_t, qam, n_sc, n_sym, snr, chains, sweeps,
                                      stages, init):
    d = W.det_slot(5100 + n_r + n_t + qam + chains, n_r, n_t, qam, n_sc, n_sym, snr)
    H, y = dev(d.H), dev(d.y)
    beta2 = W.linear_beta2(sweeps, *W.det_beta_range(qam, n_r, d.noise_var))
    seed = W.job_seed(51 + chains)
    note(f"search {n_r}x{n_t} qam={qam} {n_sc}x{n_sym} {chains}x{sweeps}x{stages} init={init}")
    for guesses in (3, 1, 2):
        a, b = both_paths(ctx, lambda: ctx.detect_e(H, y, qam, d.noise_var, chains, sweeps,
                                                    beta2, seed, stages=stages, init=init,
                                                    guesses=guesses))
        assert_same(a, b)
    a, b = both_paths(ctx, lambda: ctx.detect_delta(H, y, qam, d.noise_var, chains, sweeps,
                                                    beta2, seed, stages=stages, init=init))
    assert_same(a, b)
    # a caller's guess: the sliced MMSE estimate moved by one level where allowed
    rng = np.random.default_rng(n_sc)
    g = O.slice_levels(O.mmse(d.H, d.y, d.noise_var), qam).reshape(-1, 2 * n_t)
    top = int(np.sqrt(qam)) - 1
    g = np.clip(g + 2 * rng.integers(-1, 2, g.shape), -top, top).astype(np.int8)
    g = np.where(g % 2 == 0, g + 1, g).astype(np.int8)
    gd = dev(g)
    a, b = both_paths(ctx, lambda: ctx.detect_delta(H, y, qam, d.noise_var, chains, sweeps,
                                                    beta2, seed, stages=stages, init=init,
                                                    guess=gd))
    assert_same(a, b)


def test_search_without_metric_and_with_offset(ctx):
    """No metric output, and a Philox instance offset (a subcarrier shard)."""
    note("search 8x8 16-QAM 15x12: no metric, inst_base 120")
    d = W.det_slot(5201, 8, 8, 16, 15, 12, 15.0)
    H, y = dev(d.H), dev(d.y)
    beta2 = W.linear_beta2(4, *W.det_beta_range(16, 8, d.noise_var))
    a, b = both_paths(ctx, lambda: ctx.detect_e(H, y, 16, d.noise_var, 16, 4, beta2, 77,
                                                stages=2, metric=False, inst_base=120))
    assert a[1] is None and b[1] is None
    assert_same(a, b)


def test_search_full_slot_16x16_64qam_e_sampled(ctx):
    """The benchmark's 20 dB slot at its schedule (MMGaP-E 16 x 4 x 3): equal to
    the stage launches everywhere, and to the oracle on sampled instances."""
    note("search full slot 16x16 64-QAM 3276x12 20 dB MMGaP-E 16x4x3")
    d = W.det_slot(3002, 16, 16, 64, 3276, 12, 20.0)
    beta2 = W.linear_beta2(4, *W.det_beta_range(64, 16, d.noise_var))
    seed = W.job_seed(3002)
    H, y = dev(d.H), dev(d.y)
    a, b = both_paths(ctx, lambda: ctx.detect_e(H, y, 64, d.noise_var, 16, 4, beta2, seed,
                                                stages=3))
    assert_same(a, b)
    sym, met, fs = a
    rng = np.random.default_rng(14)
    ids = np.unique(np.concatenate([rng.choice(3276 * 12, 40, replace=False),
                                    [0, 3276 * 12 - 1]])).astype(np.uint32)
    ref = O.detect_e(d.H, d.y, d.noise_var, 64, 16, 4, beta2, seed, stages=3, inst_ids=ids)
    bad = np.where(np.any(sym[ids] != ref["sym"], axis=1))[0]
    assert len(bad) <= 1 and np.all(ref["sic_margin"][bad] < 1e-9), bad
    assert np.allclose(met[ids].astype(np.float64), ref["metric"], rtol=1e-4, atol=1e-6)


def test_stage_option_arguments(ctx):
    note("set_option argument errors")
    for opt, val in ((M.OPT_STAGE_LAUNCHES, 2), (99, 0)):
        assert M.lib().mmgap_set_option(ctx._h, opt, val) == -1


def test_search_non_finite_inputs_equal_stage_launches(ctx):
    """The search launch takes the zero move's energy as +0 without summing it,
    and as NaN when a coupling or a doubled move field is not finite; the stage
    launches sum it.  Subcarrier 1 gets an infinite channel entry (non-finite
    couplings) and one symbol of subcarrier 2 a received sample of 3e38 (its
    fields overflow): both paths must still agree everywhere, the finite
    subcarriers bit for bit and the poisoned ones with NaN where the other has
    NaN."""
    note("search 8x8 16-QAM 5x12 with non-finite channel and fields")
    d = W.det_slot(5301, 8, 8, 16, 5, 12, 15.0)
    Hn = d.H.copy()
    yn = d.y.copy()
    Hn[1, 0, 0] = np.complex64(np.inf)
    yn[2, 3, :] = np.complex64(3e38)
    H, y = dev(Hn), dev(yn)
    beta2 = W.linear_beta2(4, *W.det_beta_range(16, 8, d.noise_var))

    def same_nan(a, b):
        for x, z in zip(a, b):
            if x is None:
                assert z is None
                continue
            assert x.dtype == z.dtype and x.shape == z.shape
            if x.dtype == np.float32:
                nx, nz = np.isnan(x), np.isnan(z)
                assert np.array_equal(nx, nz)
                assert np.array_equal(x[~nx].view(np.uint32), z[~nz].view(np.uint32))
            else:
                assert np.array_equal(x, z)

    for guesses in (3, 1):
        a, b = both_paths(ctx, lambda: ctx.detect_e(H, y, 16, d.noise_var, 16, 4, beta2, 91,
                                                    stages=2, guesses=guesses))
        same_nan(a, b)
    a, b = both_paths(ctx, lambda: ctx.detect_delta(H, y, 16, d.noise_var, 16, 4, beta2, 91,
                                                    stages=2))
    same_nan(a, b)
    # the finite subcarriers are unaffected by the poisoned ones
    clean = ctx.detect_delta(dev(d.H), dev(d.y), 16, d.noise_var, 16, 4, beta2, 91, stages=2)
    sym_c, sym_p = host(clean[0]), a[0]
    rows = np.r_[0:12, 36:60]      # subcarriers 0, 3 and 4
    assert np.array_equal(sym_c[rows], sym_p[rows])
