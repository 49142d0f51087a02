"""GPU parity of the 32x32 high-connectivity shape (paper §5.2.3: 32 receive
antennas, 32 users, up to 16-QAM, 128 anneals; K = 64 real dimensions, up to
128 spins) against the oracle: the build (couplings, fields, sliced MMSE
guess), the anneals through mmgap_solve, mmgap_detect and mmgap_detect_delta
with 64 padded dimensions, on small slots and on sampled instances of a 10 MHz
slot; and the refusals (64-QAM at this size, batches).
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


@pytest.mark.parametrize("n_r,n_t,qam,n_sc,n_sym", [(32, 32, 4, 5, 3), (32, 32, 16, 4, 2),
                                                    (40, 24, 16, 3, 4), (64, 20, 4, 2, 3)])
def test_build_32_users(ctx, n_r, n_t, qam, n_sc, n_sym):
    note(f"build det {n_r}x{n_t} qam={qam} n_sc={n_sc} n_sym={n_sym}")
    d = W.det_slot(3200 + n_t + qam, n_r, n_t, qam, n_sc, n_sym, 15.0)
    out = ctx.build_ising(M.KIND_DET, dev(d.H), dev(d.y), qam, noise_var=d.noise_var)
    G, f = O.det_ising(d.H, d.y, qam)
    assert np.array_equal(host(out["G"]), G)
    assert np.array_equal(host(out["f"]), f)
    x_fb = O.slice_levels(O.mmse(d.H, d.y, d.noise_var), qam).reshape(-1, 2 * n_t)
    assert np.array_equal(host(out["x_fb"]), x_fb)


@pytest.mark.parametrize("K,q,w,chains,sweeps,n,ipg,fb", [
    (64, 1, [1], 128, 12, 7, 3, True),
    (40, 2, [2, 1], 64, 10, 5, 1, False),     # K = 40 padded to 64
    (64, 2, [2, 1], 32, 8, 9, 9, True),
    # the workgroup's LDS copies of G: packed 4 instances per wavefront, two G per
    # workgroup, ragged last wavefront
    (64, 2, [2, 1], 16, 8, 37, 8, True),
    (64, 1, [1], 32, 10, 11, 2, False),       # packed 2 per wavefront, four G per workgroup
    (64, 2, [2, 1], 64, 8, 10, 4, True),      # one G per workgroup, last G of 2 instances
    (64, 1, [1], 192, 6, 3, 1, False),        # three wavefronts per G, across workgroups
])
def test_solve_64_dimensions(ctx, K, q, w, chains, sweeps, n, ipg, fb):
    note(f"solve K={K} q={q} chains={chains} sweeps={sweeps} n={n}")
    n_G = (n + ipg - 1) // ipg
    G, f = W.random_structured_ising(900 + K + q, n_G, ipg, K)
    f = f[:n]
    rng = np.random.default_rng(K)
    x_fb = (rng.choice([-1, 1], size=(n, K, q)) * np.array(w)).sum(-1).astype(np.int8) if fb else None
    beta2 = W.linear_beta2(sweeps, 0.05, 2.0)
    seed = W.job_seed(40 + K)
    sp, E, win = ctx.solve(dev(G), dev(f), K, q, w, chains, sweeps, beta2, seed,
                           x_fallback=None if x_fb is None else dev(x_fb), inst_per_G=ipg)
    ref = O.solve(G, f, K, q, np.array(w, np.int8), chains, sweeps, beta2, seed, x_fb=x_fb,
                  inst_per_G=ipg)
    assert np.array_equal(host(sp), ref["spins"])
    assert np.array_equal(host(E).view(np.uint32), ref["E"].view(np.uint32))
    assert np.array_equal(host(win), ref["win"])


@pytest.mark.parametrize("n_r,n_t,qam,n_sc,n_sym,chains,sweeps,init", [
    (32, 32, 4, 3, 4, 128, 16, 0),
    (32, 32, 16, 2, 3, 64, 12, 1),
    (40, 24, 16, 2, 5, 32, 14, 0),
])
def test_detect_32_users(ctx, n_r, n_t, qam, n_sc, n_sym, chains, sweeps, init):
    note(f"detect {n_r}x{n_t} qam={qam} {n_sc}x{n_sym} {chains}x{sweeps} init={init}")
    d = W.det_slot(3300 + n_t + qam, n_r, n_t, qam, n_sc, n_sym, 15.0)
    beta2 = W.linear_beta2(sweeps, *W.det_beta_range(qam, n_r, d.noise_var))
    seed = W.job_seed(41)
    sym, met = ctx.detect(dev(d.H), dev(d.y), qam, d.noise_var, chains, sweeps, beta2, seed,
                          init=init)
    ref = O.detect(d.H, d.y, d.noise_var, qam, chains, sweeps, beta2, seed, init_mode=init)
    met = host(met).astype(np.float64)
    assert_rows_equal(host(sym), ref["sym"], met, ref["metric"])
    assert np.allclose(met, ref["metric"], rtol=1e-4, atol=1e-6)


def test_delta_32_users(ctx):
    note("delta 32x32 16-QAM 3x3 32x10 2 stages")
    d = W.det_slot(3401, 32, 32, 16, 3, 3, 20.0)
    beta2 = W.linear_beta2(10, *W.det_beta_range(16, 32, d.noise_var))
    seed = W.job_seed(42)
    sym, met = ctx.detect_delta(dev(d.H), dev(d.y), 16, d.noise_var, 32, 10, beta2, seed, stages=2)
    ref = O.detect_delta(d.H, d.y, d.noise_var, 16, 32, 10, beta2, seed, stages=2)
    met = host(met).astype(np.float64)
    assert_rows_equal(host(sym), ref["sym"], met, ref["metric"])
    assert np.allclose(met, ref["metric"], rtol=1e-4, atol=1e-6)


def test_full_slot_32x32_16qam_sampled(ctx):
    """A 10 MHz slot (288 subcarriers x 12 symbols) of 32x32 16-QAM at 15 dB with
    128 anneals of 100 sweeps, the launch the benchmark times; the oracle
    recomputes a sample and every metric is the float64 residual of its
    symbols, never above the MMSE guess's."""
    note("full slot 32x32 16-QAM 288x12 128x100")
    d = W.det_slot(3501, 32, 32, 16, 288, 12, 15.0)
    beta2 = W.linear_beta2(100, *W.det_beta_range(16, 32, d.noise_var))
    seed = W.job_seed(3501)
    sym, met = ctx.detect(dev(d.H), dev(d.y), 16, d.noise_var, 128, 100, beta2, seed)
    sym, met = host(sym), host(met).astype(np.float64)
    rng = np.random.default_rng(14)
    ids = np.unique(np.concatenate([rng.choice(288 * 12, 10, replace=False),
                                    [0, 288 * 12 - 1]])).astype(np.uint32)
    ref = O.detect(d.H, d.y, d.noise_var, 16, 128, 100, beta2, seed, inst_ids=ids)
    assert_rows_equal(sym[ids], ref["sym"], met[ids], ref["metric"])
    li, lq = W.symbol_levels(sym, 16)
    m64 = O.det_metric(d.H, d.y, np.concatenate([li, lq], axis=1), 16)
    assert np.allclose(met, m64, rtol=1e-4, atol=1e-6)
    xmm = O.slice_levels(O.mmse(d.H, d.y, d.noise_var), 16).reshape(-1, 64)
    assert np.all(m64 <= O.det_metric(d.H, d.y, xmm, 16) * (1 + 1e-5) + 1e-6)


def test_32_users_refusals(ctx):
    note("32 users: refusals")
    d = W.det_slot(3601, 32, 32, 64, 2, 2, 20.0)
    b = np.ones(4, np.float32)
    with pytest.raises(M.MmgapError) as e:                 # 64-QAM: 192 spins
        ctx.detect(dev(d.H), dev(d.y), 64, d.noise_var, 32, 4, b, 1)
    assert e.value.code == -4
    d = W.det_slot(3602, 32, 32, 16, 2, 2, 20.0)
    job = ctx.det_job(dev(d.H), dev(d.y), 16, d.noise_var, 32, 4, b, 1, stages=1)
    with pytest.raises(M.MmgapError) as e:                 # stages in a batch: up to 32 dims
        ctx.plan_create([job])
    assert e.value.code == -4
    with pytest.raises(M.MmgapError) as e:                 # MMSE-SIC up to 16 users
        ctx.detect_sic(dev(d.H), dev(d.y), 16, d.noise_var)
    assert e.value.code == -4
