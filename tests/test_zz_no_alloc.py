"""The allocation-free detection entry point (mmgap_detect_noalloc) against
mmgap_detect, through the C ABI: same symbols and metrics on two calls in a
row (the second smaller, so the fixed scratch holds the first call's data when
it starts), a call at the full 3276 x 12 slot, and the size limit."""
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


def run_both(ctx, d, qam, chains, sweeps, init, seed):
    n_r, n_t = d.H.shape[1], d.H.shape[2]
    beta2 = W.linear_beta2(sweeps, *W.det_beta_range(qam, n_r, d.noise_var))
    H, y = dev(d.H), dev(d.y)
    n = d.y.shape[0] * d.y.shape[1]
    sym = torch.empty((n, n_t), dtype=torch.uint8, device="cuda:0")
    met = torch.empty((n,), dtype=torch.float32, device="cuda:0")
    ctx.detect_noalloc(H, y, qam, d.noise_var, chains, sweeps, beta2, seed, init=init,
                       sym=sym, metric=met)
    rs, rm = ctx.detect(H, y, qam, d.noise_var, chains, sweeps, beta2, seed, init=init)
    torch.cuda.synchronize()
    return sym.cpu().numpy(), met.cpu().numpy(), rs.cpu().numpy(), rm.cpu().numpy(), beta2


@pytest.mark.parametrize("first,second", [
    # (n_r, n_t, qam, n_sc, n_sym, snr, chains, sweeps, init)
    ((8, 8, 16, 300, 12, 15.0, 64, 40, 0), (8, 8, 16, 37, 3, 15.0, 64, 40, 1)),
    ((16, 16, 64, 96, 12, 25.0, 128, 12, 1), (4, 4, 4, 64, 1, 10.0, 32, 100, 0)),
])
def test_noalloc_equals_detect_on_two_calls(ctx, first, second):
    for k, (n_r, n_t, qam, n_sc, n_sym, snr, C, S, init) in enumerate((first, second)):
        note(f"noalloc call {k}: {n_r}x{n_t} {qam}-QAM {n_sc}x{n_sym} C={C} S={S} init={init}")
        d = W.det_slot(8100 + k, n_r, n_t, qam, n_sc, n_sym, snr)
        seed = W.job_seed(8100 + k)
        s0, m0, s1, m1, beta2 = run_both(ctx, d, qam, C, S, init, seed)
        assert np.array_equal(s0, s1), "symbols differ from mmgap_detect"
        assert m0.tobytes() == m1.tobytes(), "metrics differ from mmgap_detect"
        if k == 1:       # the small call also against the oracle, instance by instance
            ref = O.detect(d.H, d.y, d.noise_var, qam, C, S, beta2, seed, init_mode=init)
            assert np.array_equal(s0, ref["sym"])
            assert np.allclose(m0.astype(np.float64), ref["metric"], rtol=1e-4, atol=1e-6)


def test_noalloc_full_slot(ctx):
    note("noalloc full 8x8 16-QAM slot 3276x12, 64 x 20")
    d = W.det_slot(8200, 8, 8, 16, 3276, 12, 15.0)
    s0, m0, s1, m1, _ = run_both(ctx, d, 16, 64, 20, 1, W.job_seed(8200))
    assert np.array_equal(s0, s1)
    assert m0.tobytes() == m1.tobytes()


def test_noalloc_size_limit(ctx):
    note("noalloc above its fixed scratch: refused on the host")
    d = W.det_slot(8300, 16, 16, 64, 3276, 12, 25.0)
    H, y = dev(d.H), dev(d.y)
    beta2 = W.linear_beta2(4, *W.det_beta_range(64, 16, d.noise_var))
    # 3276 x 12 instances x 256 chains x 16 bytes of chain state > 128 MiB
    with pytest.raises(RuntimeError, match="fixed"):
        ctx.detect_noalloc(H, y, 64, d.noise_var, 256, 4, beta2, W.job_seed(8300), init=1)
    # the context stays usable
    s0, _ = ctx.detect_noalloc(H[:8].contiguous(), y[:8].contiguous(), 64, d.noise_var, 32, 4,
                               beta2, W.job_seed(8300), init=1)
    s1, _ = ctx.detect(H[:8].contiguous(), y[:8].contiguous(), 64, d.noise_var, 32, 4, beta2,
                       W.job_seed(8300), init=1)
    torch.cuda.synchronize()
    assert np.array_equal(s0.cpu().numpy(), s1.cpu().numpy())
