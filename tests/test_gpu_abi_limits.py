"""The size limits documented in include/mmgap.h, through the C ABI: every call
at a limit succeeds (MMGAP_OK) and the same call one step past it is refused
with MMGAP_EUNSUPPORTED before anything is enqueued.  Problems are one
subcarrier and one symbol with short schedules, so each call is tiny."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workload import synth as W

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # collected on CPU hosts only with -m gpu
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2510_01579_amd as M

EUNSUPPORTED = -4


def note(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = M.Context(0)
    yield c
    c.close()


def det_inputs(n_r, n_t, n_sym=1, seed=1):
    rng = np.random.default_rng(seed)
    H = (rng.standard_normal((1, n_r, n_t)) + 1j * rng.standard_normal((1, n_r, n_t))) / 2 ** 0.5
    y = (rng.standard_normal((1, n_sym, n_r)) + 1j * rng.standard_normal((1, n_sym, n_r)))
    return (torch.from_numpy(H.astype(np.complex64)).to("cuda:0"),
            torch.from_numpy(y.astype(np.complex64)).to("cuda:0"))


def ok_then_refused(ok, refused):
    ok()
    torch.cuda.synchronize()
    with pytest.raises(M.MmgapError) as e:
        refused()
    assert e.value.code == EUNSUPPORTED, str(e.value)


def b2(n):
    return W.linear_beta2(n, 0.1, 2.0)


@pytest.mark.parametrize("qam", [4, 16])
def test_det_users(ctx, qam):
    note(f"DET 32 users ({qam}-QAM) ok, 33 refused")
    ok_then_refused(lambda: ctx.detect(*det_inputs(32, 32), qam, 1.0, 4, 2, b2(2), 1),
                    lambda: ctx.detect(*det_inputs(33, 33), qam, 1.0, 4, 2, b2(2), 1))


def test_det_users_64qam(ctx):
    note("DET 16 users at 64-QAM ok, 17 refused")
    ok_then_refused(lambda: ctx.detect(*det_inputs(16, 16), 64, 1.0, 4, 2, b2(2), 1),
                    lambda: ctx.detect(*det_inputs(17, 17), 64, 1.0, 4, 2, b2(2), 1))


def test_det_receive_antennas(ctx):
    note("DET 64 receive antennas ok, 65 refused")
    ok_then_refused(lambda: ctx.detect(*det_inputs(64, 8), 16, 1.0, 4, 2, b2(2), 1),
                    lambda: ctx.detect(*det_inputs(65, 8), 16, 1.0, 4, 2, b2(2), 1))


def test_vpp_sizes(ctx):
    note("VPP 16 users x 64 antennas ok; 17 users, 65 antennas refused")
    ok_then_refused(lambda: ctx.vpp_precode(*det_inputs(16, 64), 16, 4, 2, b2(2), 1),
                    lambda: ctx.vpp_precode(*det_inputs(17, 64), 16, 4, 2, b2(2), 1))
    ok_then_refused(lambda: ctx.vpp_precode(*det_inputs(8, 64), 16, 4, 2, b2(2), 1),
                    lambda: ctx.vpp_precode(*det_inputs(8, 65), 16, 4, 2, b2(2), 1))


def test_symbols_per_subcarrier(ctx):
    note("n_sym 64 ok, 65 refused")
    ok_then_refused(lambda: ctx.detect(*det_inputs(4, 4, n_sym=64), 4, 1.0, 4, 2, b2(2), 1),
                    lambda: ctx.detect(*det_inputs(4, 4, n_sym=65), 4, 1.0, 4, 2, b2(2), 1))


def test_chains_and_sweeps(ctx):
    note("chains 1024 ok / 1025 refused; sweeps 8192 ok / 8193 refused")
    ok_then_refused(lambda: ctx.detect(*det_inputs(4, 4), 4, 1.0, 1024, 2, b2(2), 1),
                    lambda: ctx.detect(*det_inputs(4, 4), 4, 1.0, 1025, 2, b2(2), 1))
    ok_then_refused(lambda: ctx.detect(*det_inputs(2, 1), 4, 1.0, 1, 8192, b2(8192), 1),
                    lambda: ctx.detect(*det_inputs(2, 1), 4, 1.0, 1, 8193, b2(8193), 1))


def solve_call(ctx, K, q, w):
    G, f = W.random_structured_ising(9, 1, 1, K)
    dev = "cuda:0"
    return ctx.solve(torch.from_numpy(G).to(dev), torch.from_numpy(f).to(dev), K, q, w, 4, 2,
                     b2(2), 1)


def test_solve_structure(ctx):
    note("solve K=64 q=2 ok / q=3 refused; K=32 q=4 ok / q=5 refused; K=65 refused")
    ok_then_refused(lambda: solve_call(ctx, 64, 2, [2, 1]),
                    lambda: solve_call(ctx, 64, 3, [4, 2, 1]))
    ok_then_refused(lambda: solve_call(ctx, 32, 4, [8, 4, 2, 1]),
                    lambda: solve_call(ctx, 32, 5, [16, 8, 4, 2, 1]))
    ok_then_refused(lambda: solve_call(ctx, 64, 1, [1]),
                    lambda: solve_call(ctx, 65, 1, [1]))


def test_sic_and_mmgap_e_users(ctx):
    note("MMSE-SIC and MMGaP-E 16 users ok, 17 refused")
    ok_then_refused(lambda: ctx.detect_sic(*det_inputs(16, 16), 16, 1.0),
                    lambda: ctx.detect_sic(*det_inputs(17, 17), 16, 1.0))
    ok_then_refused(lambda: ctx.detect_e(*det_inputs(16, 16), 16, 1.0, 4, 2, b2(2), 1),
                    lambda: ctx.detect_e(*det_inputs(17, 17), 16, 1.0, 4, 2, b2(2), 1))


def test_stages(ctx):
    note("detection around a guess: 64 stages ok, 65 refused")
    ok_then_refused(lambda: ctx.detect_delta(*det_inputs(4, 4), 16, 1.0, 4, 1, b2(1), 1,
                                             stages=64),
                    lambda: ctx.detect_delta(*det_inputs(4, 4), 16, 1.0, 4, 1, b2(1), 1,
                                             stages=65))


def test_cim_spins(ctx):
    note("CIM-CAC 64 spins (16x16 16-QAM) ok, 96 (16x16 64-QAM) refused")
    ok_then_refused(lambda: ctx.detect(*det_inputs(16, 16), 16, 1.0, 4, 4, None, 1, cim={}),
                    lambda: ctx.detect(*det_inputs(16, 16), 64, 1.0, 4, 4, None, 1, cim={}))


def test_batch_limits(ctx):
    note("batches: binary 32 users ok / 33 refused; stages 16 users ok / 17 refused; "
         "256 chains ok / 257 refused")

    def plan(n_t, chains, stages=0):
        H, y = det_inputs(n_t, n_t)
        j = ctx.det_job(H, y, 4, 1.0, chains, 2, b2(2), 1, stages=stages)
        p = ctx.plan_create([j], graph=False)
        p.plan_launch()
        torch.cuda.synchronize()
        p.plan_destroy()

    ok_then_refused(lambda: plan(32, 4), lambda: plan(33, 4))          # plain route above 16
    ok_then_refused(lambda: plan(16, 4, 1), lambda: plan(17, 4, 1))    # moves: 32 dimensions
    ok_then_refused(lambda: plan(8, 256), lambda: plan(8, 257))
