"""Pins the oracle's chain contract against plain Metropolis at workload scale.

The oracle's chains (and the GPU's, bit for bit) accept an uphill flip iff the
16-bit draw m is below T[floor(64 z)], T[j] = round(2^16 2^(-j/64)), with
z = beta2_t dE computed in float32 and the field of a dimension recomputed as a
float32 fma row at each visit.  That is Metropolis acceptance 2^-z with z
floored to 1/64 (probability at most 1.1% above 2^-z, plus 2^-16 of rounding).
The paper's processing flow (§3.2: the anneals' final states are the
candidates, ranked by the ML energy of Eq. ml) does not depend on that choice
at the level of solution quality; these tests check it against a plain
Metropolis reference -- the same anneals from the same draws, computed from the
definitions in float64, accepting iff (m + 1/2)/2^16 < 2^-z exactly -- on
2016 sampled instances of three detection slots:

  * 8x8 16-QAM, 15 dB, 64 chains x 200 sweeps, random start;
  * 8x8 16-QAM, 15 dB, 64 chains x 50 sweeps, fallback start;
  * 16x16 64-QAM, 25 dB, 128 chains x 400 sweeps, fallback start.

For each slot the symbol error rate and the mean final residual ||y - Hx||^2
(the energy up to the constant ||y||^2) of the two must agree within three
standard errors of their paired per-instance differences (the two chains share
instances and draws, so the paired error is the relevant one; the unpaired
error is larger still).  The per-instance results are stored in
tests/golden/acceptance_quality.json by tests/golden/make_acceptance_quality.py,
which calls only the oracle; here the two 8x8 slots are recomputed in full and
the 16x16 slot on a sample of its instances, and must reproduce the stored
values exactly.
"""
import importlib.util
import json
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


def _maker():
    spec = importlib.util.spec_from_file_location(
        "make_acceptance_quality", os.path.join(GOLDEN, "make_acceptance_quality.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


MAKER = _maker()
STORED = json.load(open(os.path.join(GOLDEN, "acceptance_quality.json")))
CASES = {c[0]: c for c in MAKER.CASES}


def paired_check(a, b, scale=1.0):
    """|mean(a - b)| <= 3 standard errors of the paired differences."""
    d = (np.asarray(a, np.float64) - np.asarray(b, np.float64)) / scale
    se = d.std(ddof=1) / np.sqrt(d.size)
    return float(d.mean()), float(se)


def check_stats(rec, n_t):
    assert len(rec["ids"]) >= 2000
    m, se = paired_check(rec["err_table"], rec["err_exact"], scale=n_t)
    assert abs(m) <= 3.0 * se + 1e-12, f"SER differs by {m:.5f} (paired SE {se:.5f})"
    m, se = paired_check(rec["res_table"], rec["res_exact"])
    assert abs(m) <= 3.0 * se + 1e-12, f"mean residual differs by {m:.5f} (paired SE {se:.5f})"


def check_reproduces(rec, fresh, rows):
    for key in ("err_table", "err_exact"):
        assert np.array_equal(np.asarray(rec[key])[rows], np.asarray(fresh[key])), key
    for key in ("res_table", "res_exact"):
        assert np.allclose(np.asarray(rec[key])[rows], np.asarray(fresh[key]), rtol=1e-11,
                           atol=0.0), key


@pytest.mark.parametrize("name", ["8x8-16qam-15dB-64x200-random",
                                  "8x8-16qam-15dB-64x50-fallback"])
def test_table_acceptance_matches_exact_metropolis_8x8(name):
    case = CASES[name]
    rec = STORED["cases"][name]
    fresh = MAKER.run_case(case)                     # every stored instance, recomputed
    assert fresh["ids"] == rec["ids"]
    check_reproduces(rec, fresh, np.arange(len(rec["ids"])))
    check_stats(rec, case[2])


def test_table_acceptance_matches_exact_metropolis_16x16():
    name = "16x16-64qam-25dB-128x400-fallback"
    case = CASES[name]
    rec = STORED["cases"][name]
    rows = np.sort(np.random.default_rng(3).choice(len(rec["ids"]), 40, replace=False))
    fresh = MAKER.run_case(case, ids=np.asarray(rec["ids"])[rows])
    check_reproduces(rec, fresh, rows)
    check_stats(rec, case[2])


def test_exact_reference_is_plain_metropolis():
    """The reference chain itself: at a fixed temperature the final states of
    independent chains (4000 instances of one tiny problem, three one-spin
    dimensions, 40 sweeps each) follow the Boltzmann law over all 8 states
    (chi-square, 7 degrees of freedom, p = 0.001), and at zero temperature
    (beta -> infinity) every final state is a one-flip local minimum."""
    from oracle import oracle as O
    rng = np.random.default_rng(11)
    K, n_runs, sweeps, beta = 3, 4000, 40, 0.2
    A = rng.standard_normal((K, K))
    G = (A.T @ A / K).astype(np.float32)[None]
    f = rng.standard_normal((1, K)).astype(np.float32)
    b2 = np.full(sweeps, beta / np.log(2.0), np.float32)
    res = O.solve_exact(np.repeat(G, n_runs, 0), np.repeat(f, n_runs, 0), K, 1,
                        np.array([1], np.int8), 1, sweeps, b2, 77,
                        inst_ids=np.arange(n_runs, dtype=np.uint32))
    seen = {}
    for s in res["spins"]:
        key = tuple(int(v) for v in s)
        seen[key] = seen.get(key, 0) + 1
    keys, energies = [], []
    for s in np.ndindex(2, 2, 2):
        x = 2.0 * np.array(s) - 1.0
        keys.append(tuple(int(v) for v in x))
        energies.append(float(x @ G[0].astype(np.float64) @ x - 2.0 * f[0].astype(np.float64) @ x))
    w = np.exp(-beta * (np.array(energies) - min(energies)))
    expect = n_runs * w / w.sum()
    obs = np.array([seen.get(k, 0) for k in keys], np.float64)
    assert expect.min() > 5.0
    chi2 = float(np.sum((obs - expect) ** 2 / expect))
    assert chi2 < 24.3, chi2

    G2, f2 = np.repeat(G, 50, 0), rng.standard_normal((50, K)).astype(np.float32)
    res = O.solve_exact(G2, f2, K, 1, np.array([1], np.int8), 4, 20,
                        np.full(20, 1e6, np.float32), 5, inst_ids=np.arange(50, dtype=np.uint32))
    for n in range(50):
        x = res["spins"][n].astype(np.float64)
        e0 = x @ G2[n] @ x - 2 * f2[n] @ x
        for k in range(K):
            y = x.copy()
            y[k] = -y[k]
            assert y @ G2[n] @ y - 2 * f2[n] @ y >= e0 - 1e-9
