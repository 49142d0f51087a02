"""Pins of the oracle's MMSE-SIC detector and of MMGaP-E (paper §1, §4 MMSE-SIC
baseline; §3.2 Fig. 6 two guesses, several stages, best answer) against facts
that do not come from the oracle itself:

* one user: MMSE-SIC is the sliced MMSE estimate (``mmse`` solves the normal
  equations with a library solver);
* the ordering and the nulling rows equal the MMSE V-BLAST construction through
  the augmented channel [H; sigma I] and its pseudo-inverse (an SVD routine):
  the user detected first has the pseudo-inverse row of smallest norm, and its
  estimate is that row applied to [y; 0];
* noise-free received vectors of a well-conditioned channel are recovered
  exactly, whatever the ordering;
* at high SNR the ordered cancellation makes fewer symbol errors than the
  linear MMSE detector (a dropped cancellation or a wrong conjugate fails it);
* MMGaP-E returns, per instance, whichever of its two chains' answers has the
  lower float32 energy, never above either guess, and reaches the brute-force
  ML answer on tiny problems where the guesses are near it.
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O
from workload import synth as W


def test_single_user_is_sliced_mmse():
    d = W.det_slot(61, 4, 1, 16, 30, 4, 12.0)
    r = O.mmse_sic(d.H, d.y, d.noise_var, 16)
    ref = O.slice_levels(O.mmse(d.H, d.y, d.noise_var), 16).reshape(-1, 2)
    assert np.array_equal(r["levels"], ref)


def vblast_first(H, y, noise_var):
    """The first step of MMSE V-BLAST via the augmented channel."""
    n_r, n_t = H.shape
    Ha = np.vstack([H, np.sqrt(noise_var) * np.eye(n_t)])
    Pinv = np.linalg.pinv(Ha)                              # [n_t][n_r + n_t]
    i = int(np.argmin((np.abs(Pinv) ** 2).sum(axis=1)))
    est = Pinv[i] @ np.concatenate([y, np.zeros(n_t)])
    return i, est


@pytest.mark.parametrize("n_r,n_t,snr", [(4, 4, 10.0), (8, 6, 15.0), (16, 16, 20.0)])
def test_ordering_and_first_estimate_follow_the_augmented_channel(n_r, n_t, snr):
    qam = 16
    d = W.det_slot(62 + n_t, n_r, n_t, qam, 12, 2, snr)
    r = O.mmse_sic(d.H, d.y, d.noise_var, qam)
    c = O.qam_scale(qam)
    for sc in range(12):
        H = d.H[sc].astype(np.complex128)
        i, est = vblast_first(H, d.y[sc, 0].astype(np.complex128), d.noise_var)
        assert r["order"][sc, 0] == i
        lv = r["levels"][sc * 2]
        li = np.clip(2 * np.floor(est.real / c / 2) + 1, -3, 3)
        lq = np.clip(2 * np.floor(est.imag / c / 2) + 1, -3, 3)
        assert (lv[i], lv[n_t + i]) == (li, lq)
        # the whole ordering by deleting the detected column and repeating
        rem = list(range(n_t))
        for step in range(n_t):
            Ha = np.vstack([H[:, rem], np.sqrt(d.noise_var) * np.eye(len(rem))])
            nrm = (np.abs(np.linalg.pinv(Ha)) ** 2).sum(axis=1)
            j = rem[int(np.argmin(nrm))]
            assert r["order"][sc, step] == j, (sc, step)
            rem.remove(j)


def test_noise_free_signals_are_recovered_exactly():
    rng = np.random.default_rng(7)
    n_sc, n_sym, n_r, n_t, qam = 6, 5, 8, 8, 64
    H = (rng.standard_normal((n_sc, n_r, n_t)) + 1j * rng.standard_normal((n_sc, n_r, n_t))) / 2
    H += 3 * np.eye(n_r, n_t)[None]                        # well conditioned
    sym = rng.integers(0, qam, size=(n_sc, n_sym, n_t))
    x = W.symbol_points(sym, qam)
    y = np.einsum("srt,sbt->sbr", H, x)
    r = O.mmse_sic(H.astype(np.complex64), y.astype(np.complex64), 1e-9, qam)
    assert np.array_equal(r["sym"], sym.reshape(-1, n_t))


def test_cancellation_beats_linear_mmse_at_high_snr():
    d = W.det_slot(63, 8, 8, 16, 200, 10, 20.0)
    truth = d.sym.reshape(-1, 8)
    sic = np.mean(O.mmse_sic(d.H, d.y, d.noise_var, 16)["sym"] != truth)
    lin = np.mean(O.levels_to_symbols(
        O.slice_levels(O.mmse(d.H, d.y, d.noise_var), 16).reshape(-1, 16), 16) != truth)
    assert sic < 0.5 * lin, (sic, lin)


def test_inst_ids_select_the_same_answers():
    d = W.det_slot(64, 6, 4, 64, 9, 5, 25.0)
    full = O.mmse_sic(d.H, d.y, d.noise_var, 64)
    ids = np.array([0, 4, 5, 17, 44], dtype=np.uint32)
    part = O.mmse_sic(d.H, d.y, d.noise_var, 64, inst_ids=ids)
    assert np.array_equal(part["levels"], full["levels"][ids])
    assert np.allclose(part["metric"], full["metric"][ids])


def test_mmgap_e_picks_the_lower_energy_chain():
    d = W.det_slot(65, 8, 8, 64, 5, 4, 25.0)
    b2 = W.linear_beta2(30, *W.det_beta_range(64, 8, d.noise_var))
    r = O.detect_e(d.H, d.y, d.noise_var, 64, 16, 30, b2, 11, stages=2)
    G, f = O.det_ising(d.H, d.y, 64)
    xm = O.slice_levels(O.mmse(d.H, d.y, d.noise_var), 64).reshape(-1, 16)
    xs = O.mmse_sic(d.H, d.y, d.noise_var, 64)["levels"]
    for n in range(20):
        Gi = G[n // 4]
        ea = O.level_energy32(Gi, f[n], r["a"]["levels"][n])
        eb = O.level_energy32(Gi, f[n], r["b"]["levels"][n])
        e = O.level_energy32(Gi, f[n], r["levels"][n])
        assert e == min(ea, eb)
        assert r["from_sic"][n] == (eb < ea)
        assert e <= O.level_energy32(Gi, f[n], xm[n])
        assert e <= O.level_energy32(Gi, f[n], xs[n])
    assert np.allclose(r["metric"], O.det_metric(d.H, d.y, r["levels"], 64))


def test_mmgap_e_reaches_the_ml_answer_on_tiny_problems():
    d = W.det_slot(66, 3, 2, 16, 10, 1, 14.0)
    b2 = W.linear_beta2(40, *W.det_beta_range(16, 3, d.noise_var))
    r = O.detect_e(d.H, d.y, d.noise_var, 16, 16, 40, b2, 5, stages=2)
    ml = np.stack([O.brute_force_ml(d.H[s], d.y[s, 0], 16) for s in range(10)])
    m_ml = O.det_metric(d.H, d.y, ml, 16)
    assert np.all(r["metric"] >= m_ml * (1 - 1e-9) - 1e-12)
    assert np.sum(np.isclose(r["metric"], m_ml, rtol=1e-6)) >= 9


def test_mmgap_e_single_chains_are_the_plain_searches():
    """guesses = 1 is the search from the MMSE guess (keys seed + s);
    guesses = 2 is the search from the MMSE-SIC guess with keys seed + 64 + s."""
    d = W.det_slot(67, 6, 4, 16, 5, 3, 15.0)
    b2 = W.linear_beta2(20, *W.det_beta_range(16, 6, d.noise_var))
    r1 = O.detect_e(d.H, d.y, d.noise_var, 16, 16, 20, b2, 8, stages=2, guesses=1)
    a = O.detect_delta(d.H, d.y, d.noise_var, 16, 16, 20, b2, 8, stages=2)
    assert np.array_equal(r1["levels"], a["levels"]) and not r1["from_sic"].any()
    r2 = O.detect_e(d.H, d.y, d.noise_var, 16, 16, 20, b2, 8, stages=2, guesses=2)
    g = O.mmse_sic(d.H, d.y, d.noise_var, 16)["levels"]
    b = O.detect_delta(d.H, d.y, d.noise_var, 16, 16, 20, b2, 8 + 64, stages=2, guess=g)
    assert np.array_equal(r2["levels"], b["levels"]) and r2["from_sic"].all()
    r3 = O.detect_e(d.H, d.y, d.noise_var, 16, 16, 20, b2, 8, stages=2)
    G, f = O.det_ising(d.H, d.y, 16)
    for n in range(15):
        e3 = O.level_energy32(G[n // 3], f[n], r3["levels"][n])
        assert e3 == min(O.level_energy32(G[n // 3], f[n], a["levels"][n]),
                         O.level_energy32(G[n // 3], f[n], b["levels"][n]))
