"""Pins of the oracle's detection around a guess (paper §2.3 Delta-Ising form,
§3.2 MMGaP-E stages) against facts that do not come from the oracle itself:

* energy identity: with f' = f - G x_g, the move energy z^T G z - 2 f'^T z equals
  E(x_g + z) - E(x_g) for the level energy E (float64 closed form);
* brute force: on small problems the best move found equals the minimum over all
  3^K moves (exhaustive enumeration in float64);
* the ML point is a fixed point: started at the brute-force ML solution a stage
  keeps it;
* stages never increase the energy of the guess, and with one stage of a
  Metropolis search the result equals the enumeration's best clamped move
  whenever that move is inside the constellation.
"""
import itertools

import numpy as np

from oracle import oracle as O
from workload import synth as W


def energy64(G, f, x):
    x = np.asarray(x, dtype=np.float64)
    return float(x @ G.astype(np.float64) @ x - 2.0 * f.astype(np.float64) @ x)


def test_move_energy_identity():
    d = W.det_slot(41, 6, 4, 16, 5, 3, 15.0)
    G, f = O.det_ising(d.H, d.y, 16)
    K = 8
    xg = O.slice_levels(O.mmse(d.H, d.y, d.noise_var), 16).reshape(-1, K)
    fp = O.delta_fields(G, f, xg, inst_per_G=3)
    rng = np.random.default_rng(2)
    for n in range(15):
        Gi = G[n // 3]
        for _ in range(5):
            z = rng.choice([-2, 0, 2], size=K)
            lhs = energy64(Gi, fp[n], z)
            rhs = energy64(Gi, f[n], xg[n] + z) - energy64(Gi, f[n], xg[n])
            assert abs(lhs - rhs) <= 1e-5 * max(1.0, abs(rhs)), (n, lhs, rhs)


def test_best_move_matches_enumeration():
    d = W.det_slot(42, 4, 2, 16, 12, 2, 12.0)           # K = 4: 81 moves per instance
    G, f = O.det_ising(d.H, d.y, 16)
    K = 4
    xg = O.slice_levels(O.mmse(d.H, d.y, d.noise_var), 16).reshape(-1, K)
    fp = O.delta_fields(G, f, xg, inst_per_G=2)
    b2 = W.linear_beta2(60, *W.det_beta_range(16, 4, d.noise_var))
    res = O.solve(G, fp, K, 2, O.DELTA_WEIGHTS, 32, 60, b2, 9, x_fb=np.zeros_like(xg),
                  inst_per_G=2)
    z = O.levels_from_spins(res["spins"], K, 2, O.DELTA_WEIGHTS)
    moves = np.array(list(itertools.product((-2, 0, 2), repeat=K)))
    hits = 0
    for n in range(xg.shape[0]):
        Gi = G[n // 2]
        e = np.array([energy64(Gi, fp[n], m) for m in moves])
        hits += abs(energy64(Gi, fp[n], z[n]) - e.min()) <= 1e-5 * max(1.0, abs(e.min()))
    assert hits == xg.shape[0]


def test_ml_point_is_a_fixed_point():
    d = W.det_slot(43, 3, 2, 16, 8, 1, 10.0)
    K = 4
    ml = np.stack([O.brute_force_ml(d.H[s], d.y[s, 0], 16) for s in range(8)]).astype(np.int8)
    b2 = W.linear_beta2(40, *W.det_beta_range(16, 3, d.noise_var))
    r = O.detect_delta(d.H, d.y, d.noise_var, 16, 16, 40, b2, 3, stages=2, guess=ml)
    assert np.array_equal(r["levels"], ml)


def test_stages_never_raise_the_energy_and_stay_in_the_constellation():
    d = W.det_slot(44, 8, 8, 64, 6, 4, 22.0)
    G, f = O.det_ising(d.H, d.y, 64)
    b2 = W.linear_beta2(30, *W.det_beta_range(64, 8, d.noise_var))
    r = O.detect_delta(d.H, d.y, d.noise_var, 64, 32, 30, b2, 5, stages=3)
    xg = O.slice_levels(O.mmse(d.H, d.y, d.noise_var), 64).reshape(-1, 16)
    prev = [O.level_energy32(G[n // 4], f[n], xg[n]) for n in range(24)]
    for lv in r["stage_levels"]:
        assert np.all(np.abs(lv) <= 7) and np.all(lv % 2 != 0)
        cur = [O.level_energy32(G[n // 4], f[n], lv[n]) for n in range(24)]
        assert all(c <= p for c, p in zip(cur, prev))
        prev = cur
    # the metric is the float64 residual of the final levels
    assert np.allclose(r["metric"], O.det_metric(d.H, d.y, r["levels"], 64))
