"""Pins of the oracle's CIM-CAC dynamics (paper §2.3 Eqs. cim1/cim2, integrated
by Euler steps as in §3.2 and Appendix A) against facts that do not come from
the oracle itself:

* the fixed points of the uncoupled model and the Euler map's exact growth of
  the error variables there (closed forms of the equations);
* the coupling term, recovered from one Euler step, equals the dense spin-domain
  sum_{j != i} J_ij x_j + h_i x_a built from the plain definition of J and h;
* the model is odd in the amplitudes: negated initial amplitudes give an exactly
  negated trajectory and the same (gauge-fixed) spins;
* on tiny problems the best of a few anneals reaches the brute-force ground state
  (a quality pin: a sign or index mistake in the coupling fails it).
"""
import itertools

import numpy as np
import pytest

from oracle import oracle as O


def params(**kw):
    P = dict(O.CIM_DEFAULTS)
    P.update(kw)
    return P


def random_problem(rng, K, q):
    A = rng.standard_normal((K + 2, K))
    G = (A.T @ A / (K + 2)).astype(np.float32)
    f = rng.standard_normal(K).astype(np.float32)
    w = np.array([1 << (q - 1 - b) for b in range(q)], dtype=np.int8)
    return G, f, w


def test_uncoupled_amplitudes_settle_at_the_fixed_points():
    """G = 0, f = 0: dx/dt = (p - 1) x - x^3, so x -> +-sqrt(p - 1) keeping
    its sign for p > 1, and x -> 0 for p < 1."""
    K, q = 3, 2
    G = np.zeros((K, K), np.float32)
    f = np.zeros(K, np.float32)
    w = np.array([2, 1], np.int8)
    for seed in (1, 2, 3):
        x0 = O.cim_trajectory(G, f, K, q, w, 0, params(p=1.5), seed)["amp"]
        r = O.cim_trajectory(G, f, K, q, w, 4000, params(p=1.5, dt=0.02), seed)
        assert np.all(np.sign(r["amp"]) == np.sign(x0))
        assert np.allclose(np.abs(r["amp"]), np.sqrt(0.5), rtol=1e-5)
        r = O.cim_trajectory(G, f, K, q, w, 4000, params(p=0.5, dt=0.02), seed)
        assert np.all(np.abs(r["amp"]) < 1e-6)


def test_error_variables_follow_the_euler_map_at_the_fixed_point():
    """With x at its fixed point x^2 = p - 1, each Euler step multiplies e by
    1 - dt zeta (p - 1 - a) exactly (up to float32 rounding)."""
    K, q = 2, 1
    G = np.zeros((K, K), np.float32)
    f = np.zeros(K, np.float32)
    w = np.array([1], np.int8)
    dt, zeta, p, a = 0.02, 0.5, 1.5, 1.0
    P = params(p=p, dt=dt, zeta=zeta, a=a)
    e1 = O.cim_trajectory(G, f, K, q, w, 3000, P, 7)["err"].astype(np.float64)
    e2 = O.cim_trajectory(G, f, K, q, w, 3100, P, 7)["err"].astype(np.float64)
    factor = (1.0 - dt * zeta * (p - 1.0 - a)) ** 100
    assert np.allclose(e2 / e1, factor, rtol=1e-4)
    # x -> 0 (p < 1): each step multiplies e by 1 + dt zeta a
    P = params(p=0.5, dt=dt, zeta=0.01, a=a)
    e1 = O.cim_trajectory(G, f, K, q, w, 3000, P, 7)["err"].astype(np.float64)
    e2 = O.cim_trajectory(G, f, K, q, w, 3050, P, 7)["err"].astype(np.float64)
    assert np.allclose(e2 / e1, (1.0 + dt * 0.01 * a) ** 50, rtol=1e-4)


@pytest.mark.parametrize("K,q", [(4, 1), (3, 2), (4, 3)])
def test_coupling_term_equals_the_dense_spin_form(K, q):
    """One Euler step from the start: (x1 - x0)/dt - (p - 1) x0 + x0^3 equals
    eps * e0 * c(x0) with e0 = 1 and c from the dense J, h (float64)."""
    rng = np.random.default_rng(K * 10 + q)
    G, f, w = random_problem(rng, K, q)
    J, h, _ = O.spin_ising(G, f, q, w)
    N = K * q
    dt, eps, p = 0.02, 0.75, 0.9
    for seed in range(4):
        P = params(dt=dt, eps=eps, p=p, amp0=0.8)
        x0 = O.cim_trajectory(G, f, K, q, w, 0, P, seed)["amp"].astype(np.float64)
        x1 = O.cim_trajectory(G, f, K, q, w, 1, P, seed)["amp"].astype(np.float64)
        c_obs = ((x1 - x0) / dt - (p - 1.0) * x0 + x0 ** 3) / eps
        xs, xa = x0[:N], x0[N]
        c_ref = np.concatenate([J @ xs + h * xa, [h @ xs]])
        scale = np.abs(J).sum(axis=1).max() + np.abs(h).sum()
        assert np.allclose(c_obs, c_ref, rtol=0, atol=2e-5 * scale / dt * 1e-2 + 1e-4 * scale)


def test_dynamics_are_odd_in_the_amplitudes():
    rng = np.random.default_rng(5)
    K, q = 4, 2
    G, f, w = random_problem(rng, K, q)
    xfb = np.array([3, -1, 1, -3], np.int8)
    a = O.cim_trajectory(G, f, K, q, w, 150, params(amp0=0.3), 9, x_fb=xfb, init_mode=1)
    b = O.cim_trajectory(G, f, K, q, w, 150, params(amp0=-0.3), 9, x_fb=xfb, init_mode=1)
    assert np.array_equal(a["amp"].view(np.uint32), (-b["amp"]).view(np.uint32))
    assert np.array_equal(a["err"].view(np.uint32), b["err"].view(np.uint32))
    assert np.array_equal(a["spins"], b["spins"])


def test_refresh_period_one_and_two_differ_only_through_the_held_coupling():
    """f_mvm = 1 and f_mvm = 2 agree after a single step (both use c(x0))."""
    rng = np.random.default_rng(11)
    K, q = 3, 2
    G, f, w = random_problem(rng, K, q)
    a = O.cim_trajectory(G, f, K, q, w, 1, params(f_mvm=1), 4)
    b = O.cim_trajectory(G, f, K, q, w, 1, params(f_mvm=2), 4)
    assert np.array_equal(a["amp"], b["amp"])
    a = O.cim_trajectory(G, f, K, q, w, 2, params(f_mvm=1), 4)
    b = O.cim_trajectory(G, f, K, q, w, 2, params(f_mvm=2), 4)
    assert not np.array_equal(a["amp"], b["amp"])


def test_best_anneal_reaches_the_brute_force_ground_state_on_tiny_problems():
    rng = np.random.default_rng(21)
    K, q = 3, 1
    hits, trials = 0, 30
    for t in range(trials):
        G, f, w = random_problem(rng, K, q)
        best = min(O.level_energy32(G, f, np.array(lv, np.int8))
                   for lv in itertools.product((-1, 1), repeat=K))
        r = O.cim_solve(G[None], f[None], K, q, w, 16, 300, params(), 100 + t)
        hits += bool(r["E"][0] <= best + 1e-5 * max(1.0, abs(best)))
    assert hits >= 27, hits


def test_solve_selects_like_the_metropolis_solver():
    """Selection and fallback are shared: with the fallback at the ground state
    the result is never worse than the fallback."""
    rng = np.random.default_rng(31)
    K, q = 4, 2
    G, f, w = random_problem(rng, K, q)
    lvs = list(itertools.product((-3, -1, 1, 3), repeat=K))
    es = [O.level_energy32(G, f, np.array(lv, np.int8)) for lv in lvs]
    gs = np.array(lvs[int(np.argmin(es))], np.int8)
    r = O.cim_solve(G[None], f[None], K, q, w, 4, 20, params(), 3, x_fb=gs[None])
    assert r["E"][0] <= min(es) + 1e-6
    assert 0 <= r["win"][0] <= 4


def test_divergence_rule_on_hand_built_states():
    amp = np.array([0.5, -2.0, 0.1, 1.0], np.float32)       # 3 spins + auxiliary
    err = np.ones(4, np.float32)
    assert not O.cim_diverged(amp, err, 3)
    for bad in (np.float32(1e4), np.float32(np.inf), np.float32(np.nan)):
        a = amp.copy(); a[1] = bad
        assert O.cim_diverged(a, err, 3)
        a = amp.copy(); a[3] = bad                           # the auxiliary amplitude
        assert O.cim_diverged(a, err, 3)
        a = amp.copy(); a[2] = bad                           # a padded spin is not checked
        assert not O.cim_diverged(a, err, 2)
    e = err.copy(); e[0] = np.inf
    assert O.cim_diverged(amp, e, 3)


def random_ising(seed, n, K):
    from workload import synth as W
    J, h = W.random_dense_ising(seed, n, K)
    return (-J / 2).astype(np.float32), (h / 2).astype(np.float32)


def test_integration_metrics_follow_the_step_size():
    """Appendix A: the fine-step reference against itself has no errors; a
    finer step stays close to it (Euler converges to the ODE solution); the
    sign errors grow with the step size and with the refresh period."""
    K, w = 12, np.array([1], np.int8)
    G, f = random_ising(3, 60, K)
    ref = O.cim_chains(G, f, K, 1, w, 1, 256, dict(dt=0.01, f_mvm=1), 7)
    m = O.cim_integration_metrics(ref["spins"], ref["diverged"], ref["spins"], ref["diverged"])
    assert m["p_error"] == 0.0 and m["p_diverge"] == 0.0
    fine = O.cim_chains(G, f, K, 1, w, 1, 512, dict(dt=0.005, f_mvm=1), 7)
    assert O.cim_integration_metrics(ref["spins"], ref["diverged"], fine["spins"],
                                     fine["diverged"])["p_error"] < 0.05
    errs = {}
    for dt, fm in ((0.02, 1), (0.08, 1), (0.08, 4)):
        r = O.cim_chains(G, f, K, 1, w, 1, int(round(2.56 / dt)), dict(dt=dt, f_mvm=fm), 7)
        errs[(dt, fm)] = O.cim_integration_metrics(ref["spins"], ref["diverged"], r["spins"],
                                                   r["diverged"])["p_error"]
    assert errs[(0.02, 1)] < errs[(0.08, 1)] < errs[(0.08, 4)]


def test_uncoupled_signs_survive_any_stable_step():
    """G = 0, f = 0: each amplitude keeps its sign under every Euler step with
    dt (1 - p + x^2) < 1, so every setting reproduces the reference spins."""
    K, w = 8, np.array([1], np.int8)
    G = np.zeros((20, K, K), np.float32)
    f = np.zeros((20, K), np.float32)
    ref = O.cim_chains(G, f, K, 1, w, 1, 256, dict(dt=0.01, f_mvm=1), 3)
    for dt, fm in ((0.02, 2), (0.08, 8)):
        r = O.cim_chains(G, f, K, 1, w, 1, int(round(2.56 / dt)), dict(dt=dt, f_mvm=fm), 3)
        m = O.cim_integration_metrics(ref["spins"], ref["diverged"], r["spins"], r["diverged"])
        assert m["p_error"] == 0.0 and m["p_diverge"] == 0.0
