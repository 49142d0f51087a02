"""CPU oracle of the MMGaP Ising hot path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the GPU library: the plain
definitions are written out here in float64 numpy, and the stochastic chains
(which must reproduce the GPU's spins under identical Philox streams) are the
plain C loops of ``mmgap_oracle.c``.

Paper passages followed (arXiv 2510.01579):

* §2.1 Eq. 1 and Eq. ``ml``: y = Hx + noise, x_ML = argmin ||y - Hx||^2.
* §2.1 MMSE: x_MMSE = (H^H H + rho I)^-1 H^H y, rho = E|noise|^2 / E|x|^2.
* §1/§4 MMSE-SIC baseline and §3.2 MMGaP-E (two guesses, MMSE and MMSE-SIC,
  several stages each, best answer overall): ``mmse_sic``, ``detect_e``; the
  SIC ordering rule is not given in the paper (reading: smallest MMSE error
  variance first).
* §2.2 ZF precoder W = H^H (H H^H)^-1 and the VPP problem
  v* = argmin ||W (u + tau v)||; §3.3 rewrites it with y~ = W u and
  H_p = -tau W / 2 as argmin_{v in 2Z} ||y~ - H_p v||, solved like detection
  with an all-zeros vector in place of the MMSE solution.
* §2.3 Ising problem; §3.2 "Processing Flow": N_a anneals per problem, each
  anneal's final state is a candidate, candidates are ranked by the Eq. ``ml``
  energy, the MMSE solution replaces a candidate whose energy is larger, and
  the best candidate is returned.

Readings (where the paper is silent), all shared with the GPU library's
contract: binary-weighted spin encoding x_k = sum_b 2^(q-1-b) s_{k,b} of the
odd PAM levels (VPP: two unit-weight spins per real dimension, levels
{-2, 0, 2} = 2v); a single-spin-flip Metropolis anneal (the default dynamics),
with the local field of a dimension recomputed from the current levels at each
visit (one row of the coupling matrix-vector product) and a 16-bit uniform
compared with a tabulated 2^16 * 2^-z, z quantised to 1/64; couplings and
fields built in float64 and rounded once to float32.  The paper's own CIM-CAC
dynamics (§2.3 Eqs. cim1/cim2, integrated as in §3.2 and Appendix A) is the
second dynamics, ``cim_solve``: Euler steps of the amplitudes and error
variables, the coupling term through the structured K x K product, refreshed
every f_mvm steps, spins read as signs; its free parameters a, p, zeta, eps and
the initial amplitude are readings (``CIM_DEFAULTS``).

Parity pins live in tests/test_oracle_*.py (closed forms, library routines,
brute force, known-answer vectors, invariants).  The chain dynamics themselves
have no numeric reference in the paper (its solver is CIM-CAC and its figures
are not available): *parity unpinned* for solution quality versus the paper.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    """Load (building if needed) the oracle's C library."""
    global _lib
    if _lib is None:
        path = _build.build_oracle(force=False)
        L = ctypes.CDLL(path)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.oracle_philox4x32_10.restype = None
        L.oracle_draw16.argtypes = [ctypes.c_uint32] * 4 + [ctypes.c_uint64]
        L.oracle_draw16.restype = ctypes.c_uint32
        L.oracle_accept.argtypes = [ctypes.c_float, ctypes.c_uint32]
        L.oracle_accept.restype = ctypes.c_int
        L.oracle_accept_table.argtypes = [ctypes.c_void_p]
        L.oracle_accept_table.restype = None
        L.oracle_solve.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,  # n K q w
            ctypes.c_void_p, ctypes.c_int, ctypes.c_long,                # G inst_per_G g_base
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,           # f x_fb inst_ids
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        L.oracle_solve.restype = ctypes.c_int
        L.oracle_solve_exact.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,  # n K q w
            ctypes.c_void_p, ctypes.c_int, ctypes.c_long,                # G inst_per_G g_base
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,           # f x_fb inst_ids
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        L.oracle_solve_exact.restype = ctypes.c_int
        L.oracle_level_energy.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.c_void_p]
        L.oracle_level_energy.restype = ctypes.c_float
        L.oracle_vpp_build.argtypes = [ctypes.c_int] * 4 + [ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_int]
        L.oracle_vpp_build.restype = ctypes.c_int
        L.oracle_cim_solve.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,  # n K q w
            ctypes.c_void_p, ctypes.c_int, ctypes.c_long,                # G inst_per_G g_base
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,           # f x_fb inst_ids
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int,
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        L.oracle_cim_solve.restype = ctypes.c_int
        L.oracle_cim_trajectory.argtypes = [
            ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
            ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_void_p]
        L.oracle_cim_trajectory.restype = ctypes.c_int
        L.oracle_delta_fields.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                          ctypes.c_int, ctypes.c_long, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        L.oracle_delta_fields.restype = ctypes.c_int
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Constellation and encoding (reading of the paper's unspecified encoding)

def qam_bits(qam: int) -> int:
    """q = log2(M)/2 spins per real dimension."""
    q = {4: 1, 16: 2, 64: 3, 256: 4}.get(int(qam))
    if q is None:
        raise ValueError(f"unsupported QAM order {qam}")
    return q


def qam_scale(qam: int) -> float:
    """c with unit average energy: E|x|^2 = 2 c^2 (M-1)/3 = 1."""
    return 1.0 / math.sqrt(2.0 * (qam - 1) / 3.0)


def det_weights(qam: int) -> np.ndarray:
    """Binary weights w_b = 2^(q-1-b), MSB first (int8)."""
    q = qam_bits(qam)
    return np.array([1 << (q - 1 - b) for b in range(q)], dtype=np.int8)


VPP_WEIGHTS = np.array([1, 1], dtype=np.int8)


def levels_from_spins(spins: np.ndarray, K: int, q: int, w: np.ndarray) -> np.ndarray:
    s = np.asarray(spins, dtype=np.int64).reshape(-1, K, q)
    return (s * np.asarray(w, dtype=np.int64)[None, None, :]).sum(axis=2)


def vpp_tau(qam: int) -> float:
    """tau = 2 (c_max + d/2) = 2 sqrt(M) c for the square M-QAM alphabet."""
    return 2.0 * math.sqrt(qam) * qam_scale(qam)


# --------------------------------------------------------------------------
# Real decomposition and the Ising form (float64 definitions)

def real_matrix(H: np.ndarray) -> np.ndarray:
    """H_r = [[Re H, -Im H], [Im H, Re H]] so that (H x)_r = H_r x_r."""
    A = H.real.astype(np.float64)
    B = H.imag.astype(np.float64)
    top = np.concatenate([A, -B], axis=-1)
    bot = np.concatenate([B, A], axis=-1)
    return np.concatenate([top, bot], axis=-2)


def real_vector(y: np.ndarray) -> np.ndarray:
    """y_r = [Re y; Im y] along the last axis."""
    return np.concatenate([y.real, y.imag], axis=-1).astype(np.float64)


def det_ising64(H: np.ndarray, y: np.ndarray, qam: int):
    """float64 couplings and fields of the detection problem.

    ||y - H c x||^2 = ||y||^2 + x^T (c^2 H_r^T H_r) x - 2 (c H_r^T y_r)^T x, so
    G = c^2 H_r^T H_r (per subcarrier) and f = c H_r^T y_r (per instance).
    H_r^T H_r is the real form [[X, -Y], [Y, X]] of the Hermitian Gram
    H^H H = X + iY, taken exactly Hermitian (upper triangle mirrored, real
    diagonal); H_r^T y_r = [Re F; Im F] with F = H^H y.
    H: [n_sc][n_r][n_t]; y: [n_sc][n_sym][n_r].
    """
    c = qam_scale(qam)
    c2 = 1.0 / (2.0 * (qam - 1) / 3.0)
    Hc = H.astype(np.complex128)
    n_t = Hc.shape[-1]
    Cg = np.einsum("sra,srb->sab", np.conj(Hc), Hc)
    iu = np.triu_indices(n_t, 1)
    X = Cg.real.copy()
    Y = Cg.imag.copy()
    X[:, iu[1], iu[0]] = X[:, iu[0], iu[1]]
    Y[:, iu[1], iu[0]] = 0.0 - Y[:, iu[0], iu[1]]
    Y[:, np.arange(n_t), np.arange(n_t)] = 0.0
    top = np.concatenate([X, 0.0 - Y], axis=-1)
    bot = np.concatenate([Y, X], axis=-1)
    Gr = np.concatenate([top, bot], axis=-2)
    F = np.einsum("sra,sbr->sba", np.conj(Hc), y.astype(np.complex128))
    fr = np.concatenate([F.real, F.imag], axis=-1)
    return Gr * c2, fr * c


def det_ising(H: np.ndarray, y: np.ndarray, qam: int):
    """float32 couplings [n_sc][K][K] and fields [n_sc*n_sym][K], each rounded once."""
    G64, f64 = det_ising64(H, y, qam)
    K = G64.shape[-1]
    return G64.astype(np.float32), f64.reshape(-1, K).astype(np.float32)


def mmse(H: np.ndarray, y: np.ndarray, noise_var: float) -> np.ndarray:
    """x_MMSE = (H^H H + rho I)^-1 H^H y with rho = sigma^2 (unit-energy symbols)."""
    H = H.astype(np.complex128)
    y = y.astype(np.complex128)
    n_t = H.shape[-1]
    Hh = np.conj(np.swapaxes(H, -1, -2))
    A = Hh @ H + noise_var * np.eye(n_t)[None]
    rhs = Hh @ np.swapaxes(y, -1, -2)                           # [n_sc][n_t][n_sym]
    x = np.linalg.solve(A, rhs)
    return np.swapaxes(x, -1, -2)                                # [n_sc][n_sym][n_t]


def slice_levels(x: np.ndarray, qam: int) -> np.ndarray:
    """Nearest odd PAM level per real dimension: 2 floor(t/2) + 1 with t = x/c,
    clamped to +-(2^q - 1).  Returns int8 [..., 2 n_t] in real-form order."""
    q = qam_bits(qam)
    top = (1 << q) - 1
    t = real_vector(x) / qam_scale(qam)
    lv = 2.0 * np.floor(t / 2.0) + 1.0
    lv = np.clip(lv, -top, top)
    return lv.astype(np.int8)


def levels_to_symbols(levels: np.ndarray, qam: int) -> np.ndarray:
    """Real-form levels [..., 2 n_t] -> Gray-labelled symbol indices [..., n_t]."""
    q = qam_bits(qam)
    lv = np.asarray(levels, dtype=np.int64)
    n_t = lv.shape[-1] // 2
    top = (1 << q) - 1
    pI = (lv[..., :n_t] + top) // 2
    pQ = (lv[..., n_t:] + top) // 2
    gI = pI ^ (pI >> 1)
    gQ = pQ ^ (pQ >> 1)
    return ((gI << q) | gQ).astype(np.uint8)


def det_metric(H: np.ndarray, y: np.ndarray, levels: np.ndarray, qam: int) -> np.ndarray:
    """||y - H c x||^2 (Eq. ml objective) in float64, per instance.

    H [n_sc][n_r][n_t]; y [n_sc][n_sym][n_r]; levels [n_sc*n_sym][2 n_t]."""
    n_sc, n_sym, n_r = y.shape
    n_t = H.shape[-1]
    lv = np.asarray(levels, dtype=np.float64).reshape(n_sc, n_sym, 2 * n_t)
    x = qam_scale(qam) * (lv[..., :n_t] + 1j * lv[..., n_t:])
    r = y.astype(np.complex128) - np.einsum("srt,sbt->sbr", H.astype(np.complex128), x)
    return (np.abs(r) ** 2).sum(axis=-1).reshape(-1)


# --------------------------------------------------------------------------
# The anneal (C loops) and selection

def solve(G, f, K, q, w, chains, sweeps, beta2, seed, x_fb=None, inst_per_G=1,
          inst_ids=None, init_mode=0, nthreads=0, want_chain_energies=False):
    """Best-of-`chains` Metropolis anneals per instance, with optional fallback.

    G [n_G][K][K] float32 (instance n uses G[inst_ids[n] // inst_per_G - g_base]
    where g_base is inst_ids.min() // inst_per_G); f [n][K]; x_fb [n][K] int8 or
    None.  Returns dict(spins int8 [n][K*q], E float32 [n], win int32 [n],
    chain_E [n][chains] if requested).
    """
    G = np.ascontiguousarray(G, dtype=np.float32).reshape(-1, K, K)
    f = np.ascontiguousarray(f, dtype=np.float32).reshape(-1, K)
    n = f.shape[0]
    w = np.ascontiguousarray(w, dtype=np.int8)
    if w.shape != (q,):
        raise ValueError("w must have q entries")
    beta2 = np.ascontiguousarray(beta2, dtype=np.float32)
    if beta2.shape != (sweeps,):
        raise ValueError("beta2 must have `sweeps` entries")
    if inst_ids is None:
        ids = None
        g_base = 0
    else:
        ids = np.ascontiguousarray(inst_ids, dtype=np.uint32)
        if ids.shape != (n,):
            raise ValueError("inst_ids must have one entry per instance")
        g_base = 0
    if x_fb is not None:
        x_fb = np.ascontiguousarray(x_fb, dtype=np.int8).reshape(n, K)
    spins = np.zeros((n, K * q), dtype=np.int8)
    E = np.zeros(n, dtype=np.float32)
    win = np.zeros(n, dtype=np.int32)
    chainE = np.zeros((n, chains), dtype=np.float32) if want_chain_energies else None
    rc = lib().oracle_solve(n, K, q, _ptr(w), _ptr(G), int(inst_per_G), int(g_base), _ptr(f),
                            _ptr(x_fb), _ptr(ids), int(chains), int(sweeps), _ptr(beta2),
                            int(seed) & 0xFFFFFFFFFFFFFFFF, int(init_mode), _ptr(spins),
                            _ptr(E), _ptr(win), _ptr(chainE), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_solve failed ({rc})")
    out = dict(spins=spins, E=E, win=win)
    if chainE is not None:
        out["chain_E"] = chainE
    return out


def solve_exact(G, f, K, q, w, chains, sweeps, beta2, seed, x_fb=None, inst_per_G=1,
                inst_ids=None, init_mode=0, nthreads=0):
    """Plain Metropolis reference anneals (a quality reference, not a parity
    target): the anneal of ``solve`` -- same sweep order, initial spins and
    16-bit draws m -- computed from the definitions in float64, accepting a
    flip iff dE <= 0 or (m + 1/2)/2^16 < 2^(-beta2_t dE) exactly (no threshold
    table, z not quantised), candidates ranked by the float64 energy.  Same
    arguments as ``solve``; returns dict(spins, E float64, win)."""
    G = np.ascontiguousarray(G, dtype=np.float32).reshape(-1, K, K)
    f = np.ascontiguousarray(f, dtype=np.float32).reshape(-1, K)
    n = f.shape[0]
    w = np.ascontiguousarray(w, dtype=np.int8)
    beta2 = np.ascontiguousarray(beta2, dtype=np.float32)
    if w.shape != (q,) or beta2.shape != (sweeps,):
        raise ValueError("w must have q entries and beta2 `sweeps` entries")
    ids = None if inst_ids is None else np.ascontiguousarray(inst_ids, dtype=np.uint32)
    if ids is not None and ids.shape != (n,):
        raise ValueError("inst_ids must have one entry per instance")
    if x_fb is not None:
        x_fb = np.ascontiguousarray(x_fb, dtype=np.int8).reshape(n, K)
    spins = np.zeros((n, K * q), dtype=np.int8)
    E = np.zeros(n, dtype=np.float64)
    win = np.zeros(n, dtype=np.int32)
    rc = lib().oracle_solve_exact(n, K, q, _ptr(w), _ptr(G), int(inst_per_G), 0, _ptr(f),
                                  _ptr(x_fb), _ptr(ids), int(chains), int(sweeps), _ptr(beta2),
                                  int(seed) & 0xFFFFFFFFFFFFFFFF, int(init_mode), _ptr(spins),
                                  _ptr(E), _ptr(win), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_solve_exact failed ({rc})")
    return dict(spins=spins, E=E, win=win)


# CIM-CAC model parameters (paper §2.3 Eqs. cim1/cim2, Appendix A): the
# integration step and coupling refresh period are the paper's choice
# (dt = 0.02, f_mvm = 2, 128 steps = the 2.56 time units of its reference
# 256 x 0.01); a, p, zeta, eps and the initial amplitude are not given in the
# paper and are this implementation's reading.
CIM_DEFAULTS = dict(dt=0.02, f_mvm=2, p=0.9, a=1.0, zeta=1.0, eps=1.0, amp0=0.1)
CIM_KEYS = ("dt", "f_mvm", "p", "a", "zeta", "eps", "amp0")


def cim_param_vector(cim: dict) -> np.ndarray:
    """The 7 model parameters as the float32 vector the C oracle takes."""
    P = dict(CIM_DEFAULTS)
    P.update(cim or {})
    return np.array([P[k] for k in CIM_KEYS], dtype=np.float32)


def cim_solve(G, f, K, q, w, chains, steps, cim, seed, x_fb=None, inst_per_G=1,
              inst_ids=None, init_mode=0, nthreads=0, want_chain_energies=False):
    """Best-of-`chains` CIM-CAC anneals of `steps` Euler steps per instance, with
    optional fallback (same selection as solve()).  cim: model parameters
    (keys of CIM_DEFAULTS; missing keys take the defaults)."""
    G = np.ascontiguousarray(G, dtype=np.float32).reshape(-1, K, K)
    f = np.ascontiguousarray(f, dtype=np.float32).reshape(-1, K)
    n = f.shape[0]
    w = np.ascontiguousarray(w, dtype=np.int8)
    if w.shape != (q,):
        raise ValueError("w must have q entries")
    ids = None if inst_ids is None else np.ascontiguousarray(inst_ids, dtype=np.uint32)
    if ids is not None and ids.shape != (n,):
        raise ValueError("inst_ids must have one entry per instance")
    if x_fb is not None:
        x_fb = np.ascontiguousarray(x_fb, dtype=np.int8).reshape(n, K)
    params = cim_param_vector(cim)
    spins = np.zeros((n, K * q), dtype=np.int8)
    E = np.zeros(n, dtype=np.float32)
    win = np.zeros(n, dtype=np.int32)
    chainE = np.zeros((n, chains), dtype=np.float32) if want_chain_energies else None
    rc = lib().oracle_cim_solve(n, K, q, _ptr(w), _ptr(G), int(inst_per_G), 0, _ptr(f),
                                _ptr(x_fb), _ptr(ids), int(chains), int(steps), _ptr(params),
                                int(seed) & 0xFFFFFFFFFFFFFFFF, int(init_mode), _ptr(spins),
                                _ptr(E), _ptr(win), _ptr(chainE), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_cim_solve failed ({rc})")
    out = dict(spins=spins, E=E, win=win)
    if chainE is not None:
        out["chain_E"] = chainE
    return out


def cim_trajectory(G, f, K, q, w, steps, cim, seed, inst=0, ch=0, x_fb=None, init_mode=0):
    """Amplitudes [K q + 1] and error variables [K q + 1] of one CIM-CAC anneal
    after `steps` steps (auxiliary spin last), its final spins and energy."""
    G = np.ascontiguousarray(G, dtype=np.float32).reshape(K, K)
    f = np.ascontiguousarray(f, dtype=np.float32).reshape(K)
    w = np.ascontiguousarray(w, dtype=np.int8)
    N = K * q
    amp = np.zeros(N + 1, dtype=np.float32)
    err = np.zeros(N + 1, dtype=np.float32)
    spins = np.zeros(N, dtype=np.int8)
    E = np.zeros(1, dtype=np.float32)
    if x_fb is not None:
        x_fb = np.ascontiguousarray(x_fb, dtype=np.int8).reshape(K)
    rc = lib().oracle_cim_trajectory(K, q, _ptr(w), _ptr(G), _ptr(f), _ptr(x_fb), int(steps),
                                     _ptr(cim_param_vector(cim)), int(seed) & 0xFFFFFFFFFFFFFFFF,
                                     int(inst), int(ch), int(init_mode), _ptr(amp), _ptr(err),
                                     _ptr(spins), _ptr(E))
    if rc != 0:
        raise RuntimeError(f"oracle_cim_trajectory failed ({rc})")
    return dict(amp=amp, err=err, spins=spins, E=float(E[0]))



# Largest final amplitude magnitude of a CIM-CAC run not counted as diverged
# (reading: the paper calls a run diverged when its integration fails to
# converge, without a threshold; the amplitudes' fixed points are O(1)).
CIM_DIVERGE_BOUND = 1000.0


def cim_diverged(amp, err, n_real):
    """The divergence rule: an amplitude of one of the first n_real spins or of
    the auxiliary one (last) beyond the bound or not finite, or such an error
    variable not finite."""
    idx = list(range(n_real)) + [len(amp) - 1]
    a = np.abs(np.asarray(amp, dtype=np.float32)[idx])
    e = np.abs(np.asarray(err, dtype=np.float32)[idx])
    return bool(np.any(~(a <= CIM_DIVERGE_BOUND)) or np.any(~np.isfinite(e)))


def cim_chains(G, f, K, q, w, chains, steps, cim, seed, x_fb=None, inst_per_G=1, init_mode=0,
               inst_ids=None):
    """Every CIM-CAC anneal's final state (paper Appendix A studies): spins
    [m][chains][K q] (sign(x_i) sign(x_a)), energies [m][chains] and divergence
    flags [m][chains] for the instances `inst_ids` (default all)."""
    f = np.ascontiguousarray(f, dtype=np.float32)
    n = f.shape[0]
    G = np.ascontiguousarray(G, dtype=np.float32).reshape(-1, K, K)
    ids = np.arange(n) if inst_ids is None else np.asarray(inst_ids, dtype=np.int64)
    N = K * q
    spins = np.zeros((ids.size, chains, N), dtype=np.int8)
    E = np.zeros((ids.size, chains), dtype=np.float32)
    div = np.zeros((ids.size, chains), dtype=np.uint8)
    for r, i in enumerate(ids):
        xf = None if x_fb is None else np.asarray(x_fb)[i]
        for c in range(chains):
            t = cim_trajectory(G[i // inst_per_G], f[i], K, q, w, steps, cim, seed, inst=int(i),
                               ch=c, x_fb=xf, init_mode=init_mode)
            spins[r, c] = t["spins"]
            E[r, c] = t["E"]
            div[r, c] = cim_diverged(t["amp"], t["err"], N)
    return dict(spins=spins, E=E, diverged=div)


def cim_integration_metrics(ref_spins, ref_div, spins, div):
    """Appendix A's metrics of a setting against the fine-step reference run
    from the same initial values: P_diverge = diverged runs / runs; P_error =
    final spins whose sign differs from the reference's / spins, over the runs
    that diverged in neither."""
    ref_div = np.asarray(ref_div).astype(bool).reshape(-1)
    div = np.asarray(div).astype(bool).reshape(-1)
    N = np.asarray(spins).shape[-1]
    ok = ~ref_div & ~div
    a = np.asarray(ref_spins).reshape(-1, N)[ok]
    b = np.asarray(spins).reshape(-1, N)[ok]
    p_err = float(np.mean(a != b)) if a.size else float("nan")
    return dict(p_diverge=float(np.mean(div)), p_error=p_err, runs=int(div.size),
                compared=int(ok.sum()))

def level_energy32(G: np.ndarray, f: np.ndarray, levels: np.ndarray) -> float:
    """The float32 selection energy of given levels (same arithmetic as the chains)."""
    G = np.ascontiguousarray(G, dtype=np.float32)
    f = np.ascontiguousarray(f, dtype=np.float32)
    lv = np.ascontiguousarray(levels, dtype=np.int8)
    return float(lib().oracle_level_energy(int(f.shape[-1]), _ptr(G), _ptr(f), _ptr(lv)))


def detect(H, y, noise_var, qam, chains, sweeps, beta2, seed, inst_ids=None,
           init_mode=0, nthreads=0, cim=None):
    """Uplink ML-MIMO detection through the Ising reduction (paper §3.2).

    Returns dict(sym uint8 [n][n_t], metric float64 [n], levels int8 [n][K],
    E float32 [n], win int32 [n], spins int8 [n][K q]) for the instances
    inst = sc * n_sym + sym listed in inst_ids (all by default).
    """
    n_sc, n_sym, n_r = y.shape
    n_t = H.shape[-1]
    K, q = 2 * n_t, qam_bits(qam)
    w = det_weights(qam)
    G, f_all = det_ising(H, y, qam)
    x_fb_all = slice_levels(mmse(H, y, noise_var), qam).reshape(-1, K)
    ids = np.arange(n_sc * n_sym, dtype=np.uint32) if inst_ids is None \
        else np.asarray(inst_ids, dtype=np.uint32)
    if cim is None:
        res = solve(G, f_all[ids], K, q, w, chains, sweeps, beta2, seed,
                    x_fb=x_fb_all[ids], inst_per_G=n_sym, inst_ids=ids,
                    init_mode=init_mode, nthreads=nthreads)
    else:   # CIM-CAC anneals of `sweeps` Euler steps (beta2 unused)
        res = cim_solve(G, f_all[ids], K, q, w, chains, sweeps, cim, seed,
                        x_fb=x_fb_all[ids], inst_per_G=n_sym, inst_ids=ids,
                        init_mode=init_mode, nthreads=nthreads)
    lv = levels_from_spins(res["spins"], K, q, w).astype(np.int8)
    sc = ids // n_sym
    sy = ids % n_sym
    H_sel = H[sc]
    y_sel = y[sc, sy][:, None, :]
    metric = det_metric(H_sel, y_sel, lv, qam)
    res.update(sym=levels_to_symbols(lv, qam), metric=metric, levels=lv, inst_ids=ids,
               x_fb=x_fb_all[ids])
    return res


def detect_exact(H, y, noise_var, qam, chains, sweeps, beta2, seed, inst_ids=None,
                 init_mode=0, nthreads=0):
    """``detect`` with the plain float64 Metropolis reference anneals of
    ``solve_exact`` in place of the chain contract (same build, fallback,
    draws and decode).  A quality reference for the tabulated acceptance."""
    n_sc, n_sym, n_r = y.shape
    n_t = H.shape[-1]
    K, q = 2 * n_t, qam_bits(qam)
    w = det_weights(qam)
    G, f_all = det_ising(H, y, qam)
    x_fb_all = slice_levels(mmse(H, y, noise_var), qam).reshape(-1, K)
    ids = np.arange(n_sc * n_sym, dtype=np.uint32) if inst_ids is None \
        else np.asarray(inst_ids, dtype=np.uint32)
    res = solve_exact(G, f_all[ids], K, q, w, chains, sweeps, beta2, seed, x_fb=x_fb_all[ids],
                      inst_per_G=n_sym, inst_ids=ids, init_mode=init_mode, nthreads=nthreads)
    lv = levels_from_spins(res["spins"], K, q, w).astype(np.int8)
    sc = ids // n_sym
    sy = ids % n_sym
    metric = det_metric(H[sc], y[sc, sy][:, None, :], lv, qam)
    res.update(sym=levels_to_symbols(lv, qam), metric=metric, levels=lv, inst_ids=ids)
    return res


# --------------------------------------------------------------------------
# Downlink vector perturbation (paper §2.2, §3.3)

# --------------------------------------------------------------------------
# Detection around a guess (paper §2.3 Fig. 5 Delta-Ising form; §3.2 MMGaP-E)

DELTA_WEIGHTS = np.array([1, 1], dtype=np.int8)


def delta_fields(G, f, xg, inst_per_G=1, inst_ids=None):
    """f' = f - G x_g (float32, fma chain over l ascending from 0) per instance."""
    f = np.ascontiguousarray(f, dtype=np.float32)
    n, K = f.shape
    G = np.ascontiguousarray(G, dtype=np.float32).reshape(-1, K, K)
    xg = np.ascontiguousarray(xg, dtype=np.int8).reshape(n, K)
    ids = None if inst_ids is None else np.ascontiguousarray(inst_ids, dtype=np.uint32)
    out = np.zeros((n, K), dtype=np.float32)
    rc = lib().oracle_delta_fields(n, K, _ptr(G), int(inst_per_G), 0, _ptr(f), _ptr(xg),
                                   _ptr(ids), _ptr(out))
    if rc != 0:
        raise RuntimeError(f"oracle_delta_fields failed ({rc})")
    return out


def detect_delta(H, y, noise_var, qam, chains, sweeps, beta2, seed, stages=1, inst_ids=None,
                 init_mode=0, nthreads=0, cim=None, guess=None):
    """Detection by moves around a guess (paper §2.3 Delta-Ising form, §3.2
    MMGaP-E multi-stage).  Each real dimension moves by z in {-2, 0, 2} levels
    (one neighbouring constellation point either way), encoded by two
    unit-weight spins; the Ising problem keeps G and takes the fields
    f' = f - G x_g.  A stage anneals it (Metropolis, or CIM-CAC when `cim` is
    given) with the zero move as the fallback and the job seed + stage as the
    Philox key; the winning move is applied and clamped to the constellation,
    and the result replaces the guess only if its float32 energy is strictly
    lower.  The guess starts at the sliced MMSE estimate (or `guess`, int8
    levels [n][K]) and each stage starts from the previous stage's result.
    Returns dict(sym, metric, levels, stage_levels [stages][n][K])."""
    n_sc, n_sym, n_r = y.shape
    n_t = H.shape[-1]
    K, q = 2 * n_t, qam_bits(qam)
    top = (1 << q) - 1
    G, f_all = det_ising(H, y, qam)
    ids = np.arange(n_sc * n_sym, dtype=np.uint32) if inst_ids is None \
        else np.asarray(inst_ids, dtype=np.uint32)
    f = f_all[ids]
    if guess is None:
        xg = slice_levels(mmse(H, y, noise_var), qam).reshape(-1, K)[ids].astype(np.int8)
    else:
        xg = np.ascontiguousarray(guess, dtype=np.int8).reshape(ids.size, K).copy()
    zero = np.zeros((ids.size, K), dtype=np.int8)
    history = []
    for st in range(stages):
        fp = delta_fields(G, f, xg, inst_per_G=n_sym, inst_ids=ids)
        key = (int(seed) + st) & 0xFFFFFFFFFFFFFFFF
        if cim is None:
            res = solve(G, fp, K, 2, DELTA_WEIGHTS, chains, sweeps, beta2, key, x_fb=zero,
                        inst_per_G=n_sym, inst_ids=ids, init_mode=init_mode, nthreads=nthreads)
        else:
            res = cim_solve(G, fp, K, 2, DELTA_WEIGHTS, chains, sweeps, cim, key, x_fb=zero,
                            inst_per_G=n_sym, inst_ids=ids, init_mode=init_mode,
                            nthreads=nthreads)
        z = levels_from_spins(res["spins"], K, 2, DELTA_WEIGHTS).astype(np.int64)
        xc = np.clip(xg.astype(np.int64) + z, -top, top).astype(np.int8)
        for r in range(ids.size):
            Gi = G[ids[r] // n_sym]
            if level_energy32(Gi, f[r], xc[r]) < level_energy32(Gi, f[r], xg[r]):
                xg[r] = xc[r]
        history.append(xg.copy())
    sc = ids // n_sym
    sy = ids % n_sym
    metric = det_metric(H[sc], y[sc, sy][:, None, :], xg, qam)
    return dict(sym=levels_to_symbols(xg, qam), metric=metric, levels=xg, inst_ids=ids,
                stage_levels=history)



def mmse_sic(H, y, noise_var, qam, inst_ids=None):
    """MMSE successive interference cancellation (the paper's MMSE-SIC
    baseline, §1 and §4; MMGaP-E's second guess, §3.2).  The paper does not
    give the ordering rule; the reading here is the ordered MMSE-SIC: at each
    step the remaining user with the smallest MMSE error variance (the
    smallest diagonal entry of (H_R^H H_R + sigma^2 I)^-1, i.e. the largest
    post-detection SINR; ties to the lower user index) is estimated by its
    row of (H_R^H H_R + sigma^2 I)^-1 H_R^H applied to the residual, sliced to
    the nearest constellation point per real dimension, and its contribution
    h_i s_i is subtracted from the residual.  The ordering depends on H and
    sigma^2 only.  float64 throughout.

    Returns dict(levels int8 [n][2 n_t] (real-form order), order int
    [n_sc][n_t] (user detected at each step), sym, metric, margin [n]: the
    smallest distance of any scaled estimate x/c to a slicing boundary that
    changes the level, so that implementations summing in another order can
    only differ where it is tiny)."""
    n_sc, n_sym, n_r = y.shape
    n_t = H.shape[-1]
    q = qam_bits(qam)
    top = (1 << q) - 1
    c = qam_scale(qam)
    ids = np.arange(n_sc * n_sym) if inst_ids is None else np.asarray(inst_ids, dtype=np.int64)
    H = H.astype(np.complex128)
    y = y.astype(np.complex128)
    levels = np.zeros((ids.size, 2 * n_t), dtype=np.int8)
    order = np.zeros((n_sc, n_t), dtype=np.int64)
    margin = np.full(ids.size, np.inf)

    def boundary_gap(t):
        b = np.clip(2.0 * np.round(t / 2.0), -(top - 1), top - 1)
        return np.abs(t - b)
    for sc in np.unique(ids // n_sym):
        rows = np.where(ids // n_sym == sc)[0]
        Hs = H[sc]
        r = y[sc, ids[rows] % n_sym].copy()                  # residuals [m][n_r]
        remaining = list(range(n_t))
        for step in range(n_t):
            HR = Hs[:, remaining]
            P = np.linalg.inv(HR.conj().T @ HR + noise_var * np.eye(len(remaining)))
            d = np.real(np.diag(P))
            pos = int(np.argmin(d))                            # first index of the minimum
            i = remaining[pos]
            order[sc, step] = i
            w = P[pos] @ HR.conj().T                           # nulling row [n_r]
            xh = r @ w                                         # estimates [m]
            li = np.clip(2.0 * np.floor(xh.real / c / 2.0) + 1.0, -top, top)
            lq = np.clip(2.0 * np.floor(xh.imag / c / 2.0) + 1.0, -top, top)
            margin[rows] = np.minimum(margin[rows], np.minimum(boundary_gap(xh.real / c),
                                                               boundary_gap(xh.imag / c)))
            levels[rows, i] = li.astype(np.int8)
            levels[rows, n_t + i] = lq.astype(np.int8)
            r = r - np.outer(c * (li + 1j * lq), Hs[:, i])
            remaining.pop(pos)
    sc = ids // n_sym
    sy = ids % n_sym
    metric = det_metric(H[sc].astype(np.complex64), y[sc, sy][:, None, :], levels, qam)
    return dict(levels=levels, order=order, sym=levels_to_symbols(levels, qam), metric=metric,
                margin=margin)


# Philox key offset of the chain of stages that starts from the MMSE-SIC guess
# (the chain from the MMSE guess takes seed + s): keys never coincide for the
# at most 64 stages of a chain.
SIC_KEY_OFFSET = 64


def detect_e(H, y, noise_var, qam, chains, sweeps, beta2, seed, stages=1, inst_ids=None,
             init_mode=0, nthreads=0, cim=None, guesses=3):
    """MMGaP-E (paper §3.2, Fig. 6): per problem two chains of `stages`
    stages of moves around a guess, one from the MMSE estimate (Philox keys
    seed + s) and one from the MMSE-SIC estimate (keys seed + 64 + s); the
    output is the better of the two final answers by float32 level energy
    (the MMSE-SIC chain's only if strictly lower).  Returns dict(sym, metric,
    levels, from_sic bool [n], the two chains' results a, b, and sic_margin,
    the MMSE-SIC guess's slicing margin per instance).  `guesses` (bit 1 the
    MMSE chain, bit 2 the MMSE-SIC chain) may select one chain alone, whose
    answer is then the output."""
    n_sc, n_sym, _ = y.shape
    n_t = H.shape[-1]
    K = 2 * n_t
    ids = np.arange(n_sc * n_sym, dtype=np.uint32) if inst_ids is None \
        else np.asarray(inst_ids, dtype=np.uint32)
    if guesses not in (1, 2, 3):
        raise ValueError("guesses must be 1 (MMSE), 2 (MMSE-SIC) or 3 (both)")
    a = b = None
    sic = {"margin": np.full(ids.size, np.inf)}
    if guesses & 1:
        a = detect_delta(H, y, noise_var, qam, chains, sweeps, beta2, seed, stages=stages,
                         inst_ids=ids, init_mode=init_mode, nthreads=nthreads, cim=cim)
    if guesses & 2:
        sic = mmse_sic(H, y, noise_var, qam, inst_ids=ids)
        b = detect_delta(H, y, noise_var, qam, chains, sweeps, beta2,
                         (int(seed) + SIC_KEY_OFFSET) & 0xFFFFFFFFFFFFFFFF, stages=stages,
                         inst_ids=ids, init_mode=init_mode, nthreads=nthreads, cim=cim,
                         guess=sic["levels"])
    if b is None or a is None:
        one = a if b is None else b
        return dict(sym=one["sym"], metric=one["metric"], levels=one["levels"],
                    from_sic=np.full(ids.size, b is not None), inst_ids=ids, a=a, b=b,
                    sic_margin=sic["margin"])
    G, f_all = det_ising(H, y, qam)
    f = f_all[ids]
    lv = a["levels"].copy()
    from_sic = np.zeros(ids.size, dtype=bool)
    for r in range(ids.size):
        Gi = G[ids[r] // n_sym]
        if level_energy32(Gi, f[r], b["levels"][r]) < level_energy32(Gi, f[r], a["levels"][r]):
            lv[r] = b["levels"][r]
            from_sic[r] = True
    sc = ids // n_sym
    sy = ids % n_sym
    metric = det_metric(H[sc], y[sc, sy][:, None, :], lv.reshape(-1, K), qam)
    return dict(sym=levels_to_symbols(lv, qam), metric=metric, levels=lv, from_sic=from_sic,
                inst_ids=ids, a=a, b=b, sic_margin=sic["margin"])

def zf_precoder(H: np.ndarray) -> np.ndarray:
    """W = H^H (H H^H)^-1 in float64.  H [.., n_u, n_t] -> W [.., n_t, n_u]."""
    H = H.astype(np.complex128)
    Hh = np.conj(np.swapaxes(H, -1, -2))
    return Hh @ np.linalg.inv(H @ Hh)


def vpp_build(H: np.ndarray, u: np.ndarray, tau: float, nthreads: int = 0):
    """VPP couplings [n_sc][K][K], fields [n_sc*n_sym][K] (float32), and
    A^-1 = (H H^H)^-1 [n_sc][n_u][n_u] complex128, by the fixed-order
    LDL^H arithmetic of mmgap_oracle.c."""
    H = np.ascontiguousarray(H, dtype=np.complex64)
    u = np.ascontiguousarray(u, dtype=np.complex64)
    n_sc, n_u, n_t = H.shape
    n_sym = u.shape[1]
    K = 2 * n_u
    G = np.zeros((n_sc, K, K), dtype=np.float32)
    f = np.zeros((n_sc * n_sym, K), dtype=np.float32)
    Ainv = np.zeros((n_sc, n_u, n_u), dtype=np.complex128)
    rc = lib().oracle_vpp_build(n_sc, n_sym, n_u, n_t, _ptr(H), _ptr(u), float(tau),
                                _ptr(G), _ptr(f), _ptr(Ainv), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle_vpp_build failed ({rc})")
    return G, f, Ainv


def vpp_precode(H, u, qam, chains, sweeps, beta2, seed, tau=None, inst_ids=None,
                init_mode=0, nthreads=0, cim=None):
    """Vector-perturbation precoding through the Ising reduction (paper §3.3).

    Perturbation alphabet {-1, 0, 1} per real dimension, two unit-weight spins
    each (levels 2v); fallback v = 0 (plain ZF).  Returns dict(v int8 [n][K],
    x complex128 [n][n_t] = W (u + tau v), gamma float64 [n] = ||x||^2, E, win,
    spins) for the listed instances.
    """
    n_sc, n_sym, n_u = u.shape
    n_t = H.shape[-1]
    K = 2 * n_u
    tau = vpp_tau(qam) if tau is None or tau <= 0 else float(tau)
    G, f_all, _ = vpp_build(H, u, tau, nthreads=nthreads)
    ids = np.arange(n_sc * n_sym, dtype=np.uint32) if inst_ids is None \
        else np.asarray(inst_ids, dtype=np.uint32)
    x_fb = np.zeros((ids.size, K), dtype=np.int8)
    if cim is None:
        res = solve(G, f_all[ids], K, 2, VPP_WEIGHTS, chains, sweeps, beta2, seed, x_fb=x_fb,
                    inst_per_G=n_sym, inst_ids=ids, init_mode=init_mode, nthreads=nthreads)
    else:   # CIM-CAC anneals of `sweeps` Euler steps (beta2 unused)
        res = cim_solve(G, f_all[ids], K, 2, VPP_WEIGHTS, chains, sweeps, cim, seed, x_fb=x_fb,
                        inst_per_G=n_sym, inst_ids=ids, init_mode=init_mode, nthreads=nthreads)
    lv = levels_from_spins(res["spins"], K, 2, VPP_WEIGHTS)
    v = (lv // 2).astype(np.int8)
    sc = ids // n_sym
    sy = ids % n_sym
    W = zf_precoder(H[sc])                                       # [n][n_t][n_u]
    pert = u[sc, sy].astype(np.complex128) + tau * (v[:, :n_u] + 1j * v[:, n_u:])
    x = np.einsum("ntu,nu->nt", W, pert)
    res.update(v=v, x=x, gamma=(np.abs(x) ** 2).sum(axis=-1), inst_ids=ids, tau=tau)
    return res


# --------------------------------------------------------------------------
# Brute force (tiny sizes only) and the spin-domain expansion

def brute_force_ml(H: np.ndarray, y: np.ndarray, qam: int) -> np.ndarray:
    """Exhaustive Eq. ``ml`` over Omega^{n_t} for one instance: H [n_r][n_t],
    y [n_r]; returns the minimising real-form levels (int8 [2 n_t])."""
    q = qam_bits(qam)
    n_t = H.shape[-1]
    pam = np.arange(-(1 << q) + 1, 1 << q, 2)
    grids = np.meshgrid(*([pam] * (2 * n_t)), indexing="ij")
    cand = np.stack([g.reshape(-1) for g in grids], axis=1)      # [M^n_t][2 n_t]
    x = qam_scale(qam) * (cand[:, :n_t] + 1j * cand[:, n_t:])
    r = y.astype(np.complex128)[None, :] - x @ H.astype(np.complex128).T
    cost = (np.abs(r) ** 2).sum(axis=1)
    return cand[int(np.argmin(cost))].astype(np.int8)


def brute_force_vpp(H: np.ndarray, u: np.ndarray, tau: float) -> tuple[np.ndarray, float]:
    """Exhaustive VPP over v in {-1,0,1}^(2 n_u): H [n_u][n_t], u [n_u].
    Returns (v int8 [2 n_u], gamma = ||W (u + tau v)||^2)."""
    n_u = H.shape[0]
    W = zf_precoder(H)
    grids = np.meshgrid(*([np.array([-1, 0, 1])] * (2 * n_u)), indexing="ij")
    cand = np.stack([g.reshape(-1) for g in grids], axis=1)
    pert = u.astype(np.complex128)[None, :] + tau * (cand[:, :n_u] + 1j * cand[:, n_u:])
    x = pert @ W.T
    cost = (np.abs(x) ** 2).sum(axis=1)
    i = int(np.argmin(cost))
    return cand[i].astype(np.int8), float(cost[i])


def spin_ising(G: np.ndarray, f: np.ndarray, q: int, w: np.ndarray):
    """Expand the level-domain form into a dense spin Ising problem (paper §2.3).

    With x_k = sum_b w_b s_{k,b} and spin index i = k q + b:
      x^T G x - 2 f^T x = -sum_{i<j} J_ij s_i s_j - sum_i h_i s_i + const,
      J_ij = -2 w_i w_j G_{k(i)k(j)} (i != j), h_i = 2 w_i f_{k(i)},
      const = sum_i w_i^2 G_{k(i)k(i)}.
    Returns float64 (J [N][N] zero diagonal, h [N], const).
    """
    G = np.asarray(G, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    K = G.shape[-1]
    wv = np.tile(np.asarray(w, dtype=np.float64), K)
    kk = np.repeat(np.arange(K), q)
    J = -2.0 * wv[:, None] * wv[None, :] * G[kk][:, kk]
    np.fill_diagonal(J, 0.0)
    h = 2.0 * wv * f[kk]
    const = float((wv ** 2 * G[kk, kk]).sum())
    return J, h, const


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (ctypes.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def draw16(i, t, ch, inst, seed) -> int:
    return int(lib().oracle_draw16(i, t, ch, inst, int(seed) & 0xFFFFFFFFFFFFFFFF))


def accept(z: float, m: int) -> bool:
    return bool(lib().oracle_accept(z, m))


def accept_table() -> np.ndarray:
    """The Metropolis threshold table T[0..1024] (uint32)."""
    out = np.zeros(1025, dtype=np.uint32)
    lib().oracle_accept_table(_ptr(out))
    return out


def nthreads_env() -> int:
    v = os.environ.get("OMP_NUM_THREADS")
    return int(v) if v and v.isdigit() else 0
