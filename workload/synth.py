"""Seeded synthetic inputs for the MIMO detection / vector-perturbation workloads.

This module only *generates inputs*: channels, transmitted symbols, noise, the
received signal of the uplink model (paper §2.1, Eq. 1: y = Hx + noise) and the
annealing schedule tables that both the CPU oracle and the GPU library take as
arguments.  It holds none of the detection/precoding arithmetic (no Gram
matrices, no Ising reduction, no solver), so that the oracle and the GPU path
can both consume it without sharing any of the method's code.

Conventions (input side):

* Complex channels are i.i.d. CN(0, 1): real and imaginary parts N(0, 1/2).
* M-QAM with q = log2(M)/2 bits per real dimension.  A symbol index
  a in [0, M) splits into (aI, aQ) = (a >> q, a & (2^q - 1)); each half is a
  Gray label g whose binary position p = gray^-1(g) gives the PAM level
  2p - (2^q - 1).  The point is c * (lI + j*lQ) with c = sqrt(3 / (2(M-1))),
  i.e. unit average symbol energy.
* SNR is per receive antenna: sigma^2 = n_t / 10^(SNR/10) (unit-energy symbols,
  unit-variance channel taps).  The noise draw n0 ~ CN(0,1) is made once per
  seed, so SNR points share H, x and n0.
* Random draws use numpy's PCG64 in float64 and are cast to complex64 for the
  device boundary.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

QAM_ORDERS = (4, 16, 64)


def bits_per_dim(qam: int) -> int:
    q = int(round(math.log2(qam))) // 2
    if qam not in (4, 16, 64, 256) or (1 << (2 * q)) != qam:
        raise ValueError(f"unsupported QAM order {qam}")
    return q


def qam_scale(qam: int) -> float:
    """Amplitude c of the unit-energy square constellation (FP64)."""
    return 1.0 / math.sqrt(2.0 * (qam - 1) / 3.0)


def _gray_to_pos(g: np.ndarray) -> np.ndarray:
    p = g.copy()
    shift = g >> 1
    while np.any(shift):
        p ^= shift
        shift >>= 1
    return p


def symbol_levels(idx: np.ndarray, qam: int) -> tuple[np.ndarray, np.ndarray]:
    """Integer PAM levels (lI, lQ) of symbol indices (input-side labelling)."""
    q = bits_per_dim(qam)
    idx = np.asarray(idx, dtype=np.int64)
    gi = idx >> q
    gq = idx & ((1 << q) - 1)
    top = (1 << q) - 1
    li = 2 * _gray_to_pos(gi) - top
    lq = 2 * _gray_to_pos(gq) - top
    return li, lq


def symbol_points(idx: np.ndarray, qam: int) -> np.ndarray:
    """Complex constellation points (complex128) of symbol indices."""
    li, lq = symbol_levels(idx, qam)
    return qam_scale(qam) * (li + 1j * lq)


def rayleigh(rng: np.random.Generator, shape) -> np.ndarray:
    """i.i.d. CN(0,1) draws, complex128."""
    s = math.sqrt(0.5)
    return s * rng.standard_normal(shape) + 1j * s * rng.standard_normal(shape)


def noise_var(snr_db: float, n_t: int) -> float:
    """Per-receive-antenna noise variance for unit-energy symbols."""
    return n_t / (10.0 ** (snr_db / 10.0))


@dataclass
class DetSlot:
    H: np.ndarray        # complex64 [n_sc][n_r][n_t]
    y: np.ndarray        # complex64 [n_sc][n_sym][n_r]
    sym: np.ndarray      # uint8 [n_sc][n_sym][n_t] transmitted symbol indices
    noise_var: float     # sigma^2 per complex receive sample
    qam: int
    snr_db: float


def det_slot(seed: int, n_r: int, n_t: int, qam: int, n_sc: int, n_sym: int,
             snr_db: float) -> DetSlot:
    """One uplink slot: H held per subcarrier for n_sym symbols, y = Hx + n."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H = rayleigh(rng, (n_sc, n_r, n_t))
    sym = rng.integers(0, qam, size=(n_sc, n_sym, n_t))
    n0 = rayleigh(rng, (n_sc, n_sym, n_r))
    H64 = H.astype(np.complex64)
    x = symbol_points(sym, qam)
    s2 = noise_var(snr_db, n_t)
    # received signal from the complex64 channel that the detector will see
    y = np.einsum("srt,sbt->sbr", H64.astype(np.complex128), x) + math.sqrt(s2) * n0
    return DetSlot(H=H64, y=y.astype(np.complex64), sym=sym.astype(np.uint8),
                   noise_var=s2, qam=qam, snr_db=snr_db)


@dataclass
class VppSlot:
    H: np.ndarray        # complex64 [n_sc][n_u][n_t]  (users x transmit antennas)
    u: np.ndarray        # complex64 [n_sc][n_sym][n_u]
    sym: np.ndarray      # uint8 [n_sc][n_sym][n_u]
    qam: int


def vpp_slot(seed: int, n_u: int, n_t: int, qam: int, n_sc: int, n_sym: int) -> VppSlot:
    """One downlink slot: channel and the users' intended symbols."""
    rng = np.random.Generator(np.random.PCG64(seed))
    H = rayleigh(rng, (n_sc, n_u, n_t))
    sym = rng.integers(0, qam, size=(n_sc, n_sym, n_u))
    u = symbol_points(sym, qam)
    return VppSlot(H=H.astype(np.complex64), u=u.astype(np.complex64),
                   sym=sym.astype(np.uint8), qam=qam)


def random_structured_ising(seed: int, n_G: int, inst_per_G: int, K: int):
    """Random symmetric couplings G [n_G][K][K] and fields f [n_G*inst_per_G][K]
    (float32), drawn as the Gram matrix / matched filter of a random real
    matrix so that they have the statistics of a channel problem."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = rng.standard_normal((n_G, K, K)) / math.sqrt(K)
    G = np.einsum("gik,gil->gkl", A, A)
    f = rng.standard_normal((n_G * inst_per_G, K))
    return G.astype(np.float32), f.astype(np.float32)


def random_dense_ising(seed: int, n_inst: int, n: int):
    """Random dense spin-glass couplings J (symmetric, zero diagonal) and fields h."""
    rng = np.random.Generator(np.random.PCG64(seed))
    J = rng.standard_normal((n_inst, n, n))
    J = (J + np.transpose(J, (0, 2, 1))) / 2
    for i in range(n):
        J[:, i, i] = 0.0
    h = rng.standard_normal((n_inst, n))
    return J.astype(np.float32), h.astype(np.float32)


def linear_beta2(sweeps: int, beta0: float, beta1: float) -> np.ndarray:
    """Linear-in-beta annealing table, stored as beta_t * log2(e) in float32.

    beta_t = beta0 + (beta1 - beta0) * t / (S - 1) for t = 0..S-1 (a single
    sweep uses beta1).  The factor log2(e) lets acceptance use 2^(-z).
    """
    if sweeps <= 0:
        raise ValueError("sweeps must be positive")
    if sweeps == 1:
        b = np.array([beta1], dtype=np.float64)
    else:
        t = np.arange(sweeps, dtype=np.float64)
        b = beta0 + (beta1 - beta0) * t / (sweeps - 1)
    return (b * (1.0 / math.log(2.0))).astype(np.float32)


def det_beta_range(qam: int, n_r: int, noise_var_: float) -> tuple[float, float]:
    """Default inverse-temperature endpoints for detection problems.

    beta0 makes the typical cheapest uphill move (one least-significant level
    step, energy about 4 c^2 n_r) accepted with probability e^-1; beta1 = 1/sigma^2
    ends the anneal at the temperature whose Boltzmann weight exp(-beta ||y-Hx||^2)
    is the posterior of the Gaussian channel.
    """
    c2 = 1.0 / (2.0 * (qam - 1) / 3.0)
    beta0 = 1.0 / (4.0 * c2 * n_r)
    beta1 = 1.0 / max(noise_var_, 1e-6)
    return beta0, max(beta1, beta0)


def vpp_beta_range(qam: int, n_t: int) -> tuple[float, float]:
    """Default inverse-temperature endpoints for VPP problems, in units of the
    perturbation step energy (tau/2)^2 = M c^2."""
    c2 = 1.0 / (2.0 * (qam - 1) / 3.0)
    step = qam * c2                             # (tau/2)^2 with tau = 2 sqrt(M) c
    return 0.1 / step, 4.0 / step


def job_seed(job_id: int) -> int:
    """64-bit Philox key of a job."""
    return (0x4D4D4741_50000000 + int(job_id)) & 0xFFFFFFFFFFFFFFFF
