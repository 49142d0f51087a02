"""Writes acceptance_quality.json: per-instance results of the oracle's chain
contract (tabulated acceptance, float32 chains) and of its plain float64
Metropolis reference (exact acceptance from the same draws) on sampled
instances of three detection slots.  Calls only the oracle and the input
generator.  Run:  python tests/golden/make_acceptance_quality.py
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import oracle as O       # noqa: E402
from workload import synth as W      # noqa: E402

OUT = os.path.join(HERE, "acceptance_quality.json")
N_SC, N_SYM = 3276, 12
N_SAMPLE = 2016

# (name, n_r, n_t, qam, snr_db, chains, sweeps, init, slot seed)
CASES = [
    ("8x8-16qam-15dB-64x200-random", 8, 8, 16, 15.0, 64, 200, 0, 7101),
    ("8x8-16qam-15dB-64x50-fallback", 8, 8, 16, 15.0, 64, 50, 1, 7102),
    ("16x16-64qam-25dB-128x400-fallback", 16, 16, 64, 25.0, 128, 400, 1, 7201),
]


def case_inputs(case, n_sample=N_SAMPLE):
    name, n_r, n_t, qam, snr, chains, sweeps, init, seed = case
    d = W.det_slot(seed, n_r, n_t, qam, N_SC, N_SYM, snr)
    beta2 = W.linear_beta2(sweeps, *W.det_beta_range(qam, n_r, d.noise_var))
    ids = np.sort(np.random.default_rng(seed).choice(N_SC * N_SYM, n_sample, replace=False))
    return d, beta2, ids.astype(np.uint32)


def run_case(case, ids=None):
    """Per-instance symbol errors and float64 residuals ||y - Hx||^2 of both chains."""
    name, n_r, n_t, qam, snr, chains, sweeps, init, seed = case
    d, beta2, all_ids = case_inputs(case)
    ids = all_ids if ids is None else np.asarray(ids, dtype=np.uint32)
    truth = d.sym.reshape(-1, n_t)[ids]
    key = W.job_seed(seed)
    a = O.detect(d.H, d.y, d.noise_var, qam, chains, sweeps, beta2, key, inst_ids=ids,
                 init_mode=init)
    b = O.detect_exact(d.H, d.y, d.noise_var, qam, chains, sweeps, beta2, key, inst_ids=ids,
                       init_mode=init)
    return dict(ids=ids.tolist(),
                err_table=(a["sym"] != truth).sum(axis=1).tolist(),
                err_exact=(b["sym"] != truth).sum(axis=1).tolist(),
                res_table=[float(f"{v:.12g}") for v in a["metric"]],
                res_exact=[float(f"{v:.12g}") for v in b["metric"]])


def main():
    out = {"n_sc": N_SC, "n_sym": N_SYM, "cases": {}}
    for case in CASES:
        r = run_case(case)
        ea, eb = np.array(r["err_table"]), np.array(r["err_exact"])
        n_t = case[2]
        print(f"{case[0]}: SER table {ea.sum() / (ea.size * n_t):.5f} exact "
              f"{eb.sum() / (eb.size * n_t):.5f}; residual table {np.mean(r['res_table']):.5f} "
              f"exact {np.mean(r['res_exact']):.5f}", flush=True)
        out["cases"][case[0]] = dict(params=list(case[1:]), **r)
    with open(OUT, "w") as fh:
        json.dump(out, fh, separators=(",", ":"))


if __name__ == "__main__":
    main()
