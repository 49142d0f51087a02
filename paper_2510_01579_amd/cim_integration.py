"""The paper's integration study of the CIM-CAC dynamics (Appendix A) on the GPU.

For each step size dt and coupling refresh period f_mvm, every run integrates
the same random Ising instance from the same initial amplitudes over the same
length N_I * dt = 2.56 as the fine-step reference (dt = 0.01, f_mvm = 1,
N_I = 256), through ``Context.cim_chains`` (one anneal per instance).  Two
figures per setting:

* P_diverge: diverged runs / runs (a run diverges when an amplitude ends beyond
  1000 in magnitude or not finite, or an error variable ends not finite);
* P_error: final spins sign(x_i) sign(x_a) that differ from the reference's /
  spins, over the runs that diverged in neither.

Instances: dense random couplings J (symmetric, entries of variance 1/2, zero
diagonal) and fields h of unit variance on n spins, one spin per dimension
(q = 1), i.e. G = -J / 2, f = h / 2 in the level form x^T G x - 2 f^T x.

    python -m paper_2510_01579_amd.cim_integration [--instances 10000] [--spins 16]
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

REF = (0.01, 1)
LENGTH = 2.56
DTS = (0.01, 0.02, 0.04, 0.08, 0.16, 0.32)
FMVMS = (1, 2, 4, 8)


def instances(seed: int, n_inst: int, n_spins: int):
    """G [n][K][K] and f [n][K] (float32) of random dense Ising instances."""
    from workload import synth as W
    J, h = W.random_dense_ising(seed, n_inst, n_spins)
    return (-J / 2).astype(np.float32), (h / 2).astype(np.float32)


def metrics(ref_spins, ref_div, spins, div):
    ref_div = np.asarray(ref_div).astype(bool).reshape(-1)
    div = np.asarray(div).astype(bool).reshape(-1)
    n = np.asarray(spins).shape[-1]
    ok = ~ref_div & ~div
    a = np.asarray(ref_spins).reshape(-1, n)[ok]
    b = np.asarray(spins).reshape(-1, n)[ok]
    return dict(p_diverge=float(np.mean(div)),
                p_error=float(np.mean(a != b)) if a.size else None,
                compared=int(ok.sum()))


def run(ctx, n_inst=10000, n_spins=16, seed=11, anneal_seed=5, dts=DTS, fmvms=FMVMS, cim=None):
    """The (dt, f_mvm) grid.  Returns dict(reference, grid: list of rows)."""
    import torch
    G, f = instances(seed, n_inst, n_spins)
    dev = torch.device("cuda", ctx.device)
    Gd, fd = torch.from_numpy(G).to(dev), torch.from_numpy(f).to(dev)
    base = dict(cim or {})

    def one(dt, f_mvm):
        steps = max(1, int(round(LENGTH / dt)))
        s, _, d = ctx.cim_chains(Gd, fd, n_spins, 1, [1], 1, steps, anneal_seed,
                                 cim=dict(base, dt=dt, f_mvm=f_mvm))
        torch.cuda.synchronize()
        return steps, s.cpu().numpy(), d.cpu().numpy()

    _, rs, rd = one(*REF)
    rows = []
    for dt in dts:
        for fm in fmvms:
            steps, s, d = one(dt, fm)
            rows.append(dict(dt=dt, f_mvm=fm, steps=steps, **metrics(rs, rd, s, d)))
    return dict(reference=dict(dt=REF[0], f_mvm=REF[1], steps=int(round(LENGTH / REF[0])),
                               p_diverge=float(np.mean(rd))),
                instances=n_inst, spins=n_spins, grid=rows)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--instances", type=int, default=10000)
    ap.add_argument("--spins", type=int, default=16)
    ap.add_argument("--seed", type=int, default=11)
    args = ap.parse_args(argv)
    import paper_2510_01579_amd as M
    ctx = M.Context(0)
    res = run(ctx, args.instances, args.spins, args.seed)
    ctx.close()
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
