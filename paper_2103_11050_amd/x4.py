"""The water-oil finger-growth experiment of Section 5 (last subsection) on the GPU path.

[0,3] x [0,1/2], 300 x 50 cells in 15 x 5 subdomains of 20 x 10, homogeneous K = 1, M = 4,
p = 0 / -1e4 on the left / right, no flow on the bottom and top, an initial water front with a
small perturbation at the channel centre. MRCM with one fine face per interface element
(H-bar = h) reproduces the undecomposed fine solution, so the reference is MRCM with a new basis
at every elliptic step; MPM-2P (Algorithm 1, eta = 1e-2, C_n = 1) reuses its basis until the
switch asks for a new one. Both take T_e elliptic steps (2000 in the paper); after every step
the relative L2(Omega) flux error and the relative L1(Omega) saturation error of MPM-2P against
the reference are taken. Reported: the errors at the reference's breakthrough and at the end,
their maxima, T_m and the relative cost reduction of Section 4.3.

    python -m paper_2103_11050_amd.x4 --steps 2000
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import binding, inputs
from .x1 import _norms, homogeneous_bf_count, rcr


def run_experiment(steps: int = 2000, eta: float = 1e-2, curves: bool = False) -> dict:
    import torch
    dev = torch.device("cuda:0")
    cfg = inputs.x4_config(eta=eta, steps=steps)
    Kt = torch.from_numpy(inputs.permeability(cfg)).to(dev)
    s0 = torch.from_numpy(inputs.initial_saturation(cfg)).to(dev)
    ref = binding.Run(cfg, Kt, s0)
    mpm = binding.Run(cfg, Kt, s0)
    ref.start()
    mpm.start()
    fe, se, bt_step = [], [], None
    for n in range(1, steps + 1):
        ref.step(binding.FORCE_MRCM)
        mpm.step()
        rux, ruy = (t.cpu().numpy() for t in ref.velocity())
        ux, uy = (t.cpu().numpy() for t in mpm.velocity())
        rs = ref.saturation().cpu().numpy()
        s = mpm.saturation().cpu().numpy()
        fe.append(float(np.sqrt(_norms(cfg, ux - rux, uy - ruy) / _norms(cfg, rux, ruy))))
        se.append(float(np.abs(s - rs).sum() / np.abs(rs).sum()))
        if bt_step is None and ref.stats()["breakthrough"]:
            bt_step = n
        if n % 250 == 0:
            print(f"[x4] step {n}: flux err {fe[-1]:.3e} sat err {se[-1]:.3e} T_m {mpm.stats()['tm']}",
                  file=sys.stderr, flush=True)
    st, rst = mpm.stats(), ref.stats()
    nsub = (cfg["nx"] // cfg["sub_x"]) * (cfg["ny"] // cfg["sub_y"])
    n_hat = homogeneous_bf_count(cfg)
    out = {"grid": [cfg["nx"], cfg["ny"]], "subdomains": nsub, "sub": [cfg["sub_x"], cfg["sub_y"]],
           "te": st["te"], "tm": st["tm"], "n_hat": n_hat, "rcr_percent": round(rcr(st["te"], st["tm"], nsub, n_hat), 2),
           "pvi_end": round(rst["pvi"], 4), "breakthrough_elliptic_step": bt_step,
           "flux_err_end": fe[-1], "sat_err_end": se[-1], "flux_err_max": max(fe), "sat_err_max": max(se)}
    if bt_step is not None:
        out["flux_err_at_breakthrough"] = fe[bt_step - 1]
        out["sat_err_at_breakthrough"] = se[bt_step - 1]
    if curves:
        out["flux_err"] = fe
        out["sat_err"] = se
    ref.close()
    mpm.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--eta", type=float, default=1e-2)
    args = ap.parse_args(argv)
    binding.load()
    print(json.dumps(run_experiment(args.steps, args.eta)), flush=True)


if __name__ == "__main__":
    sys.exit(main())
