"""The Gaussian-field experiment of Section 5.1 on the GPU path.

64^2 cells in 4x4 subdomains of 16^2, p = 1 / 0 on the left / right, M = 40, K = 0.8 exp(delta xi)
with a self-similar field of contrast 1e3 or 1e6 (seeded, synthetic: the paper's sample is not
available). For each contrast and each C_n the runs are:

* the fine reference: MRCM with one fine face per interface element (H-bar = h), which is the
  undecomposed fine solution, recomputed at every elliptic step;
* MRCM with H-bar = H and H / 2, basis recomputed at every elliptic step;
* MPM-2P with H-bar = H and H / 2 (Algorithm 1, eta = 1e-2), and with --first-order also with
  the first-order term of eq:mpm_tf_4;
* with --linear, MRCM and MPM-2P with the -POL spaces of Section 5.2 (U_H, P_H linear per
  element) at H-bar = H and H / 2.

Every run takes its own CFL sub-steps, so the runs are compared at equal simulated time: after
each elliptic step of the reference (time T), every other run is stepped until its time reaches
T, and its velocity and saturation at T are interpolated linearly in time between its last two
steps; the relative L2(Omega) flux error and the relative L1(Omega) saturation error against the
reference are taken there. The runs stop at the reference's breakthrough (where each run's T_e
and T_m are read). Reported per run: the errors at breakthrough and their maxima, T_e, T_m and
the relative cost reduction of Section 4.3 RCR = (T_e - T_m) / T_e (1 - 2 N / (N-hat + 2 N)).

With --readings the MPM-2P runs at H / 2 are repeated under the other readings of the switch
(the absolute L2(Omega) norm of epsilon; epsilon of the current saturation, the description
before Algorithm 1); --cfl sets the fraction of the monotone time-step bound for every run
(the paper's T_e follows from a step the paper does not state).

    python -m paper_2103_11050_amd.x1 --contrast 1e3 --cn 1
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import binding, inputs


def rcr(te: int, tm: int, n_sub: int, n_hat: int) -> float:
    """Relative cost reduction of MPM-2P against MRCM (Section 4.3), in percent."""
    return 100.0 * (te - tm) / te * (1.0 - 2.0 * n_sub / (n_hat + 2.0 * n_sub))


def homogeneous_bf_count(cfg: dict) -> int:
    """N-hat: homogeneous basis functions over all subdomains, k_U + k_P per interface element
    side of every subdomain (flux and pressure functions), physical-boundary sides excluded."""
    sx, sy = cfg["nx"] // cfg["sub_x"], cfg["ny"] // cfg["sub_y"]
    vert = (sx - 1) * sy * cfg["ne_y"]        # elements on vertical interfaces
    horiz = sx * (sy - 1) * cfg["ne_x"]
    npol = cfg.get("iface_degree", 0) + 1
    return 2 * 2 * npol * (vert + horiz)      # two sides, 2 npol unknowns per element


def _norms(cfg, ux, uy):
    area = cfg["lx"] * cfg["ly"] / (cfg["nx"] * cfg["ny"])
    return 0.5 * area * (np.sum(ux[:, :-1] ** 2) + np.sum(ux[:, 1:] ** 2) + np.sum(uy[:-1, :] ** 2) +
                         np.sum(uy[1:, :] ** 2))


def _state(r):
    ux, uy = (t.cpu().numpy() for t in r.velocity())
    return r.stats()["t"], ux, uy, r.saturation().cpu().numpy()


def run_experiment(contrast: float, cn: int, max_steps: int = 20000, seed: int = 11, curves: bool = False,
                   first_order: bool = False, linear: bool = False, readings: bool = False,
                   cfl: float = 0.5) -> dict:
    import torch
    dev = torch.device("cuda:0")
    base = inputs.x1_config(contrast, ne=1, cn=cn, seed=seed)
    base["cfl"] = cfl
    K = inputs.permeability(base)
    Kt = torch.from_numpy(K).to(dev)
    s0 = torch.from_numpy(inputs.initial_saturation(base)).to(dev)
    cases = {
        "reference": (dict(ne_x=16, ne_y=16, eta=0.0), binding.FORCE_MRCM),
        "MRCM H": (dict(ne_x=1, ne_y=1, eta=0.0), binding.FORCE_MRCM),
        "MRCM H/2": (dict(ne_x=2, ne_y=2, eta=0.0), binding.FORCE_MRCM),
        "MPM-2P H": (dict(ne_x=1, ne_y=1, eta=1e-2), binding.AUTO),
        "MPM-2P H/2": (dict(ne_x=2, ne_y=2, eta=1e-2), binding.AUTO),
    }
    if first_order:   # with the first-order term of eq:mpm_tf_4, which the paper neglects
        cases["MPM-2P H, l=1"] = (dict(ne_x=1, ne_y=1, eta=1e-2, mpm_order=1), binding.AUTO)
        cases["MPM-2P H/2, l=1"] = (dict(ne_x=2, ne_y=2, eta=1e-2, mpm_order=1), binding.AUTO)
    if linear:        # the -POL spaces of Section 5.2
        cases["MRCM-POL H"] = (dict(ne_x=1, ne_y=1, eta=0.0, iface_degree=1), binding.FORCE_MRCM)
        cases["MRCM-POL H/2"] = (dict(ne_x=2, ne_y=2, eta=0.0, iface_degree=1), binding.FORCE_MRCM)
        cases["MPM-2P-POL H"] = (dict(ne_x=1, ne_y=1, eta=1e-2, iface_degree=1), binding.AUTO)
        cases["MPM-2P-POL H/2"] = (dict(ne_x=2, ne_y=2, eta=1e-2, iface_degree=1), binding.AUTO)
    if readings:      # the other readings of the switch criterion (Section 4.1, Algorithm 1)
        cases["MPM-2P H/2, abs eps"] = (dict(ne_x=2, ne_y=2, eta=1e-2, eps_norm="abs"), binding.AUTO)
        cases["MPM-2P H/2, text rule"] = (dict(ne_x=2, ne_y=2, eta=1e-2, switch_rule="text"), binding.AUTO)
    runs = {}
    for name, (over, force) in cases.items():
        cfg = dict(base, **over)
        r = binding.Run(cfg, Kt, s0)
        r.start()
        st = _state(r)
        runs[name] = [cfg, r, force, st, st]        # the last two states (time, ux, uy, s)
    err = {name: ([], []) for name in cases if name != "reference"}
    bt_step = None
    ref_cfg, ref, ref_force = runs["reference"][:3]
    for n in range(1, max_steps + 1):
        ref.step(ref_force)
        T, rux, ruy, rs = _state(ref)
        den_u = _norms(ref_cfg, rux, ruy)
        den_s = np.abs(rs).sum()
        for name, rec in runs.items():
            if name == "reference":
                continue
            cfg, r, force = rec[:3]
            while rec[4][0] < T:
                r.step(force)
                rec[3], rec[4] = rec[4], _state(r)
            (t0, ux0, uy0, s0_), (t1, ux1, uy1, s1_) = rec[3], rec[4]
            w = 1.0 if t1 <= t0 else (T - t0) / (t1 - t0)   # linear in time between the two steps
            ux, uy, s = (1 - w) * ux0 + w * ux1, (1 - w) * uy0 + w * uy1, (1 - w) * s0_ + w * s1_
            err[name][0].append(float(np.sqrt(_norms(cfg, ux - rux, uy - ruy) / den_u)))
            err[name][1].append(float(np.abs(s - rs).sum() / den_s) if den_s > 0 else 0.0)
        if ref.stats()["breakthrough"]:
            bt_step = n
            break
    ref_stats = ref.stats()
    out = {"contrast": contrast, "cn": cn, "cfl": cfl, "seed": seed, "kmax_over_kmin": float(K.max() / K.min()),
           "breakthrough_elliptic_step": bt_step, "breakthrough_pvi": round(ref_stats["pvi"], 4),
           "breakthrough_time": ref_stats["t"], "compared_at": "equal simulated time", "runs": {}}
    for name, (cfg, r, _, _, _) in runs.items():
        if name == "reference":
            continue
        st = r.stats()
        fe, se = err[name]
        rec = {"flux_err_at_breakthrough": fe[-1], "sat_err_at_breakthrough": se[-1],
               "flux_err_max": max(fe), "sat_err_max": max(se), "te": st["te"], "tm": st["tm"],
               "n_hat": homogeneous_bf_count(cfg)}
        if name.startswith("MPM"):
            nsub = (cfg["nx"] // cfg["sub_x"]) * (cfg["ny"] // cfg["sub_y"])
            rec["rcr_percent"] = round(rcr(st["te"], st["tm"], nsub, rec["n_hat"]), 2)
        if curves:
            rec["flux_err"] = fe
            rec["sat_err"] = se
        out["runs"][name] = rec
    for rec in runs.values():
        rec[1].close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--contrast", type=float, nargs="+", default=[1e3, 1e6])
    ap.add_argument("--cn", type=int, nargs="+", default=[1, 20])
    ap.add_argument("--max-steps", type=int, default=20000)
    ap.add_argument("--first-order", action="store_true", help="also MPM-2P with the first-order term")
    ap.add_argument("--linear", action="store_true", help="also MRCM and MPM-2P with linear interface spaces")
    ap.add_argument("--readings", action="store_true",
                    help="also MPM-2P at H/2 with the absolute epsilon norm and with the text switch rule")
    ap.add_argument("--cfl", type=float, default=0.5, help="fraction of the monotone time-step bound")
    args = ap.parse_args(argv)
    binding.load()
    for c in args.contrast:
        for cn in args.cn:
            print(json.dumps(run_experiment(c, cn, args.max_steps, first_order=args.first_order,
                                            linear=args.linear, readings=args.readings, cfl=args.cfl)), flush=True)


if __name__ == "__main__":
    sys.exit(main())
