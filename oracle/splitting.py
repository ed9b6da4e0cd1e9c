"""The modified operator splitting (Section 4.2, Algorithm 1).

Test infrastructure only (see the package header).

Steps: compute kappa^0 from s^0 and the velocity by MRCM, keep the basis functions, set
n = 1, l = 0 and epsilon = eta; then, while n < T_e: C_n transport sub-steps with the
velocity frozen; kappa^n from the new saturation; MRCM (and a new stored basis) if
epsilon > eta, else MPM-2P with the stored basis; epsilon = ||kappa^n - kappa^m||; n += 1.

Readings:

* kappa = lambda(s) K (the algorithm's first line omits K);
* epsilon is relative by default: ||kappa^n - kappa^m||_2 / ||kappa^m||_2 over cells (cells
  are equal, so |c| cancels); ``eps_norm = "abs"`` gives the absolute L2(Omega) norm;
* ``switch_rule = "alg1"`` is the algorithm as written (the decision at step n uses the
  epsilon of step n-1); ``"text"`` uses epsilon of the current saturation (the description
  before the algorithm: MRCM at the first time with epsilon > eta);
* T_m counts basis-set computations including the initial one (l + 1).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .mpm import mpm_velocity, mrcm_velocity
from .physics import conductivity
from .transport import boundary_inflow, saturation_step, time_step, water_cut


def eps_norm(cfg, kappa_n, kappa_m):
    d = kappa_n - kappa_m
    if cfg.get("eps_norm", "rel") == "abs":
        ny, nx = kappa_n.shape
        area = cfg["lx"] * cfg["ly"] / (nx * ny)
        return float(np.sqrt(area * np.sum(d * d)))
    return float(np.sqrt(np.sum(d * d)) / np.sqrt(np.sum(kappa_m * kappa_m)))


@dataclass
class Run:
    cfg: dict
    K: np.ndarray
    q: np.ndarray
    s: np.ndarray
    ux: np.ndarray = None
    uy: np.ndarray = None
    state: object = None
    eps: float = 0.0
    n: int = 0                 # elliptic solves done (T_e so far)
    ell: int = 0               # updates after the initial basis
    dt: float = 0.0
    t: float = 0.0
    pvi: float = 0.0
    wcut: float = 0.0
    history: list = field(default_factory=list)


def start(cfg, K, s0, q=None) -> Run:
    """Algorithm 1, first four lines."""
    q = np.zeros_like(K) if q is None else q
    run = Run(cfg, K.copy(), q, s0.copy())
    kappa = conductivity(run.s, K, cfg["mu_w"], cfg["mu_o"])
    run.ux, run.uy, run.state, _ = mrcm_velocity(cfg, kappa, q)
    run.n = 1
    run.ell = 0
    run.eps = cfg["eta"]
    run.dt = time_step(cfg, run.ux, run.uy)
    run.history.append(dict(n=0, branch="mrcm", eps=None))
    return run


def transport(run: Run, nsteps: int):
    cfg = run.cfg
    area = cfg["lx"] * cfg["ly"]
    qin = boundary_inflow(cfg, run.ux, run.uy)
    for _ in range(nsteps):
        run.s = saturation_step(cfg, run.s, run.ux, run.uy, run.dt)
        run.t += run.dt
        run.pvi += run.dt * qin / area
    run.wcut = water_cut(cfg, run.s, run.ux, run.uy)


def step(run: Run, force=None):
    """One pass of the while loop of Algorithm 1. ``force``: None (automatic), "mrcm" or
    "mpm" (used to replay a decision sequence)."""
    cfg = run.cfg
    transport(run, cfg["cn"])
    kappa_n = conductivity(run.s, run.K, cfg["mu_w"], cfg["mu_o"])
    if cfg.get("switch_rule", "alg1") == "text":
        decide = eps_norm(cfg, kappa_n, run.state.kappa_m)
    else:
        decide = run.eps
    branch = "mrcm" if decide > cfg["eta"] else "mpm"
    if force is not None:
        branch = force
    if branch == "mrcm":
        run.ell += 1
        run.ux, run.uy, run.state, _ = mrcm_velocity(cfg, kappa_n, run.q)
    else:
        run.ux, run.uy, _ = mpm_velocity(cfg, run.state, kappa_n, run.q, order=cfg.get("mpm_order", 0))
    run.eps = eps_norm(cfg, kappa_n, run.state.kappa_m)
    run.dt = time_step(cfg, run.ux, run.uy)
    run.history.append(dict(n=run.n, branch=branch, eps=run.eps, decide=decide))
    run.n += 1
    return branch


def simulate(cfg, K, s0, n_elliptic: int, q=None, stop_at_breakthrough=False, forced=None):
    """Run Algorithm 1 until ``n_elliptic`` elliptic solves (T_e) have been made."""
    run = start(cfg, K, s0, q)
    while run.n < n_elliptic:
        f = None if forced is None else forced[run.n]
        step(run, f)
        if stop_at_breakthrough and run.wcut >= cfg["breakthrough_cut"]:
            break
    return run
