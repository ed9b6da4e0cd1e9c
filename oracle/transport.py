"""Explicit saturation transport (Section 4: explicit Euler in time, first-order upwind in
space, velocity frozen over the transport sub-steps; eq. BL2D).

Test infrastructure only (see the package header).

Readings where the paper is silent:

* porosity is scaled out (Section 2), so the pore volume of a cell is |c|;
* the sub-step is dt = cfl * min_c |c| / (f'_max * sum of |f| u_f over the faces where the
  flux leaves c), recomputed after every velocity update (the monotonicity bound of the
  upwind step, cfl in (0, 1]);
* the upwind saturation on a boundary face with inflow (u.n < 0) is the injected s-bar;
* PVI grows by dt * (inflow through the boundary) / |Omega|;
* the water cut is sum |f| u_f f(s_c) / sum |f| u_f over boundary faces with outflow, and
  breakthrough is a water cut at or above the configured threshold.
"""
from __future__ import annotations

import numpy as np

from .physics import frac_flow, max_frac_flow_deriv


def _geometry(cfg, s):
    ny, nx = s.shape
    return cfg["lx"] / nx, cfg["ly"] / ny


def max_outflow_rate(cfg, ux, uy):
    """max over cells of (sum of |f| u_f over outflow faces) / |c|."""
    ny, nx = ux.shape[0], uy.shape[1]
    hx, hy = cfg["lx"] / nx, cfg["ly"] / ny
    out = (hy * (np.maximum(ux[:, 1:], 0.0) + np.maximum(-ux[:, :-1], 0.0))
           + hx * (np.maximum(uy[1:, :], 0.0) + np.maximum(-uy[:-1, :], 0.0)))
    return float(out.max()) / (hx * hy)


def time_step(cfg, ux, uy):
    M = cfg["mu_o"] / cfg["mu_w"]
    fmax, _ = max_frac_flow_deriv(M)
    rate = max_outflow_rate(cfg, ux, uy)
    return cfg["cfl"] / (fmax * rate)


def saturation_step(cfg, s, ux, uy, dt):
    """s <- s - dt/|c| sum_f |f| u_f f(s_upwind)."""
    M = cfg["mu_o"] / cfg["mu_w"]
    hx, hy = _geometry(cfg, s)
    s_inj = cfg["s_inj"]
    ny, nx = s.shape
    # upwind saturation on every x-face (+x orientation)
    sl = np.empty((ny, nx + 1))
    sr = np.empty((ny, nx + 1))
    sl[:, 1:] = s
    sr[:, :-1] = s
    sl[:, 0] = s_inj          # outside the W boundary
    sr[:, -1] = s_inj         # outside the E boundary
    supx = np.where(ux > 0.0, sl, sr)
    # y-faces
    sb = np.empty((ny + 1, nx))
    st = np.empty((ny + 1, nx))
    sb[1:, :] = s
    st[:-1, :] = s
    sb[0, :] = s_inj
    st[-1, :] = s_inj
    supy = np.where(uy > 0.0, sb, st)
    Fx = hy * ux * frac_flow(supx, M)
    Fy = hx * uy * frac_flow(supy, M)
    div = (Fx[:, 1:] - Fx[:, :-1]) + (Fy[1:, :] - Fy[:-1, :])
    return s - dt / (hx * hy) * div


def boundary_inflow(cfg, ux, uy):
    """Total inflow through the domain boundary (volume per unit time)."""
    ny, nx = ux.shape[0], uy.shape[1]
    hx, hy = cfg["lx"] / nx, cfg["ly"] / ny
    return float(hy * (np.maximum(ux[:, 0], 0).sum() + np.maximum(-ux[:, -1], 0).sum())
                 + hx * (np.maximum(uy[0, :], 0).sum() + np.maximum(-uy[-1, :], 0).sum()))


def water_cut(cfg, s, ux, uy):
    M = cfg["mu_o"] / cfg["mu_w"]
    ny, nx = s.shape
    hx, hy = cfg["lx"] / nx, cfg["ly"] / ny
    outs = [(hy * np.maximum(-ux[:, 0], 0), s[:, 0]), (hy * np.maximum(ux[:, -1], 0), s[:, -1]),
            (hx * np.maximum(-uy[0, :], 0), s[0, :]), (hx * np.maximum(uy[-1, :], 0), s[-1, :])]
    q = sum(float(w.sum()) for w, _ in outs)
    qw = sum(float((w * frac_flow(sc, M)).sum()) for w, sc in outs)
    return qw / q if q > 0 else 0.0
