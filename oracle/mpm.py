"""MRCM velocity update and the MPM-2P velocity update (Sections 3 and 4.1).

Test infrastructure only (see the package header).

MPM-2P (Section 4.1): with the basis functions of kappa^m kept, the velocity for kappa^n is
obtained from the zeroth-order problem eq:mpm_tf_3 solved by MRCM with kappa^m, i.e. one
non-homogeneous local solve per subdomain and one interface solve:

* source q + div(kappa^n grad p^m) and, on Neumann boundaries, flux z + kappa^n grad p^m . n;
  the discrete kappa^n grad p^m is -v with v_f = (t^n_f / t^m_f) u~^m_f, t the face
  transmissibility of the fine system (on boundary faces the ratio kappa^n_c / kappa^m_c of
  the adjacent cell), u~^m the conservative velocity of the last MRCM update;
* Dirichlet datum g - p^m = 0 (the data do not depend on time);
* u-bar = u^m + delta u^n = u-hat_0 + v on every subdomain's faces, then the mean of both
  sides on Gamma, then downscaling with kappa^n (eq. mpm_upd).

With order = 1 the first-order term of the expansion (eq:mpm_tf_4 with l = 1) is added before
the downscaling. With eps kappa_eps = kappa^n - kappa^m, the problem for u-hat_1 = -kappa^m
grad delta p_1 has source div((kappa^n - kappa^m) grad delta p_0) and zero data, and the
velocity correction is u-hat_1 - (kappa^n - kappa^m) grad delta p_0. Discretely (reading): the
flux w = (t^n / t^m - 1) u-hat_0 on every face (t^n / t^m the same ratio as for v; u-hat_0 the
local fluxes of the zeroth-order MRCM solution, the mean of both sides on Gamma; w = 0 on
Neumann faces, which carry no flux unknown), the first-order problem with source -div w,
Dirichlet and Neumann data 0 solved by MRCM with the same basis, and u-bar gains u-hat_1 + w.
With one fine face per interface element this is the second step of the Richardson iteration
delta p = A_m^-1 (b_n - A_n p^m), delta p_1 = -A_m^-1 (A_n - A_m) delta p_0.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .downscale import downscale
from .fine import DIR, NEU, W, E, S, N, Side, interior_trans, physical_sides
from .mrcm import Decomposition, MRCMBasis, average_on_skeleton, build_basis, physical_data, solve_with_basis


@dataclass
class VelocityState:
    """What the splitting keeps between elliptic solves."""
    basis: MRCMBasis           # BFs, local factorisations and interface factorisation of kappa^m
    kappa_m: np.ndarray
    ux_m: np.ndarray           # conservative velocity u~^m of the last MRCM update
    uy_m: np.ndarray


def _q_of(dec, q):
    def f(I, J):
        j0, j1, i0, i1 = dec.cells(I, J)
        return q[j0:j1, i0:i1]
    return f


def mrcm_velocity(cfg, kappa, q=None):
    """Full MRCM solve with new basis functions and downscaling with the same kappa.

    Returns (ux, uy, state, diagnostics)."""
    if q is None:
        q = np.zeros_like(kappa)
    basis = build_basis(cfg, kappa)
    dec = basis.dec
    sol = solve_with_basis(basis, physical_data(cfg), _q_of(dec, q))
    uxb, uyb = average_on_skeleton(dec, sol.ux, sol.uy)
    ux, uy, defects = downscale(cfg, kappa, uxb, uyb, q)
    state = VelocityState(basis, kappa.copy(), ux, uy)
    return ux, uy, state, dict(solution=sol, ux_bar=uxb, uy_bar=uyb, defects=defects)


def perturbation_flux(cfg, kappa_n, kappa_m, ux_m, uy_m):
    """Discrete -kappa^n grad p^m as face fluxes: v = (t^n / t^m) u~^m."""
    ny, nx = kappa_n.shape
    hx, hy = cfg["lx"] / nx, cfg["ly"] / ny
    tnx, tny = interior_trans(kappa_n, hx, hy)
    tmx, tmy = interior_trans(kappa_m, hx, hy)
    rx = np.empty((ny, nx + 1))
    ry = np.empty((ny + 1, nx))
    rx[:, 1:-1] = tnx / tmx
    rx[:, 0] = kappa_n[:, 0] / kappa_m[:, 0]
    rx[:, -1] = kappa_n[:, -1] / kappa_m[:, -1]
    ry[1:-1, :] = tny / tmy
    ry[0, :] = kappa_n[0, :] / kappa_m[0, :]
    ry[-1, :] = kappa_n[-1, :] / kappa_m[-1, :]
    return rx * ux_m, ry * uy_m


def flux_ratio(cfg, kappa_n, kappa_m):
    """t^n / t^m on every face (kappa^n / kappa^m of the adjacent cell on boundary faces)."""
    return perturbation_flux(cfg, kappa_n, kappa_m, np.ones((kappa_n.shape[0], kappa_n.shape[1] + 1)),
                             np.ones((kappa_n.shape[0] + 1, kappa_n.shape[1])))


def mpm_velocity(cfg, state: VelocityState, kappa_n, q=None, order=0):
    """One MPM-2P velocity update reusing ``state``'s basis functions; ``order`` 1 adds the
    first-order perturbation term.

    Returns (ux, uy, diagnostics)."""
    if q is None:
        q = np.zeros_like(kappa_n)
    basis = state.basis
    dec = basis.dec
    vx, vy = perturbation_flux(cfg, kappa_n, state.kappa_m, state.ux_m, state.uy_m)
    # source of eq:mpm_tf_3: q - div v, cell by cell
    div_v = (dec.hy * (vx[:, 1:] - vx[:, :-1]) + dec.hx * (vy[1:, :] - vy[:-1, :])) / (dec.hx * dec.hy)
    src = q - div_v

    def phys_of(I, J):
        j0, j1, i0, i1 = dec.cells(I, J)
        ph = physical_sides(cfg, j0, j1, i0, i1)
        vout = [-vx[j0:j1, i0], vx[j0:j1, i1], -vy[j0, i0:i1], vy[j1, i0:i1]]
        res = []
        for sd in (W, E, S, N):
            s = ph[sd]
            datum = np.where(s.kind == DIR, 0.0, s.datum - vout[sd])
            res.append(Side(s.kind, s.beta, datum))
        return res

    sol = solve_with_basis(basis, phys_of, _q_of(dec, src))
    uxs, uys = [], []
    for k, (I, J) in enumerate(dec.subdomains()):
        j0, j1, i0, i1 = dec.cells(I, J)
        uxs.append(sol.ux[k] + vx[j0:j1, i0:i1 + 1])
        uys.append(sol.uy[k] + vy[j0:j1 + 1, i0:i1])
    if order >= 1:
        # w = (t^n / t^m - 1) u-hat_0, 0 on Neumann faces
        u0x, u0y = average_on_skeleton(dec, sol.ux, sol.uy)
        rx, ry = flux_ratio(cfg, kappa_n, state.kappa_m)
        wx, wy = (rx - 1.0) * u0x, (ry - 1.0) * u0y
        sides = physical_sides(cfg, 0, dec.ny, 0, dec.nx)
        wx[:, 0] = np.where(sides[W].kind == NEU, 0.0, wx[:, 0])
        wx[:, -1] = np.where(sides[E].kind == NEU, 0.0, wx[:, -1])
        wy[0, :] = np.where(sides[S].kind == NEU, 0.0, wy[0, :])
        wy[-1, :] = np.where(sides[N].kind == NEU, 0.0, wy[-1, :])
        src1 = -(dec.hy * (wx[:, 1:] - wx[:, :-1]) + dec.hx * (wy[1:, :] - wy[:-1, :])) / (dec.hx * dec.hy)

        def phys_of1(I, J):
            ph = physical_sides(cfg, *dec.cells(I, J))
            return [Side(s.kind, s.beta, np.zeros_like(s.datum)) for s in ph]

        sol1 = solve_with_basis(basis, phys_of1, _q_of(dec, src1))
        for k, (I, J) in enumerate(dec.subdomains()):
            j0, j1, i0, i1 = dec.cells(I, J)
            uxs[k] = uxs[k] + sol1.ux[k] + wx[j0:j1, i0:i1 + 1]
            uys[k] = uys[k] + sol1.uy[k] + wy[j0:j1 + 1, i0:i1]
    uxb, uyb = average_on_skeleton(dec, uxs, uys)
    ux, uy, defects = downscale(cfg, kappa_n, uxb, uyb, q)
    return ux, uy, dict(solution=sol, ux_bar=uxb, uy_bar=uyb, defects=defects, vx=vx, vy=vy)
