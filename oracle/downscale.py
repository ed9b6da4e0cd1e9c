"""Downscaling to a conservative fine velocity (Section 4.1, the local problems after
eq:soma_u, labelled mpm_upd).

Test infrastructure only (see the package header).

On every subdomain, an all-Neumann problem with conductivity kappa* is solved: the outward
flux on every face of dOmega_i is the given coarse-stage velocity u-bar, the source is q.
The problem is determined up to a constant; the pressure of the subdomain's first cell
(lowest row, then lowest column) is fixed to zero. Interior faces take the two-point flux of
the local pressure, boundary faces keep u-bar.

Such a problem has a solution only if the net outflow through dOmega_i equals the source.
The exact coarse-stage fluxes satisfy this, because each interface element carries the same
flux integral on both sides. In floating point the data miss it by a rounding-level defect;
with the first cell's equation dropped, that defect would all leave through the pinned
cell's faces. Instead, the defect divided by |Omega_i| is added to the source of every cell
before the pinned solve. The corrected data are compatible, and in exact arithmetic the
shift is zero.

The same downscaling is used after an MRCM solve (with kappa^m), where the paper cites a
downscaling method it does not describe.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .fine import NEU, W, E, S, N, Side, block_fluxes, block_matrix, block_rhs
from .mrcm import Decomposition


def boundary_outflux(dec: Decomposition, ux, uy, I, J):
    """Outward fluxes of a subdomain's boundary faces from global face arrays."""
    j0, j1, i0, i1 = dec.cells(I, J)
    return [-ux[j0:j1, i0], ux[j0:j1, i1], -uy[j0, i0:i1], uy[j1, i0:i1]]


def downscale(cfg, kappa_star, ux_bar, uy_bar, q=None):
    """Returns (ux, uy, defects); defects[i] = sum |f| w_f - sum |c| q_c on subdomain i (of the
    data, before the compatibility shift)."""
    dec = Decomposition(cfg)
    if q is None:
        q = np.zeros_like(kappa_star)
    ux = ux_bar.copy()
    uy = uy_bar.copy()
    defects = []
    for I, J in dec.subdomains():
        j0, j1, i0, i1 = dec.cells(I, J)
        kap = kappa_star[j0:j1, i0:i1]
        w = boundary_outflux(dec, ux_bar, uy_bar, I, J)
        sides = [Side(np.full(len(w[sd]), NEU), np.zeros(len(w[sd])), w[sd]) for sd in (W, E, S, N)]
        src = q[j0:j1, i0:i1]
        flux = dec.hy * (w[W].sum() + w[E].sum()) + dec.hx * (w[S].sum() + w[N].sum())
        defect = flux - dec.hx * dec.hy * src.sum()
        src = src + defect / (src.size * dec.hx * dec.hy)   # compatible data
        A = block_matrix(kap, dec.hx, dec.hy, sides, pin=(0, 0))
        b = block_rhs(kap, dec.hx, dec.hy, sides, src, pin=(0, 0))
        p = spla.spsolve(A, b)
        lux, luy, _ = block_fluxes(kap, dec.hx, dec.hy, sides, p)
        ux[j0:j1, i0 + 1:i1] = lux[:, 1:-1]
        uy[j0 + 1:j1, i0:i1] = luy[1:-1, :]
        defects.append(defect)
    return ux, uy, np.array(defects)
