"""Multiscale Robin Coupled Method (Section 3).

Test infrastructure only (see the package header).

Steps, in the paper's order:

1. Local problems (eq:mrc1) on each subdomain Omega_i with the physical boundary data on
   dOmega_i cap dOmega and the Robin condition -beta_i u.n^i + p = -beta_i U_H n.n^i + P_H
   on dOmega_i cap Gamma, beta_i = alpha H / kappa_i (eq:beta).
2. Additive split (eq:mrc_homogeneous, eq:mrc_non_homogeneous): one homogeneous basis
   function per interface degree of freedom (unit coefficient, zero source and zero physical
   data) and one non-homogeneous basis function (zero Robin datum, the source and the
   physical data).
3. Interface system (eq:mrc2), one flux equation tested with each pressure function and one
   Robin equation tested with each flux function, for the coefficients U_l, P_l of the
   expansions of U_H and P_H.
4. Reconstruction of the local solutions from the basis functions.

Interface spaces (Section 3.1, and the intermediate length H-bar of Section 5.1): each side
of each subdomain that lies on Gamma is split into n_e equal elements, and U_H, P_H are
piecewise constant on those elements (k_U = k_P = 1 per element), or, with iface_degree = 1,
piecewise linear (k_U = k_P = 2: the -POL spaces of Section 5.2), with the basis 1 and xi on
each element, xi in [-1, 1] along the global direction of the interface, projected onto the
fine faces by their midpoint values (the face average of a linear function). Per element the
unknowns are U_0 .. U_{k-1} then P_0 .. P_{k-1}; the flux equations are tested with each
pressure function and the Robin equations with each flux function (eq:mrc2). The global orientation of
the skeleton is n-check = +x on vertical interfaces and +y on horizontal ones, so n-check .
n-check^i = +1 for the subdomain on the left or below and -1 for the other one.
Physical-boundary sides carry their physical condition and no interface unknown.
H in beta is the subdomain length normal to the interface; kappa_i at a face is that of the
adjacent cell of Omega_i.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fine import (DIR, NEU, ROB, W, E, S, N, Side, block_fluxes, block_matrix, block_rhs,
                   physical_sides, side_cells, side_geometry)


class Decomposition:
    """Non-overlapping decomposition of the grid into equal rectangular subdomains."""

    def __init__(self, cfg):
        self.cfg = cfg
        self.nx, self.ny = cfg["nx"], cfg["ny"]
        self.mx, self.my = cfg["sub_x"], cfg["sub_y"]
        self.ne_x, self.ne_y = cfg["ne_x"], cfg["ne_y"]
        assert self.nx % self.mx == 0 and self.ny % self.my == 0
        assert self.mx % self.ne_x == 0 and self.my % self.ne_y == 0
        self.Sx, self.Sy = self.nx // self.mx, self.ny // self.my
        self.hx, self.hy = cfg["lx"] / self.nx, cfg["ly"] / self.ny
        self.n_vert = (self.Sx - 1) * self.Sy * self.ne_y
        self.n_horiz = self.Sx * (self.Sy - 1) * self.ne_x
        self.n_elem = self.n_vert + self.n_horiz
        self.npol = cfg.get("iface_degree", 0) + 1        # k_U = k_P
        assert self.npol == 1 or (self.mx // self.ne_x >= 2 and self.my // self.ne_y >= 2), \
            "a linear interface function needs at least two faces per element"
        self.n_dof = 2 * self.npol * self.n_elem

    def vert_elem(self, I, J, k):
        """Element k of the vertical interface between subdomains (I, J) and (I+1, J)."""
        return (J * (self.Sx - 1) + I) * self.ne_y + k

    def horiz_elem(self, I, J, k):
        """Element k of the horizontal interface between subdomains (I, J) and (I, J+1)."""
        return self.n_vert + (J * self.Sx + I) * self.ne_x + k

    def cells(self, I, J):
        return J * self.my, (J + 1) * self.my, I * self.mx, (I + 1) * self.mx

    def interface_sides(self, I, J):
        """Per side: None on the physical boundary, else (element of each face, n.n^i, H,
        values of the element's basis functions at each face, shape (npol, faces))."""
        res = [None, None, None, None]
        py, px = self.my // self.ne_y, self.mx // self.ne_x
        fy, fx = np.arange(self.my) // py, np.arange(self.mx) // px
        xiy = (2 * (np.arange(self.my) % py) + 1) / py - 1.0
        xix = (2 * (np.arange(self.mx) % px) + 1) / px - 1.0
        phy = np.stack([np.ones(self.my), xiy][:self.npol])
        phx = np.stack([np.ones(self.mx), xix][:self.npol])
        Hx, Hy = self.mx * self.hx, self.my * self.hy
        if I > 0:
            res[W] = (self.vert_elem(I - 1, J, fy), -1.0, Hx, phy)
        if I < self.Sx - 1:
            res[E] = (self.vert_elem(I, J, fy), +1.0, Hx, phy)
        if J > 0:
            res[S] = (self.horiz_elem(I, J - 1, fx), -1.0, Hy, phx)
        if J < self.Sy - 1:
            res[N] = (self.horiz_elem(I, J, fx), +1.0, Hy, phx)
        return res

    def u_dof(self, l, k):
        """Global index of the k-th flux unknown of element l (row of its Robin equation)."""
        return 2 * self.npol * l + k

    def p_dof(self, l, k):
        """Global index of the k-th pressure unknown of element l (row of its flux equation)."""
        return 2 * self.npol * l + self.npol + k

    def subdomains(self):
        for J in range(self.Sy):
            for I in range(self.Sx):
                yield I, J


@dataclass
class LocalBasis:
    """Basis functions of one subdomain for a fixed conductivity."""
    I: int
    J: int
    kap: np.ndarray                 # local conductivity (my, mx)
    iface: list                     # Decomposition.interface_sides(I, J)
    betas: list                     # per side: beta per face (zeros on physical sides)
    dofs: np.ndarray                # global interface unknowns, local order
    lu: object                      # factorisation of the local matrix
    # homogeneous basis functions, one per entry of ``dofs``
    p: np.ndarray = field(default=None)     # (ndof, my*mx)
    ux: np.ndarray = field(default=None)    # (ndof, my, mx+1)
    uy: np.ndarray = field(default=None)    # (ndof, my+1, mx)
    out: list = field(default=None)         # per side: (ndof, faces) outward flux


def robin_sides(dec: Decomposition, I, J, kap, phys: list, alpha: float):
    """Side descriptions of a local problem with zero Robin datum on Gamma."""
    iface = dec.interface_sides(I, J)
    sides, betas = [], []
    for sd in (W, E, S, N):
        if iface[sd] is None:
            sides.append(phys[sd])
            betas.append(np.zeros_like(phys[sd].datum))
        else:
            r, c = side_cells(dec.my, dec.mx, sd)
            H = iface[sd][2]
            beta = alpha * H / kap[r, c]
            sides.append(Side(np.full(len(r), ROB), beta, np.zeros(len(r))))
            betas.append(beta)
    return sides, betas, iface


def local_dofs(dec: Decomposition, iface):
    """Global interface unknowns touching a subdomain: per element, the U then the P ones."""
    dofs = []
    for sd in (W, E, S, N):
        if iface[sd] is None:
            continue
        for l in np.unique(iface[sd][0]):
            dofs += [dec.u_dof(l, k) for k in range(dec.npol)] + [dec.p_dof(l, k) for k in range(dec.npol)]
    return np.array(dofs, dtype=np.int64)


def homogeneous_data(sides, iface, dof: int, npol: int = 1):
    """Robin data of the homogeneous basis function of one interface unknown
    (eq:mrc_homogeneous with unit coefficient): r = -beta n.n^i phi_k on the faces of element l
    for U_{l,k}, r = psi_k for P_{l,k}, zero elsewhere; zero physical data."""
    l, j = dof // (2 * npol), dof % (2 * npol)
    is_p, k = j >= npol, j % npol
    out = []
    for sd in (W, E, S, N):
        s = sides[sd]
        datum = np.zeros_like(s.datum)
        if iface[sd] is not None:
            on = iface[sd][0] == l
            ph = iface[sd][3][k]
            datum = np.where(on, ph if is_p else -s.beta * iface[sd][1] * ph, 0.0)
        out.append(Side(s.kind, s.beta, datum))
    return out


def build_local_basis(dec: Decomposition, I, J, kap_global, alpha: float) -> LocalBasis:
    cfg = dec.cfg
    j0, j1, i0, i1 = dec.cells(I, J)
    kap = kap_global[j0:j1, i0:i1]
    phys = physical_sides(cfg, j0, j1, i0, i1)
    sides, betas, iface = robin_sides(dec, I, J, kap, phys, alpha)
    A = block_matrix(kap, dec.hx, dec.hy, sides)
    lu = spla.splu(A)
    dofs = local_dofs(dec, iface)
    zero_q = np.zeros_like(kap)
    if len(dofs):
        B = np.stack([block_rhs(kap, dec.hx, dec.hy, homogeneous_data(sides, iface, d, dec.npol), zero_q)
                      for d in dofs], axis=1)
        P = lu.solve(B).T
    else:
        P = np.zeros((0, kap.size))
    ux = np.zeros((len(dofs), dec.my, dec.mx + 1))
    uy = np.zeros((len(dofs), dec.my + 1, dec.mx))
    outs = [np.zeros((len(dofs), dec.my if sd in (W, E) else dec.mx)) for sd in (W, E, S, N)]
    for k, d in enumerate(dofs):
        hs = homogeneous_data(sides, iface, d, dec.npol)
        ux[k], uy[k], o = block_fluxes(kap, dec.hx, dec.hy, hs, P[k])
        for sd in (W, E, S, N):
            outs[sd][k] = o[sd]
    return LocalBasis(I, J, kap.copy(), iface, betas, dofs, lu, P, ux, uy, outs)


def nonhomogeneous_solve(dec: Decomposition, lb: LocalBasis, phys: list, q_loc):
    """Non-homogeneous basis function (eq:mrc_non_homogeneous): zero Robin datum on Gamma,
    the given physical data on the other sides and the given source.

    Returns (p, ux, uy, out)."""
    sides = []
    for sd in (W, E, S, N):
        if lb.iface[sd] is None:
            sides.append(phys[sd])
        else:
            n = len(lb.betas[sd])
            sides.append(Side(np.full(n, ROB), lb.betas[sd], np.zeros(n)))
    b = block_rhs(lb.kap, dec.hx, dec.hy, sides, q_loc)
    p = lb.lu.solve(b)
    ux, uy, out = block_fluxes(lb.kap, dec.hx, dec.hy, sides, p)
    return p, ux, uy, out


def interface_rows(dec: Decomposition, lb: LocalBasis, out_sides, dim_cols):
    """Contributions of one subdomain's traces to the interface equations (eq:mrc2).

    For every element l on the subdomain's interface sides and every basis function k:
      flux equation   F_{l,k} += sum_{f in l} |f| u_f psi_k(f)
      Robin equation  G_{l,k} += (n.n^i) sum_{f in l} |f| beta_f u_f phi_k(f)
    ``out_sides[sd]`` has shape (ncols, faces). Row u_dof(l, k) holds G_{l,k}, row p_dof(l, k)
    holds F_{l,k}. Returns a list of (row, col, value) arrays.
    """
    rows, cols, vals = [], [], []
    for sd in (W, E, S, N):
        if lb.iface[sd] is None:
            continue
        elem, s, _, ph = lb.iface[sd]
        _, flen = side_geometry(dec.hx, dec.hy, sd)
        u = out_sides[sd]                           # (ncols, faces)
        ncols = u.shape[0]
        for l in np.unique(elem):
            on = elem == l
            for k in range(dec.npol):
                F = flen * (u[:, on] * ph[k][on]).sum(axis=1)
                G = s * flen * (u[:, on] * lb.betas[sd][on] * ph[k][on]).sum(axis=1)
                rows += [np.full(ncols, dec.p_dof(l, k)), np.full(ncols, dec.u_dof(l, k))]
                cols += [dim_cols, dim_cols]
                vals += [F, G]
    return rows, cols, vals


def robin_diagonal(dec: Decomposition, lb: LocalBasis):
    """The -sum_{f in l} |f| beta_f U_H(f) phi_k(f) term of G_{l,k} contributed by one side
    (eq:mrc2): coefficient -sum_f |f| beta_f phi_k phi_k' of U_{l,k'}."""
    rows, cols, vals = [], [], []
    for sd in (W, E, S, N):
        if lb.iface[sd] is None:
            continue
        elem, s, _, ph = lb.iface[sd]
        _, flen = side_geometry(dec.hx, dec.hy, sd)
        for l in np.unique(elem):
            on = elem == l
            for k in range(dec.npol):
                for k2 in range(dec.npol):
                    rows.append(np.array([dec.u_dof(l, k)]))
                    cols.append(np.array([dec.u_dof(l, k2)]))
                    vals.append(np.array([-flen * (lb.betas[sd][on] * ph[k][on] * ph[k2][on]).sum()]))
    return rows, cols, vals


@dataclass
class MRCMBasis:
    """Everything the MRCM computes for one conductivity and MPM-2P reuses (Algorithm 1:
    "store the set of BFs")."""
    dec: Decomposition
    kappa: np.ndarray
    locals: list
    M: sp.csc_matrix           # interface matrix, rows u_dof = G, p_dof = F
    lu: object


def build_basis(cfg, kappa) -> MRCMBasis:
    dec = Decomposition(cfg)
    alpha = cfg["alpha"]
    locs = [build_local_basis(dec, I, J, kappa, alpha) for I, J in dec.subdomains()]
    nd = dec.n_dof
    rows, cols, vals = [], [], []
    for lb in locs:
        r, c, v = interface_rows(dec, lb, lb.out, lb.dofs)
        rows += r; cols += c; vals += v
        r, c, v = robin_diagonal(dec, lb)
        rows += r; cols += c; vals += v
    if nd:
        M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(nd, nd)).tocsc()
        lu = spla.splu(M)
    else:
        M, lu = sp.csc_matrix((0, 0)), None
    return MRCMBasis(dec, kappa.copy(), locs, M, lu)


@dataclass
class MRCMSolution:
    y: np.ndarray              # interface unknowns, (U_l, P_l) interleaved
    p: list                    # per subdomain local pressure (my*mx)
    ux: list                   # per subdomain local x-fluxes (my, mx+1)
    uy: list
    out: list                  # per subdomain, per side outward fluxes
    rhs: np.ndarray            # interface right-hand side


def interface_solve(basis: MRCMBasis, rhs):
    """The solution of the interface system (eq:mrc2) to working precision: the sparse LU solve,
    then two steps of iterative refinement with the residual of the assembled matrix in FP64,
    y <- y + LU^-1 (rhs - M y). (With high-contrast conductivity the system is ill-conditioned:
    on the 129,024 unknowns of the 1024^2 workload the LU solve alone leaves a relative residual
    of ~2e-11 and errors up to ~2e-9 of the largest unknown; after one step the residual is ~1e-12
    and the next correction ~3e-13.)"""
    y = basis.lu.solve(rhs)
    for _ in range(2):
        y = y + basis.lu.solve(rhs - basis.M @ y)
    return y


def solve_with_basis(basis: MRCMBasis, phys_of, q_of) -> MRCMSolution:
    """Solve the non-homogeneous local problems, the interface system with the stored
    factorisation, and reconstruct every local solution (Section 3, last paragraph).

    ``phys_of(I, J)`` gives the physical side data of a subdomain; ``q_of(I, J)`` its source.
    """
    dec = basis.dec
    nd = dec.n_dof
    nh = []
    c = np.zeros(nd)
    for lb in basis.locals:
        p0, ux0, uy0, out0 = nonhomogeneous_solve(dec, lb, phys_of(lb.I, lb.J), q_of(lb.I, lb.J))
        nh.append((p0, ux0, uy0, out0))
        r, _, v = interface_rows(dec, lb, [o[None, :] for o in out0], np.zeros(1, dtype=int))
        for rr, vv in zip(r, v):
            np.add.at(c, rr, vv)
    y = interface_solve(basis, -c) if nd else np.zeros(0)
    ps, uxs, uys, outs = [], [], [], []
    for lb, (p0, ux0, uy0, out0) in zip(basis.locals, nh):
        coef = y[lb.dofs]
        ps.append(p0 + coef @ lb.p)
        uxs.append(ux0 + np.tensordot(coef, lb.ux, axes=1))
        uys.append(uy0 + np.tensordot(coef, lb.uy, axes=1))
        outs.append([out0[sd] + coef @ lb.out[sd] for sd in (W, E, S, N)])
    return MRCMSolution(y, ps, uxs, uys, outs, -c)


def physical_data(cfg):
    dec = Decomposition(cfg)

    def phys_of(I, J):
        return physical_sides(cfg, *dec.cells(I, J))
    return phys_of


def average_on_skeleton(dec: Decomposition, uxs, uys):
    """Global face fluxes from local ones: the arithmetic mean of the two sides' fluxes on
    Gamma (global orientation), the local flux elsewhere."""
    ux = np.zeros((dec.ny, dec.nx + 1))
    uy = np.zeros((dec.ny + 1, dec.nx))
    cx = np.zeros_like(ux)
    cy = np.zeros_like(uy)
    for k, (I, J) in enumerate(dec.subdomains()):
        j0, j1, i0, i1 = dec.cells(I, J)
        ux[j0:j1, i0:i1 + 1] += uxs[k]
        cx[j0:j1, i0:i1 + 1] += 1.0
        uy[j0:j1 + 1, i0:i1] += uys[k]
        cy[j0:j1 + 1, i0:i1] += 1.0
    return ux / cx, uy / cy
