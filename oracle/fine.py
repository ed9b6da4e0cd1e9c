"""Fine-scale elliptic solver on a rectangular block of cells.

Test infrastructure only (see the package header).

Discretisation (reading of Sections 2-3, where the paper says only "mixed finite elements"):
lowest-order Raviart-Thomas on rectangles with the trapezoidal rule for the velocity mass
matrix. Eliminating the velocities gives the cell-centred two-point flux system:

* half transmissibility of cell c towards face f: tau = 2 kappa_c / d, d the cell width
  normal to f;
* interior face: t = (1/tau_c + 1/tau_d)^-1 and the flux per unit length leaving c is
  u = t (p_c - p_d);
* Dirichlet face (p = g): t = tau_c, u = t (p_c - g);
* Robin face, -beta u.n + p = r (eq:mrc1, last line): the face pressure is p_f = r + beta u,
  so u = tau_c (p_c - p_f) gives t = (1/tau_c + beta)^-1 and u = t (p_c - r);
* Neumann face: u.n = z is prescribed;
* cell balance: sum over faces of |f| u_f = |c| q_c (eq. Darcy, second line).

Sides are ordered W, E, S, N. Faces along W/E run bottom to top, along S/N left to right.
Each side is described by per-face arrays ``kind`` (DIR, NEU, ROB), ``beta`` (ROB only) and
``datum`` (g for DIR, r for ROB, outward normal flux z for NEU).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

DIR, NEU, ROB = 0, 1, 2
W, E, S, N = 0, 1, 2, 3


@dataclass
class Side:
    kind: np.ndarray   # int per face
    beta: np.ndarray   # Robin coefficient per face (0 where unused)
    datum: np.ndarray  # g, r or z per face


def side_cells(my: int, mx: int, side: int):
    """(row, col) indices of the cells adjacent to the faces of one side, in face order."""
    if side == W:
        return np.arange(my), np.zeros(my, dtype=int)
    if side == E:
        return np.arange(my), np.full(my, mx - 1)
    if side == S:
        return np.zeros(mx, dtype=int), np.arange(mx)
    return np.full(mx, my - 1), np.arange(mx)


def side_geometry(hx: float, hy: float, side: int):
    """(cell width normal to the face, face length) for faces of a side."""
    return (hx, hy) if side in (W, E) else (hy, hx)


def boundary_trans(kind, kc, d, beta):
    """Transmissibility per unit length of boundary faces (0 on Neumann faces)."""
    tau = 2.0 * kc / d
    t = np.zeros_like(kc)
    t = np.where(kind == DIR, tau, t)
    t = np.where(kind == ROB, 1.0 / (1.0 / tau + beta), t)
    return t


def interior_trans(kap, hx, hy):
    """Harmonic transmissibilities per unit length of interior x- and y-faces."""
    tx = 1.0 / (hx / (2.0 * kap[:, :-1]) + hx / (2.0 * kap[:, 1:]))
    ty = 1.0 / (hy / (2.0 * kap[:-1, :]) + hy / (2.0 * kap[1:, :]))
    return tx, ty


def block_matrix(kap, hx, hy, sides, pin=None):
    """Sparse SPD matrix of the two-point flux system on a block (csc).

    ``pin`` = (row, col) replaces that cell's equation by p = 0 (used by the all-Neumann
    downscaling problems).
    """
    my, mx = kap.shape
    n = mx * my
    idx = np.arange(n).reshape(my, mx)
    diag = np.zeros((my, mx))
    rows, cols, vals = [], [], []
    tx, ty = interior_trans(kap, hx, hy)
    wx = hy * tx
    wy = hx * ty
    diag[:, :-1] += wx
    diag[:, 1:] += wx
    diag[:-1, :] += wy
    diag[1:, :] += wy
    for a, b, w in ((idx[:, :-1], idx[:, 1:], wx), (idx[:-1, :], idx[1:, :], wy)):
        rows += [a.ravel(), b.ravel()]
        cols += [b.ravel(), a.ravel()]
        vals += [-w.ravel(), -w.ravel()]
    for sd in (W, E, S, N):
        r, c = side_cells(my, mx, sd)
        d, flen = side_geometry(hx, hy, sd)
        t = boundary_trans(sides[sd].kind, kap[r, c], d, sides[sd].beta)
        np.add.at(diag, (r, c), flen * t)
    rows.append(idx.ravel())
    cols.append(idx.ravel())
    vals.append(diag.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    if pin is not None:
        k = idx[pin]
        A = A.tolil()
        A[k, :] = 0.0
        A[:, k] = 0.0
        A[k, k] = 1.0
        A = A.tocsr()
    return A.tocsc()


def block_rhs(kap, hx, hy, sides, q, pin=None):
    """Right-hand side: |c| q + sum_{DIR,ROB} |f| t datum - sum_{NEU} |f| z."""
    my, mx = kap.shape
    b = (hx * hy) * np.asarray(q, dtype=np.float64).reshape(my, mx).copy()
    for sd in (W, E, S, N):
        r, c = side_cells(my, mx, sd)
        d, flen = side_geometry(hx, hy, sd)
        s = sides[sd]
        t = boundary_trans(s.kind, kap[r, c], d, s.beta)
        contrib = np.where(s.kind == NEU, -flen * s.datum, flen * t * s.datum)
        np.add.at(b, (r, c), contrib)
    if pin is not None:
        b[pin] = 0.0
    return b.ravel()


def block_fluxes(kap, hx, hy, sides, p):
    """Fluxes per unit length from cell pressures.

    Returns (ux, uy, out) with ux of shape (my, mx+1) positive along +x, uy of shape
    (my+1, mx) positive along +y, and ``out[side]`` the outward fluxes on that side's faces.
    """
    my, mx = kap.shape
    p = p.reshape(my, mx)
    tx, ty = interior_trans(kap, hx, hy)
    ux = np.zeros((my, mx + 1))
    uy = np.zeros((my + 1, mx))
    ux[:, 1:-1] = tx * (p[:, :-1] - p[:, 1:])
    uy[1:-1, :] = ty * (p[:-1, :] - p[1:, :])
    out = []
    for sd in (W, E, S, N):
        r, c = side_cells(my, mx, sd)
        d, _ = side_geometry(hx, hy, sd)
        s = sides[sd]
        t = boundary_trans(s.kind, kap[r, c], d, s.beta)
        u = np.where(s.kind == NEU, s.datum, t * (p[r, c] - s.datum))
        out.append(u)
    ux[:, 0] = -out[W]
    ux[:, -1] = out[E]
    uy[0, :] = -out[S]
    uy[-1, :] = out[N]
    return ux, uy, out


def face_pressures(sides, out):
    """Face pressure on Robin faces, p_f = r + beta u (outward u); g on Dirichlet faces."""
    res = []
    for sd in (W, E, S, N):
        s = sides[sd]
        pf = np.where(s.kind == ROB, s.datum + s.beta * out[sd],
                      np.where(s.kind == DIR, s.datum, np.nan))
        res.append(pf)
    return res


def physical_sides(cfg, my0: int, my1: int, mx0: int, mx1: int):
    """Physical boundary conditions of the whole domain restricted to a block's sides.

    Only meaningful for sides that lie on the domain boundary.
    """
    out = []
    for sd, length in ((W, my1 - my0), (E, my1 - my0), (S, mx1 - mx0), (N, mx1 - mx0)):
        kind_code = cfg["bc_kind"][sd]
        val = float(cfg["bc_value"][sd])
        if kind_code == 1:      # pressure
            out.append(Side(np.full(length, DIR), np.zeros(length), np.full(length, val)))
        elif kind_code == 2:    # prescribed outward flux
            out.append(Side(np.full(length, NEU), np.zeros(length), np.full(length, val)))
        else:                   # no flow
            out.append(Side(np.full(length, NEU), np.zeros(length), np.zeros(length)))
    return out


def fine_solve(cfg, kappa, q=None):
    """Undecomposed fine-grid solve on the whole domain: (p, ux, uy)."""
    ny, nx = kappa.shape
    hx, hy = cfg["lx"] / nx, cfg["ly"] / ny
    if q is None:
        q = np.zeros_like(kappa)
    sides = physical_sides(cfg, 0, ny, 0, nx)
    A = block_matrix(kappa, hx, hy, sides)
    b = block_rhs(kappa, hx, hy, sides, q)
    p = spla.spsolve(A, b)
    ux, uy, _ = block_fluxes(kappa, hx, hy, sides, p)
    return p.reshape(ny, nx), ux, uy
