"""Basis-function counts and the Relative Cost Reduction (Section 4.3).

Test infrastructure only (see the package header).

* MRCM computes 4 (k_U + k_P) homogeneous BFs per subdomain edge that lies on the skeleton
  plus one non-homogeneous BF per subdomain; N-hat is the total number of homogeneous BFs.
* cost(MRCM) ~ C_BF (N-hat + 2N) T_e; cost(MPM-2P) ~ C_BF (N-hat + 2N) T_m + 2 C_BF N (T_e - T_m).
* RCR = (T_e - T_m)/T_e * (1 - 2N/(N-hat + 2N)) * 100 %.
"""
from __future__ import annotations


def homogeneous_bf_count(Sx: int, Sy: int, ne_x: int, ne_y: int, kU: int = 1, kP: int = 1) -> int:
    """N-hat for an Sx x Sy decomposition with n_e interface elements per side.

    Every element of every interface carries kU + kP unknowns, and each unknown gives one
    homogeneous BF in each of the two subdomains that share the interface.
    """
    n_vert = (Sx - 1) * Sy * ne_y
    n_horiz = Sx * (Sy - 1) * ne_x
    return 2 * (kU + kP) * (n_vert + n_horiz)


def rcr(Te: int, Tm: int, N: int, Nhat: int) -> float:
    """Relative Cost Reduction in percent."""
    return (Te - Tm) / Te * (1.0 - 2.0 * N / (Nhat + 2.0 * N)) * 100.0
