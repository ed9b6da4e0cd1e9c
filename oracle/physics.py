"""Mobility, conductivity and fractional flow (Section 2; Corey curves of Section 5).

Test infrastructure only (see the package header).
"""
from __future__ import annotations

import numpy as np


def mobility(s, mu_w: float, mu_o: float):
    """Total mobility lambda(s) = k_rw/mu_w + k_ro/mu_o with k_rw = s^2, k_ro = (1-s)^2."""
    s = np.asarray(s, dtype=np.float64)
    return s * s / mu_w + (1.0 - s) * (1.0 - s) / mu_o


def conductivity(s, K, mu_w: float, mu_o: float):
    """kappa = lambda(s) K (Section 2; Algorithm 1 writes lambda(s) alone, read as lambda(s) K)."""
    return mobility(s, mu_w, mu_o) * np.asarray(K, dtype=np.float64)


def frac_flow(s, M: float):
    """f(s) = M s^2 / (M s^2 + (1-s)^2), M = mu_o / mu_w (Section 5)."""
    s = np.asarray(s, dtype=np.float64)
    a = M * s * s
    return a / (a + (1.0 - s) * (1.0 - s))


def frac_flow_deriv(s, M: float):
    """f'(s) = 2 M s (1-s) / (M s^2 + (1-s)^2)^2 (derivative of the Section 5 formula)."""
    s = np.asarray(s, dtype=np.float64)
    den = M * s * s + (1.0 - s) * (1.0 - s)
    return 2.0 * M * s * (1.0 - s) / (den * den)


def max_frac_flow_deriv(M: float) -> tuple[float, float]:
    """max over [0,1] of f'(s): a 10^6-interval scan, then golden-section refinement.

    Returns (f'_max, argmax).
    """
    s = np.linspace(0.0, 1.0, 1_000_001)
    d = frac_flow_deriv(s, M)
    k = int(np.argmax(d))
    a = s[max(k - 1, 0)]
    b = s[min(k + 1, len(s) - 1)]
    g = (np.sqrt(5.0) - 1.0) / 2.0
    c = b - g * (b - a)
    e = a + g * (b - a)
    fc = float(frac_flow_deriv(c, M))
    fe = float(frac_flow_deriv(e, M))
    for _ in range(200):
        if b - a < 1e-16:
            break
        if fc > fe:
            b, e, fe = e, c, fc
            c = b - g * (b - a)
            fc = float(frac_flow_deriv(c, M))
        else:
            a, c, fc = c, e, fe
            e = a + g * (b - a)
            fe = float(frac_flow_deriv(e, M))
    sm = 0.5 * (a + b)
    return float(max(frac_flow_deriv(sm, M), fc, fe, d[k])), float(sm)
