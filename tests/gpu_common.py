"""Helpers shared by the GPU parity tests: run the HIP path and the oracle on the same seeded
inputs and compare them."""
import numpy as np

from oracle import physics, splitting

FP64_VEL_TOL = 1e-10     # relative L2 velocity error, FP64 path
FP64_SAT_TOL = 1e-9      # relative L1 saturation error, FP64 path
FP64_FACE_TOL = 1e-10    # largest face error over the largest face velocity, FP64 path


def vel_norm2(cfg, ux, uy):
    """RT0 norm with the trapezoidal rule: sum_c |c|/2 (u_W^2 + u_E^2 + u_S^2 + u_N^2)."""
    ny, nx = ux.shape[0], uy.shape[1]
    area = cfg["lx"] * cfg["ly"] / (nx * ny)
    return 0.5 * area * (np.sum(ux[:, :-1] ** 2) + np.sum(ux[:, 1:] ** 2) + np.sum(uy[:-1, :] ** 2) + np.sum(uy[1:, :] ** 2))


def vel_rel_err(cfg, ux, uy, rx, ry):
    return float(np.sqrt(vel_norm2(cfg, ux - rx, uy - ry) / vel_norm2(cfg, rx, ry)))


def vel_face_err(ux, uy, rx, ry):
    """Face by face: the largest error of a normal flux over the largest normal flux."""
    scale = max(float(np.abs(rx).max()), float(np.abs(ry).max()), 1e-300)
    return max(float(np.abs(ux - rx).max()), float(np.abs(uy - ry).max())) / scale


def sat_rel_err(s, r):
    den = np.abs(r).sum()
    return float(np.abs(s - r).sum() / den) if den > 0 else float(np.abs(s - r).sum())


def to_np(t):
    return t.detach().cpu().numpy()
