"""Stored oracle values at the metric workload: 1024^2 cells, 64 x 64 subdomains of 16^2, 8 interface
elements per side, log-normal K (log-variance 4, correlation length 0.05, seed 3), M = 100.

The FP64 oracle runs Algorithm 1 (Section 4.2) from s^0 = 0: the start (conductivity, MRCM basis,
interface solve of eq:mrc2, downscaling), two passes whose velocity update is MPM-2P (eq:mpm_tf_3
and eq. mpm_upd with the stored basis) and one pass whose update computes a new MRCM basis, each
pass one upwind transport sub-step (C_n = 1) first. After the start and after every pass it keeps

* the scalars: switch criterion epsilon, transport time step, outflow water cut, PVI, time;
* the velocity and the saturation of sampled subdomain tiles, face by face and cell by cell (the
  corners, the middle of each side, the subdomains around the two central separators of the
  decomposition, the quarter lines and a seeded draw);
* 256 Gaussian projections of the whole velocity, weighted so that the Euclidean norm of a
  projection estimates the RT0-trapezoidal norm, and 256 of the whole saturation; the projection
  vectors are regenerated from their seeds (``projections``), so a comparison estimates the
  error of every face and every cell;
* the exact RT0 norm of the velocity and the L2 norm of the saturation, and the largest face
  velocity.

The values are written by ``python -m tests.golden.c3_reference`` (about seven minutes on one
core), which calls only ``oracle/`` and the input generators; they are test data and nothing in
the library reads them.
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
PATH = os.path.join(HERE, "c3_reference.npz")
N_PROJ = 256
PROJ_SEED = 20210311
PASSES = ("mpm", "mpm", "mrcm")   # the branch of each pass after the start


def tiles():
    """(I, J) of the sampled subdomains of the 64 x 64 decomposition."""
    fixed = [(0, 0), (63, 0), (0, 63), (63, 63), (31, 0), (0, 32), (63, 31), (32, 63),
             (31, 31), (32, 31), (31, 32), (32, 32), (31, 10), (32, 50), (10, 31), (50, 32),
             (15, 15), (16, 16), (47, 47), (48, 16), (16, 48), (15, 47)]
    rng = np.random.default_rng(7)
    extra = [tuple(int(v) for v in rng.integers(1, 63, 2)) for _ in range(10)]
    return fixed + [t for t in extra if t not in fixed]


def velocity_weights(nx, ny, lx, ly):
    """Square roots of the face weights of the RT0-trapezoidal norm sum_c |c|/2 (u_W^2 + u_E^2 +
    u_S^2 + u_N^2): |c| on interior faces, |c|/2 on boundary faces."""
    area = lx * ly / (nx * ny)
    wx = np.full((ny, nx + 1), area)
    wx[:, 0] = wx[:, -1] = 0.5 * area
    wy = np.full((ny + 1, nx), area)
    wy[0, :] = wy[-1, :] = 0.5 * area
    return np.sqrt(wx), np.sqrt(wy)


def projections(*vecs):
    """The N_PROJ Gaussian projections of each of the given flat vectors of one length, each
    scaled by 1/sqrt(N_PROJ) so that the Euclidean norm of the result estimates that of the
    vector (for a fixed error vector the squared estimate over the squared norm is chi-square
    with N_PROJ degrees of freedom over N_PROJ: with 256 the estimate lies between 0.7 and 1.3
    times the norm except with probability 3.3e-11). One array of shape (len(vecs), N_PROJ)."""
    out = np.empty((len(vecs), N_PROJ))
    for k in range(N_PROJ):
        w = np.random.default_rng([PROJ_SEED, k]).standard_normal(vecs[0].size)
        for i, v in enumerate(vecs):
            out[i, k] = float(w @ v)
    return out / np.sqrt(N_PROJ)


def velocity_vector(cfg, ux, uy):
    sx, sy = velocity_weights(cfg["nx"], cfg["ny"], cfg["lx"], cfg["ly"])
    return np.concatenate([(sx * ux).ravel(), (sy * uy).ravel()])


def tile_fields(cfg, ux, uy, s):
    m = cfg["sub_x"]
    tx, ty, ts = [], [], []
    for I, J in tiles():
        j0, i0 = J * m, I * m
        tx.append(ux[j0:j0 + m, i0:i0 + m + 1])
        ty.append(uy[j0:j0 + m + 1, i0:i0 + m])
        ts.append(s[j0:j0 + m, i0:i0 + m])
    return np.array(tx), np.array(ty), np.array(ts)


def snapshot(cfg, run):
    ux, uy, s = run.ux, run.uy, run.s
    v = velocity_vector(cfg, ux, uy)
    area = cfg["lx"] * cfg["ly"] / (cfg["nx"] * cfg["ny"])
    sv = np.sqrt(area) * s.ravel()
    tx, ty, ts = tile_fields(cfg, ux, uy, s)
    return dict(eps=run.eps, dt=run.dt, wcut=run.wcut, pvi=run.pvi, t=run.t,
                umax=max(float(np.abs(ux).max()), float(np.abs(uy).max())),
                unorm=float(np.linalg.norm(v)), snorm=float(np.linalg.norm(sv)),
                uproj=projections(v)[0], sproj=projections(sv)[0], ux=tx, uy=ty, s=ts)


def generate(path=PATH):
    sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
    from oracle import splitting
    from paper_2103_11050_amd import inputs
    cfg = inputs.config("c3")
    K = inputs.permeability(cfg)
    s0 = inputs.initial_saturation(cfg)
    run = splitting.start(cfg, K, s0)
    snaps = [snapshot(cfg, run)]
    print("start done", flush=True)
    for b in PASSES:
        splitting.step(run, b)
        snaps.append(snapshot(cfg, run))
        print(f"pass {len(snaps) - 1} ({b}) done: eps {run.eps:.6e} dt {run.dt:.6e}", flush=True)
    out = {key: np.array([sn[key] for sn in snaps]) for key in snaps[0]}
    out["tiles"] = np.array(tiles())
    out["branches"] = np.array(["start", *PASSES])
    np.savez_compressed(path, **out)
    print(f"wrote {path}", flush=True)


def load(path=PATH):
    with np.load(path, allow_pickle=False) as z:
        return {k: z[k] for k in z.files}


if __name__ == "__main__":
    generate()
