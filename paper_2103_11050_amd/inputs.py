"""Seeded synthetic inputs shared by the HIP path, the oracle, the tests and the benchmark.

This module only produces input data (problem descriptions, permeability fields, initial
saturations). It holds none of the method's arithmetic: no mobility, no transmissibility,
no solver. Both the oracle and the HIP path consume what it returns.

Permeability: ln K = sigma * xi, where xi is a stationary zero-mean unit-variance Gaussian
field with covariance exp(-r^2 / (2 l^2)), sampled at cell centres by circulant embedding
on a periodic grid padded to twice the domain in each direction, driven by numpy's PCG64
with the given seed. This stands in for the log-normal fields of the paper's experiments
(Section 5); the paper's own samples are not available.
"""
from __future__ import annotations

import copy

import numpy as np

# boundary kinds per side, sides ordered W, E, S, N
NOFLOW, PRESSURE, FLUX = 0, 1, 2
SIDES = ("W", "E", "S", "N")

# Workloads. Sizes follow the configurations of the benchmark; physics follows the paper's
# model problem (Section 2) with quadratic Corey curves (Section 5).
_BASE = dict(
    lx=1.0, ly=1.0, alpha=1.0, eta=0.1, eps_norm="rel", switch_rule="alg1",
    mu_w=1.0, mu_o=10.0,
    # water injected on the left (unit inflow per unit length), p = 0 on the right,
    # no flow on the bottom and top
    bc_kind=[FLUX, PRESSURE, NOFLOW, NOFLOW], bc_value=[-1.0, 0.0, 0.0, 0.0],
    s_inj=1.0, cfl=0.5, cn=1, breakthrough_cut=0.01,
)

CONFIGS = {
    # plain method, FP64: 32^2 cells, 4x4 subdomains of 8^2, 2 interface elements per side
    "c1": dict(_BASE, nx=32, ny=32, sub_x=8, sub_y=8, ne_x=2, ne_y=2, mu_o=10.0,
               sigma2=1.0, corr_len=0.1, seed=1, steps=50),
    # 256^2 cells, 16x16 subdomains of 16^2, 4 interface elements per side, high contrast
    "c2": dict(_BASE, nx=256, ny=256, sub_x=16, sub_y=16, ne_x=4, ne_y=4, mu_o=100.0,
               sigma2=4.0, corr_len=0.05, seed=2, steps=200),
    # 1024^2 cells, 64x64 subdomains of 16^2, 8 interface elements per side
    "c3": dict(_BASE, nx=1024, ny=1024, sub_x=16, sub_y=16, ne_x=8, ne_y=8, mu_o=100.0,
               sigma2=4.0, corr_len=0.05, seed=3, steps=200),
}


def config(name: str, **overrides) -> dict:
    """Return a deep copy of a named workload with optional overrides."""
    cfg = copy.deepcopy(CONFIGS[name])
    cfg.update(overrides)
    return cfg


def gaussian_field(nx: int, ny: int, lx: float, ly: float, corr_len: float, seed: int) -> np.ndarray:
    """Zero-mean unit-variance Gaussian field on cell centres, shape (ny, nx), float64."""
    px, py = 2 * nx, 2 * ny
    hx, hy = lx / nx, ly / ny
    ix = np.arange(px)
    iy = np.arange(py)
    dx = np.minimum(ix, px - ix) * hx
    dy = np.minimum(iy, py - iy) * hy
    r2 = dy[:, None] ** 2 + dx[None, :] ** 2
    c = np.exp(-r2 / (2.0 * corr_len * corr_len))
    lam = np.fft.fft2(c).real
    lam = np.maximum(lam, 0.0)
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((py, px)) + 1j * rng.standard_normal((py, px))
    f = np.fft.fft2(np.sqrt(lam / (px * py)) * z)
    return np.ascontiguousarray(f.real[:ny, :nx])


def self_similar_field(nx: int, ny: int, lx: float, ly: float, seed: int, beta: float = 0.5) -> np.ndarray:
    """Zero-mean Gaussian field with the self-similar covariance |x - y|^-beta (Section 5.1
    uses beta = 1/2), shape (ny, nx): spectral synthesis with power spectrum |k|^(beta - 2)
    (the 2-D Fourier transform of the covariance) on a periodic grid padded to twice the
    domain, the constant mode removed, driven by numpy's PCG64 with `seed`. The covariance is
    singular at zero distance, so the sample has no intrinsic scale: it is returned with unit
    range (max - min = 1) over the domain; callers scale it."""
    px, py = 2 * nx, 2 * ny
    kx = np.fft.fftfreq(px, d=lx / nx)
    ky = np.fft.fftfreq(py, d=ly / ny)
    k = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
    amp = np.zeros_like(k)
    amp[k > 0] = k[k > 0] ** ((beta - 2.0) / 2.0)
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((py, px)) + 1j * rng.standard_normal((py, px))
    f = np.fft.ifft2(amp * z).real[:ny, :nx]
    f = f - f.mean()
    return np.ascontiguousarray(f / (f.max() - f.min()))


def permeability(cfg: dict) -> np.ndarray:
    """Permeability of a workload, shape (ny, nx): log-normal K = exp(sqrt(sigma2) xi) with
    Gaussian covariance, or (field = "self_similar") K = k0 exp(delta xi) with xi the
    self-similar field scaled to the range ln(contrast) / delta, or (field = "homogeneous")
    K = k0."""
    if cfg.get("field") == "homogeneous":
        return np.full((cfg["ny"], cfg["nx"]), float(cfg["k0"]))
    if cfg.get("field") == "self_similar":
        xi = self_similar_field(cfg["nx"], cfg["ny"], cfg["lx"], cfg["ly"], cfg["seed"])
        return cfg["k0"] * np.exp(np.log(cfg["contrast"]) * xi)
    xi = gaussian_field(cfg["nx"], cfg["ny"], cfg["lx"], cfg["ly"], cfg["corr_len"], cfg["seed"])
    return np.exp(np.sqrt(cfg["sigma2"]) * xi)


def x1_config(contrast: float = 1e3, ne: int = 1, cn: int = 1, eta: float = 1e-2, seed: int = 11) -> dict:
    """The Gaussian-field experiment of Section 5.1: [0,1]^2 with 64^2 cells, 4x4 subdomains of
    16^2, p = 1 on the left and p = 0 on the right, no flow on the bottom and top, no sources,
    M = 40, alpha = 1, eta = 1e-2; K = 0.8 exp(delta xi) with the self-similar field xi and
    Kmax/Kmin = contrast (1e3 for delta = 2.5, 1e6 for delta = 4.5); ne interface elements per
    side (H-bar = H / ne); C_n transport sub-steps per elliptic step."""
    cfg = dict(_BASE, nx=64, ny=64, sub_x=16, sub_y=16, ne_x=ne, ne_y=ne, mu_o=40.0, eta=eta, cn=cn,
               field="self_similar", k0=0.8, contrast=contrast, seed=seed, steps=0)
    cfg["bc_kind"] = [PRESSURE, PRESSURE, NOFLOW, NOFLOW]
    cfg["bc_value"] = [1.0, 0.0, 0.0, 0.0]
    return cfg


def x4_config(eta: float = 1e-2, cn: int = 1, steps: int = 2000) -> dict:
    """Water-oil finger growth in a homogeneous medium (the last experiment of Section 5):
    [0,3] x [0,1/2] with 300 x 50 cells in 15 x 5 subdomains of 20 x 10, K = 1, M = 4, p = 0 on
    the left and -1e4 on the right, no flow on the bottom and top, no sources, water (s-bar =
    1) entering on the left; MRCM with H-bar = h (one fine face per interface element: 20 and
    10 elements per side) for the basis updates, eta = 1e-2, C_n = 1, T_e = 2000. The initial
    water-oil front with a small perturbation at the channel centre is a reading (the paper
    shows it only in a figure): s0 = 1 on the cells with centre x < 0.1, and x < 0.15 for
    |y - 1/4| < 0.05; s0 = 0 elsewhere."""
    cfg = dict(_BASE, lx=3.0, ly=0.5, nx=300, ny=50, sub_x=20, sub_y=10, ne_x=20, ne_y=10, mu_w=1.0, mu_o=4.0,
               eta=eta, cn=cn, field="homogeneous", k0=1.0, seed=0, steps=steps,
               s0="perturbed_front", front_x=0.1, bump_x=0.05, bump_half_width=0.05)
    cfg["bc_kind"] = [PRESSURE, PRESSURE, NOFLOW, NOFLOW]
    cfg["bc_value"] = [0.0, -1.0e4, 0.0, 0.0]
    return cfg


def initial_saturation(cfg: dict) -> np.ndarray:
    """Reservoir initially filled with oil (s0 = 0 everywhere), or (s0 = "perturbed_front") water
    on the cells whose centre lies left of front_x, and left of front_x + bump_x within
    bump_half_width of the channel's mid-line."""
    s = np.zeros((cfg["ny"], cfg["nx"]))
    if cfg.get("s0") == "perturbed_front":
        xc = (np.arange(cfg["nx"]) + 0.5) * cfg["lx"] / cfg["nx"]
        yc = (np.arange(cfg["ny"]) + 0.5) * cfg["ly"] / cfg["ny"]
        bump = np.abs(yc - 0.5 * cfg["ly"]) < cfg["bump_half_width"]
        reach = cfg["front_x"] + np.where(bump, cfg["bump_x"], 0.0)
        s[xc[None, :] < reach[:, None]] = 1.0
    return s


def source(cfg: dict) -> np.ndarray:
    """No wells: q = 0 everywhere."""
    return np.zeros((cfg["ny"], cfg["nx"]))


def random_problem(seed: int, nx: int, ny: int, sub_x: int, sub_y: int, ne_x: int, ne_y: int,
                   sigma2: float = 1.0, corr_len: float = 0.2, **overrides) -> tuple[dict, np.ndarray]:
    """A small seeded problem for parity and property tests: config dict and permeability."""
    cfg = dict(_BASE, nx=nx, ny=ny, sub_x=sub_x, sub_y=sub_y, ne_x=ne_x, ne_y=ne_y,
               sigma2=sigma2, corr_len=corr_len, seed=seed, steps=10)
    cfg["bc_kind"] = list(cfg["bc_kind"])
    cfg["bc_value"] = list(cfg["bc_value"])
    cfg.update(overrides)
    return cfg, permeability(cfg)


def batch_workload(n: int = 256) -> list[dict]:
    """Batched form: n realisations of uneven sizes, class r mod 3 -> 64^2 cells in 8^2
    subdomains, 128^2 in 16^2, 256^2 in 32^2; 4 interface elements per side, log-variance 4,
    correlation length 0.05, seed 1000 + r, viscosity ratio 100, eta = 0.1."""
    out = []
    for r in range(n):
        nx, sub = ((64, 8), (128, 16), (256, 32))[r % 3]
        cfg = dict(_BASE, nx=nx, ny=nx, sub_x=sub, sub_y=sub, ne_x=4, ne_y=4, mu_o=100.0, eta=0.1,
                   sigma2=4.0, corr_len=0.05, seed=1000 + r, steps=0)
        cfg["bc_kind"] = list(cfg["bc_kind"])
        cfg["bc_value"] = list(cfg["bc_value"])
        out.append(cfg)
    return out


def serve_requests(n: int = 256, grids=(128, 256, 512), seed: int = 7) -> list[dict]:
    """Serving form: n forward-run requests; grid drawn uniformly from `grids` (16^2
    subdomains, 4 interface elements per side), log-variance uniform in [1, 4], correlation
    length 0.05, viscosity ratio uniform in [10, 100], permeability seed 5000 + r. The draws
    use numpy's PCG64 with `seed`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for r in range(n):
        nx = int(grids[rng.integers(len(grids))])
        cfg = dict(_BASE, nx=nx, ny=nx, sub_x=16, sub_y=16, ne_x=4, ne_y=4,
                   mu_o=float(rng.uniform(10.0, 100.0)), eta=0.1, sigma2=float(rng.uniform(1.0, 4.0)),
                   corr_len=0.05, seed=5000 + r, steps=0)
        cfg["bc_kind"] = list(cfg["bc_kind"])
        cfg["bc_value"] = list(cfg["bc_value"])
        out.append(cfg)
    return out
